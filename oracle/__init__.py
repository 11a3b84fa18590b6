"""Reference oracle for the multipreconditioned sweeping Helmholtz solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
product path (``paper_2408_11929_amd``) never imports, links or calls it;
the two share no code except the seeded input generators in ``workloads``,
which hold none of the method's arithmetic.

Everything here is plain, slow and FP64 (complex128) unless a function says
otherwise.  Each function cites the passage of Bootland & Rees,
"Multipreconditioning with directional sweeping methods for high-frequency
Helmholtz problems" (arXiv 2408.11929) that it follows.

Modules
-------
assemble  P1 discretisation of the impedance Helmholtz problem, eq. (1).
strips    Sequential overlapping strip decomposition (Sec. 2, Fig. 1,
          Sec. 4 setup) and the strip matrices with Robin rows, eq. (4).
sweep     Discrete Robin transmission data and the double sweep of
          eqs. (2)-(3), with LAPACK band LU for the strip solves.
mpgmres   Selective multipreconditioned GMRES (Sec. 3) with the selection
          rule of Sec. 4, plus an independent textbook right-preconditioned
          GMRES used to pin the t = 1 case.
direct    Full direct solve of the global system (LAPACK band LU or SuperLU).
recursive Double sweeps whose strip solves are inner double sweeps over
          sub-blocks along the strip (Sec. 4, closing discussion).

Parity status: every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` against closed forms, invariants, special cases
that reduce to library routines, or brute force.  End-to-end iteration counts
against the paper's Tables 1-5 are parity unpinned (the paper uses 5-point
finite differences and a third-party MPGMRES code; this oracle uses P1).
"""
