"""Double sweeps whose strip problems are themselves solved by a sweep in the
perpendicular direction (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 4, closing discussion: the strip subproblems may be decomposed again,
recursively in the perpendicular direction, and solved approximately instead
of by a direct solver.  One level of that recursion:

* The outer sweep is the double sweep of ``sweep.DoubleSweep`` (eqs. (2)-(4)):
  the same strips, order, transmission data g_s(z) = A_s R_s z - R_s A z and
  "most recent solve wins" rule.
* Each strip solve A_s u = rho is replaced by one double sweep on the strip's
  own rectangle: the strip is cut along its length into N2 sub-blocks with the
  rule of the outer strips (reading c6: m2 = (n-1)/N2 intervals, one extra
  mesh line past each internal boundary, overlap 2h).  A sub-block's matrix
  A_{s,t} is the operator of its rectangle with the impedance condition on
  all four sides (the strip's own sides keep theirs, the new internal
  boundaries get the transmission operator of eq. (4), which has the same
  form), and its transmission data come from the strip problem:
      g_{s,t}(u) = A_{s,t} R_t u - R_t A_s u   on its interface rows.
  Forward over t = 1..N2, backward over t = N2-1..1 with the forward pass's
  Gamma_{t,1} data (reading c8), the most recent sub-block solve winning.
* The result is a fixed linear operator (no inner iteration), an inexact
  strip solve: with N2 = 1 it is the exact strip solve.

Sub-block ordering: by the smaller of its two dimensions, so the band
half-width is min(w, len) + 1 (w: the strip's width in node lines, len: the
sub-block's length along the strip); wide strips thus get narrow sub-blocks.
"""
import numpy as np

from . import assemble as asm
from . import strips as st
from .sweep import DoubleSweep, StripSolver


class InnerSweep:
    """Approximate solve of one strip problem A_s u = rho by a double sweep
    over N2 sub-blocks along the strip (strip-local vectors, q = long*w + short)."""

    def __init__(self, omega, c_layers, n, N, direction, s, N2, A_s, dtype=np.complex128,
                 scheme="p1"):
        st.check_decomposition(n, N2)
        a, b = st.strip_lines(n, N, s)
        self.w = w = b - a + 1
        self.N2 = N2
        self.A_s = A_s.astype(dtype)
        self.dtype = dtype
        self.idx, self.solvers, self.Ast, self.rows1, self.rows2 = [], [], [], [], []
        for t in range(1, N2 + 1):
            c, d = st.strip_lines(n, N2, t)
            ln = d - c + 1
            # strip-local indices of the sub-block, in the sub-block's order
            L = np.arange(c, d + 1)
            T = np.arange(w)
            if w <= ln:          # across the strip fastest: q' = (l - c) w + t
                local = (L[:, None] * w + T[None, :]).ravel()
                kl = w + 1
                r1 = np.arange(w)
                r2 = (ln - 1) * w + np.arange(w)
            else:                # along the strip fastest: q' = t len + (l - c)
                local = (T[:, None] + L[None, :] * w).ravel()
                kl = ln + 1
                r1 = np.arange(w) * ln
                r2 = np.arange(w) * ln + (ln - 1)
            if direction == st.X:
                win = (a, b, c, d)
            else:
                win = (c, d, a, b)
            A_win = asm.assemble(omega, c_layers, n, window=win, scheme=scheme)
            strip_ids = st.strip_nodes(n, N, direction, s)
            A_t = A_win[strip_ids[local]][:, strip_ids[local]].tocsr()
            self.idx.append(local)
            self.Ast.append(A_t.astype(dtype))
            self.solvers.append(StripSolver(A_t, kl, dtype))
            self.rows1.append(r1 if t > 1 else np.zeros(0, dtype=np.int64))
            self.rows2.append(r2 if t < N2 else np.zeros(0, dtype=np.int64))

    def band_widths(self):
        return [sv.kl for sv in self.solvers]

    def transmission(self, t, side, u):
        """g_{s,t}(u) = A_{s,t} R_t u - R_t A_s u on the interface rows (0-based t)."""
        idx = self.idx[t]
        rows = self.rows1[t] if side == 1 else self.rows2[t]
        full = self.Ast[t] @ u[idx] - (self.A_s @ u)[idx]
        g = np.zeros(len(idx), dtype=self.dtype)
        g[rows] = full[rows]
        return g

    def solve(self, rho):
        N2 = self.N2
        rho = np.asarray(rho).astype(self.dtype)
        u = np.zeros(len(rho), dtype=self.dtype)
        g1 = [None] * N2
        for t in range(N2):
            g1[t] = self.transmission(t, 1, u)
            u[self.idx[t]] = self.solvers[t].solve(rho[self.idx[t]] + g1[t])
        for t in range(N2 - 2, -1, -1):
            rhs = rho[self.idx[t]] + g1[t] + self.transmission(t, 2, u)
            u[self.idx[t]] = self.solvers[t].solve(rhs)
        return u


class RecursiveSweep(DoubleSweep):
    """M^{-1} of the double sweep in `direction` whose 2N - 1 strip solves are
    each one inner double sweep over N2 sub-blocks (see the module docstring)."""

    def __init__(self, omega, c_layers, n, N, direction, N2, A=None, precision="fp64",
                 scheme="p1"):
        super().__init__(omega, c_layers, n, N, direction, A=A, precision=precision,
                         scheme=scheme)
        self.N2 = N2
        self.inner = [InnerSweep(omega, c_layers, n, N, direction, s, N2, self.As[s - 1],
                                 self.dtype, scheme=scheme)
                      for s in range(1, N + 1)]
        # the outer apply calls solvers[s].solve: route it through the inner sweeps
        self.solvers = [sweep for sweep in self.inner]

    def factor_elements(self):
        """Complex entries of band storage (3 kl + 1 per row) of all sub-blocks."""
        return sum((3 * kl + 1) * len(ix) for sw in self.inner
                   for kl, ix in zip(sw.band_widths(), sw.idx))
