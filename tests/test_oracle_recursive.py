"""Pins of the recursive strip solve (oracle/recursive.py, Sec. 4 closing
discussion): special cases that reduce to the pinned double sweep, the
identity the inner transmission data rest on, linearity, the sub-block band
widths, and convergence of MPGMRES with the recursive preconditioners."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import assemble as asm
from oracle import mpgmres as mp
from oracle import recursive as rc
from oracle import strips as st
from oracle import sweep as sw

OMEGA, C, N_GRID = 18.0, [1.0, 1.7, 1.2], 33


def _rand(m, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(m) + 1j * g.standard_normal(m)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_one_sub_block_is_the_exact_strip_solve():
    A = asm.assemble(OMEGA, C, N_GRID)
    r = _rand(N_GRID ** 2, 1)
    for d in (st.X, st.Y):
        ref = sw.DoubleSweep(OMEGA, C, N_GRID, 4, d, A=A).apply(r)
        got = rc.RecursiveSweep(OMEGA, C, N_GRID, 4, d, 1, A=A).apply(r)
        assert _rel(got, ref) < 1e-12


def test_one_outer_strip_is_the_perpendicular_double_sweep():
    # N = 1: the strip is the whole square and A_s = A, so the inner sweep
    # over N2 sub-blocks along x-strips' length (y) is BTB with N2 strips
    A = asm.assemble(OMEGA, C, N_GRID)
    r = _rand(N_GRID ** 2, 2)
    for outer, inner in ((st.X, st.Y), (st.Y, st.X)):
        got = rc.RecursiveSweep(OMEGA, C, N_GRID, 1, outer, 4, A=A).apply(r)
        ref = sw.DoubleSweep(OMEGA, C, N_GRID, 4, inner, A=A).apply(r)
        assert _rel(got, ref) < 1e-12


def test_exact_strip_solution_satisfies_every_sub_block_problem():
    # u* = A_s^{-1} rho solves A_{s,t} R_t u* = R_t rho + g_{s,t}(u*) on every
    # sub-block: the transmission data carry exactly what the cut removes
    n, N, N2 = N_GRID, 4, 4
    for d in (st.X, st.Y):
        for s in (1, 2, 4):
            A_s = st.strip_matrix(OMEGA, C, n, N, d, s)
            inner = rc.InnerSweep(OMEGA, C, n, N, d, s, N2, A_s)
            rho = _rand(A_s.shape[0], 3 + s)
            u = spla.spsolve(A_s.tocsc(), rho)
            for t in range(N2):
                ix = inner.idx[t]
                g = inner.transmission(t, 1, u) + inner.transmission(t, 2, u)
                lhs = inner.Ast[t] @ u[ix]
                assert _rel(lhs, rho[ix] + g) < 1e-12


def test_recursive_sweep_is_linear():
    A = asm.assemble(OMEGA, C, N_GRID)
    M = rc.RecursiveSweep(OMEGA, C, N_GRID, 4, st.X, 4, A=A)
    a, b = _rand(N_GRID ** 2, 4), _rand(N_GRID ** 2, 5)
    lhs = M.apply(2.0 * a - 3j * b)
    rhs = 2.0 * M.apply(a) - 3j * M.apply(b)
    assert _rel(lhs, rhs) < 1e-12


def test_sub_blocks_take_the_narrow_ordering():
    # a strip 34 node lines wide (n = 65, N = 2, band half-width 35) cut into
    # 8 sub-blocks of length 10 or 11 is ordered along the strip: half-widths
    # 11 and 12
    n = 65
    A_s = st.strip_matrix(OMEGA, C, n, 2, st.X, 1)
    inner = rc.InnerSweep(OMEGA, C, n, 2, st.X, 1, 8, A_s)
    assert st.band_width(n, 2, 1) == 35
    assert inner.band_widths() == [11] + [12] * 6 + [11]  # lengths 10 and 11
    # narrow strips keep the across-strip ordering
    A_s = st.strip_matrix(OMEGA, C, N_GRID, 8, st.Y, 3)
    inner = rc.InnerSweep(OMEGA, C, N_GRID, 8, st.Y, 3, 2, A_s)
    assert inner.band_widths() == [st.band_width(N_GRID, 8, 3)] * 2


def test_mpgmres_with_recursive_sweeps_reaches_the_direct_solution():
    A = asm.assemble(OMEGA, C, N_GRID)
    b = _rand(N_GRID ** 2, 6)
    x_ref = spla.spsolve(A.tocsc(), b)
    exact = [sw.DoubleSweep(OMEGA, C, N_GRID, 4, d, A=A).apply for d in (st.X, st.Y)]
    rec = [rc.RecursiveSweep(OMEGA, C, N_GRID, 4, d, 4, A=A).apply for d in (st.X, st.Y)]
    r0 = mp.mpgmres(A, exact, b, tol=1e-10, maxit=100)
    r1 = mp.mpgmres(A, rec, b, tol=1e-10, maxit=100)
    assert r0.converged and r1.converged
    assert _rel(r1.x, x_ref) < 1e-8
    # an inexact strip solve can only weaken the preconditioner here
    assert r1.iterations >= r0.iterations
