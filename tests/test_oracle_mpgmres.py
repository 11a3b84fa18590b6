"""Pins of the oracle's selective MPGMRES (Sec. 3) and selection rule (Sec. 4)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import assemble as asm
from oracle import direct as dr
from oracle import mpgmres as mp
from oracle import strips as st
from oracle import sweep as sw


def _problem(n=25, N=4, omega=15.0, c=(1.0, 2.0, 1.5)):
    A = asm.assemble(omega, list(c), n)
    rng = np.random.default_rng(0)
    b = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    SX = sw.DoubleSweep(omega, list(c), n, N, st.X, A=A)
    SY = sw.DoubleSweep(omega, list(c), n, N, st.Y, A=A)
    return A, b, SX, SY


def test_one_preconditioner_is_right_preconditioned_gmres():
    # Sec. 3: MPGMRES with a single preconditioner reduces to standard GMRES
    A, b, SX, _ = _problem()
    res = mp.mpgmres(A, [SX.apply], b, tol=1e-10, maxit=60)
    x, its, hist = mp.gmres_right(A, SX.apply, b, tol=1e-10, maxit=60)
    assert res.iterations == its
    assert np.allclose(res.res_hist, hist, rtol=1e-6, atol=1e-13)
    assert np.linalg.norm(res.x - x) < 1e-8 * np.linalg.norm(x)


def test_residual_is_monotone_and_minimal():
    A, b, SX, SY = _problem(n=17, N=2)
    res = mp.mpgmres(A, [SX.apply, SY.apply], b, tol=1e-12, maxit=6)
    h = np.array(res.res_hist)
    assert np.all(h[1:] <= h[:-1] * (1 + 1e-14))
    # brute force: the same search space built independently, dense least squares
    beta = np.linalg.norm(b)
    t = 2
    Z = []
    inputs = [b / beta] * t
    V = np.zeros((b.size, 0), dtype=complex)
    V = np.concatenate([V, (b / beta)[:, None]], axis=1)
    for k in range(res.iterations):
        Zk = [SX.apply(inputs[0]), SY.apply(inputs[1])]
        Z.extend(Zk)
        Zm = np.stack(Z, axis=1)
        y = np.linalg.lstsq(A @ Zm, b, rcond=None)[0]
        best = np.linalg.norm(b - A @ (Zm @ y)) / beta
        assert best == pytest.approx(res.res_hist[k], rel=1e-7, abs=1e-14)
        # next inputs from an orthonormal basis of [b, A Z]: the new directions
        # of A z_1 and A z_2 (Gram-Schmidt in that order), crossed over
        W = A @ np.stack(Zk, axis=1)
        q = []
        for c in range(t):
            w = W[:, c] - V @ (V.conj().T @ W[:, c])
            w = w - V @ (V.conj().T @ w)
            for qq in q:
                w = w - np.vdot(qq, w) * qq
            q.append(w / np.linalg.norm(w))
        V = np.concatenate([V, np.stack(q, axis=1)], axis=1)
        inputs = [q[1], q[0]]


def test_cross_selection_feeds_the_other_preconditioners_vector():
    A, b, SX, SY = _problem(n=17, N=2)
    seen = {0: [], 1: []}

    def rec(i, S):
        def f(v):
            seen[i].append(v.copy())
            return S.apply(v)
        return f

    mp.mpgmres(A, [rec(0, SX), rec(1, SY)], b, tol=1e-12, maxit=3)
    beta = np.linalg.norm(b)
    v1 = b / beta
    assert np.allclose(seen[0][0], v1) and np.allclose(seen[1][0], v1)
    # iteration 2: M_1 gets the basis vector from A M_2^{-1} v1, M_2 the one from A M_1^{-1} v1
    w1 = A @ SX.apply(v1)
    w2 = A @ SY.apply(v1)
    q1 = w1 - v1 * np.vdot(v1, w1)
    q1 /= np.linalg.norm(q1)
    q2 = w2 - v1 * np.vdot(v1, w2) - q1 * np.vdot(q1, w2)
    q2 /= np.linalg.norm(q2)
    assert np.linalg.norm(seen[0][1] - q2) < 1e-8
    assert np.linalg.norm(seen[1][1] - q1) < 1e-8


def test_sum_selection_for_more_than_two():
    A, b, SX, SY = _problem(n=17, N=2)
    seen = []

    def rec(S):
        def f(v):
            seen.append(v.copy())
            return S.apply(v)
        return f

    mp.mpgmres(A, [rec(SX), rec(SY), rec(SX)], b, tol=1e-12, maxit=2)
    # iteration 2: all three preconditioners see the same (summed) vector
    assert np.allclose(seen[3], seen[4]) and np.allclose(seen[4], seen[5])


@pytest.mark.parametrize("t", [1, 2, 3, 4])
def test_inner_product_count_single_pass_matches_paper(t):
    # Sec. 3: iteration k needs (k - 1/2) t^2 + (3/2) t inner products
    n, omega, c = 17, 15.0, [1.0, 2.0, 1.5]
    A = asm.assemble(omega, c, n)
    b = np.random.default_rng(0).standard_normal(n * n) + 0j
    precs = [sw.DoubleSweep(omega, c, n, N, d, A=A).apply
             for N, d in ((2, st.X), (2, st.Y), (4, st.X), (4, st.Y))][:t]
    res = mp.mpgmres(A, precs, b, tol=1e-14, maxit=4, cgs_passes=1, block_passes=1)
    checked = 0
    for k, (ip, kept) in enumerate(zip(res.ip_per_iter, res.kept_per_iter), start=1):
        if kept == t:                       # the count assumes no deflation
            assert ip == mp.inner_products_paper(k, t)
            checked += 1
    assert checked >= 3


def test_inner_product_count_two_pass():
    A, b, SX, SY = _problem(n=17, N=2)
    t = 2
    res = mp.mpgmres(A, [SX.apply, SY.apply], b, tol=1e-14, maxit=4)
    for k, ip in enumerate(res.ip_per_iter, start=1):
        assert ip == 2 * (1 + (k - 1) * t) * t + t * t


def test_single_strip_two_directions_converges_in_one_iteration():
    # N = 1 makes each sweep an exact solve: one iteration, second column deflated
    n, omega, c = 15, 10.0, [1.0, 1.8]
    A = asm.assemble(omega, c, n)
    SX = sw.DoubleSweep(omega, c, n, 1, st.X, A=A)
    SY = sw.DoubleSweep(omega, c, n, 1, st.Y, A=A)
    b = np.random.default_rng(1).standard_normal(n * n) + 0j
    res = mp.mpgmres(A, [SX.apply, SY.apply], b, tol=1e-10)
    assert res.iterations == 1 and res.converged
    assert res.true_res < 1e-12


def test_zero_rhs():
    A, _, SX, SY = _problem(n=9, N=2)
    res = mp.mpgmres(A, [SX.apply, SY.apply], np.zeros(81, dtype=complex))
    assert res.iterations == 0 and np.all(res.x == 0)


def test_converged_solution_close_to_direct():
    A, b, SX, SY = _problem(n=33, N=4)
    res = mp.mpgmres(A, [SX.apply, SY.apply], b, tol=1e-10)
    xd = dr.direct_solve(A, b)
    assert res.converged and res.true_res < 1e-10
    assert np.linalg.norm(res.x - xd) < 1e-7 * np.linalg.norm(xd)


def test_direct_band_and_sparse_agree():
    n = 41
    A = asm.assemble(25.0, [1.0, 2.0], n)
    b = np.random.default_rng(2).standard_normal(n * n) + 0j
    x1 = dr.direct_solve(A, b, method="band")
    x2 = dr.direct_solve(A, b, method="splu")
    x3 = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x1 - x3) < 1e-10 * np.linalg.norm(x3)
    assert np.linalg.norm(x2 - x3) < 1e-10 * np.linalg.norm(x3)


@pytest.mark.parametrize("names", [("LR", "RL"), ("LR", "BT", "RL", "TB")])
def test_single_sweep_combinations_reach_the_direct_solution(names):
    # Table 1's single-sweep combinations: the cross rule for t = 2 (LR+RL) and
    # the sum rule for t = 4 (LR+BT+RL+TB), run to a tight tolerance.
    n, N, omega, c = 33, 4, 16.0, [1.0, 2.0, 1.5]
    A = asm.assemble(omega, c, n)
    rng = np.random.default_rng(12)
    f = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    b = asm.source_load(n, f)
    precs = [sw.preconditioner(omega, c, n, N, nm, A=A).apply for nm in names]
    res = mp.mpgmres(A, precs, b, tol=1e-10, maxit=100)
    assert res.converged
    hist = np.asarray(res.res_hist)
    assert np.all(hist[1:] <= hist[:-1] * (1 + 1e-14))
    xd = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(res.x - xd) < 1e-7 * np.linalg.norm(xd)
