"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances: FP64 kernels agree with the oracle to 1e-12 relative, in the
2-norm and element-wise (assembly and SpMV to 1e-13: they differ only in
summation order); complex64 strips agree with the FP64 oracle to 1e-5
relative, 2-norm and element-wise, wherever the oracle's own complex64
emulation meets 1e-5, and are otherwise reported as a miss and held to three
times the emulation's error (see _parity.py; every complex64 case prints its
numbers); MPGMRES runs are compared by iteration count (exact), solution
(relative 1e-8 for FP64, both runs converged to a tighter tolerance) and the
FP64-recomputed residual.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import assemble as oasm
from oracle import direct as odr
from oracle import mpgmres as omp
from oracle import strips as ost
from oracle import sweep as osw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

hh = pytest.importorskip("paper_2408_11929_amd")

from _parity import check_fp32, check_fp64, relmax  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


CASES = [
    # (n, N, omega, c)  -- several tiles, ragged widths, layered media
    (33, 4, 18.0, [1.0, 2.0, 1.5]),
    (41, 5, 25.0, [1.0]),
    (64, 9, 30.0, [2.2, 1.1, 1.7, 2.9, 1.3]),
]
# wide strips: band half-widths 35 and 51 take the 16- and 20-term blocked maps
WIDE = [
    (65, 2, 40.0, [1.0, 1.6]),
    (97, 2, 50.0, [1.3, 0.9, 2.0]),
]
# narrow strips (two intervals each: band half-widths 5-6) and strips shorter
# than one staged chunk of LU column steps
NARROW = [
    (33, 16, 18.0, [1.0, 2.0]),
    (9, 4, 6.0, [1.0]),
]
# under-resolved meshes whose strip factorisations pivot: every strip of the
# first, only the x strips of the second (the y strips take the blocked path)
PIVOTING = [
    (33, 4, 100.0, [1.0]),
    (33, 2, 80.0, [1.0, 0.5]),
]


def _upper_diagonals(A, n):
    nn = n * n
    out = np.zeros((4, nn), dtype=np.complex128)
    Ad = A.todok() if hasattr(A, "todok") else A
    coo = A.tocoo()
    for r, c, v in zip(coo.row, coo.col, coo.data):
        d = c - r
        k = {0: 0, 1: 1, n: 2, n + 1: 3}.get(d)
        if k is not None:
            out[k, r] += v
    del Ad
    return out


@pytest.mark.parametrize("n,N,omega,c", CASES)
def test_assembly_matches_oracle(n, N, omega, c):
    pb = hh.Problem(omega, c, n)
    got = pb.get_operator()
    A = oasm.assemble(omega, c, n)
    ref = _upper_diagonals(A, n)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    # the lower triangle is the transpose (complex symmetric)
    assert abs(A - A.T).max() == 0
    pb.free()


@pytest.mark.parametrize("n,N,omega,c", CASES[:2])
def test_load_vector_and_spmv(n, N, omega, c):
    pb = hh.Problem(omega, c, n)
    f = np.stack([wl.gaussian_field(n, 0.3, 0.7, 0.05), rand(n * n, 1)])
    b = host(pb.load_vector(dev(f)))
    for v in range(2):
        assert rel(b[v], oasm.source_load(n, f[v])) < 1e-13
    x = rand((3, n * n), 2)
    y = host(pb.spmv(dev(x)))
    A = oasm.assemble(omega, c, n)
    for v in range(3):
        assert rel(y[v], A @ x[v]) < 1e-13
    pb.free()


@pytest.mark.parametrize("lu", ["", "1"])
@pytest.mark.parametrize("prec", [hh.HH_FP64, hh.HH_FP32])
@pytest.mark.parametrize("n,N,omega,c", CASES + WIDE + NARROW + PIVOTING)
def test_strip_solves_match_lapack(n, N, omega, c, prec, lu, monkeypatch):
    # lu "": strips of band half-width < 32 are factored by the kernel that
    # assumes no interchange, those that need one (PIVOTING) packed again and
    # factored with interchanges; "1" (HH_LU_INTERCHANGE): every strip by the
    # interchanging kernel
    if lu:
        monkeypatch.setenv("HH_LU_INTERCHANGE", lu)
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, prec)
    for d, dname in ((hh.HH_DIR_X, ost.X), (hh.HH_DIR_Y, ost.Y)):
        for s in range(1, N + 1):
            a, w, kl = pb.strip_info(d, s)
            a_ref, b_ref = ost.strip_lines(n, N, s)
            assert (a, w, kl) == (a_ref, b_ref - a_ref + 1, ost.band_width(n, N, s))
            As = ost.strip_matrix(omega, c, n, N, dname, s)
            rhs = rand(As.shape[0], 10 * s + d)
            x = host(pb.strip_solve(d, s, dev(rhs)))
            ref = osw.StripSolver(As, kl)
            xr = ref.solve(rhs)
            if prec == hh.HH_FP32:
                x32 = osw.StripSolver(As, kl, np.complex64).solve(rhs)
                check_fp32(x, xr, x32, f"strip solve n={n} N={N} {dname}{s} lu={lu or 'auto'}",
                           cond=ref.cond1())
            else:
                check_fp64(x, xr, f"strip solve n={n} N={N} {dname}{s}")
    pb.free()


@pytest.mark.parametrize("plan", ["0", "1", "2", "3"])
@pytest.mark.parametrize("prec", [hh.HH_FP64, hh.HH_FP32])
@pytest.mark.parametrize("n,N,omega,c", CASES + WIDE + NARROW + PIVOTING)
def test_sweeps_match_oracle(n, N, omega, c, prec, plan, monkeypatch):
    # plan 0: one workgroup per chain; plan 1: sixteen, plan 2: two (complex64
    # strips that did not pivot, where the workgroups fit; else plan 0 again);
    # 3: plan 0 with both vectors in one tile
    monkeypatch.setenv("HH_SWEEP_PLAN", plan)
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, prec)
    A = oasm.assemble(omega, c, n)
    r = rand((2, n * n), 5)
    for d, dname in ((hh.HH_DIR_X, ost.X), (hh.HH_DIR_Y, ost.Y)):
        z = host(pb.sweep_apply(d, dev(r)))
        S = osw.DoubleSweep(omega, c, n, N, dname, A=A)
        S32 = osw.DoubleSweep(omega, c, n, N, dname, A=A, precision="fp32") if prec == hh.HH_FP32 else None
        cond = max(sv.cond1() for sv in S.solvers) if S32 is not None else None
        for v in range(2):
            zr = S.apply(r[v])
            if S32 is None:
                check_fp64(z[v], zr, f"sweep n={n} N={N} {dname}")
            else:
                check_fp32(z[v], zr, S32.apply(r[v]), f"sweep n={n} N={N} {dname} v{v} plan={plan}",
                           cond=cond)
    pb.free()


@pytest.mark.parametrize("nvec", [2, 3, 5])
@pytest.mark.parametrize("n,N,omega,c", CASES + WIDE[:1] + NARROW[:1])
def test_tiles_are_bitwise_plan0(n, N, omega, c, nvec, monkeypatch):
    # tiles of two right-hand sides (a last single vector repeated) give
    # exactly the one-workgroup plan's results, vector by vector
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP32)
    r = dev(rand((nvec, n * n), 30 + nvec))
    out = {}
    for plan in ("0", "3"):
        monkeypatch.setenv("HH_SWEEP_PLAN", plan)
        out[plan] = [host(pb.precond_apply(k, r)) for k in ("LRL", "BTB", "RL")]
    for a, b in zip(out["0"], out["3"]):
        assert np.array_equal(a, b), np.abs(a - b).max()
    pb.free()


def test_mpgmres_with_tiles_is_bitwise_plan0(monkeypatch):
    n, N, omega, c = 64, 9, 30.0, [2.2, 1.1, 1.7, 2.9, 1.3]
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP32)
    pos = wl.source_positions(21, 5)
    b = pb.load_vector(dev(np.stack([wl.gaussian_field(n, x0, y0, 0.03) for x0, y0 in pos])))
    res = {}
    for plan in ("0", "3"):
        monkeypatch.setenv("HH_SWEEP_PLAN", plan)
        x, st, rc = pb.mpgmres(b, tol=1e-8, maxit=100)
        assert rc == hh.HH_OK
        res[plan] = (host(x), [s["iterations"] for s in st])
    assert res["0"][1] == res["3"][1]
    assert np.array_equal(res["0"][0], res["3"][0])
    pb.free()


SINGLE = [("LR", ost.X, "forward"), ("RL", ost.X, "reverse"),
          ("BT", ost.Y, "forward"), ("TB", ost.Y, "reverse")]


@pytest.mark.parametrize("plan", ["0", "1", "2"])
@pytest.mark.parametrize("prec", [hh.HH_FP64, hh.HH_FP32])
@pytest.mark.parametrize("n,N,omega,c", CASES + NARROW[:1] + PIVOTING[:1])
def test_single_sweeps_match_oracle(n, N, omega, c, prec, plan, monkeypatch):
    # LR, RL, BT, TB of Sec. 4 (Table 1) on both plans and precisions
    monkeypatch.setenv("HH_SWEEP_PLAN", plan)
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, prec)
    A = oasm.assemble(omega, c, n)
    r = rand((2, n * n), 15)
    for name, dname, order in SINGLE:
        z = host(pb.precond_apply(name, dev(r)))
        S = osw.SingleSweep(omega, c, n, N, dname, order=order, A=A)
        S32 = (osw.SingleSweep(omega, c, n, N, dname, order=order, A=A, precision="fp32")
               if prec == hh.HH_FP32 else None)
        for v in range(2):
            zr = S.apply(r[v])
            if S32 is None:
                check_fp64(z[v], zr, f"{name} n={n} N={N}")
            else:
                check_fp32(z[v], zr, S32.apply(r[v]), f"{name} n={n} N={N} v{v} plan={plan}")
    # the double-sweep kinds are hh_sweep_apply
    zd = host(pb.precond_apply(hh.HH_PRE_BTB, dev(r)))
    assert np.array_equal(zd, host(pb.sweep_apply(hh.HH_DIR_Y, dev(r))))
    pb.free()


@pytest.mark.parametrize("names", [("LR", "RL"), ("LR", "BT", "RL", "TB"), ("RL",),
                                   ("LRL", "BTB", "LR")])
def test_mpgmres_single_sweep_combinations_match_oracle(names):
    # Table 1's combinations: cross rule (t = 2), sum rule (t > 2), t = 1
    n, N, omega, c = 41, 5, 25.0, [1.0, 1.7]
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64)
    pb.set_preconditioners(list(names))
    b = oasm.source_load(n, wl.gaussian_field(n, 0.4, 0.6, 0.05))
    x, st, rc = pb.mpgmres(dev(b.reshape(1, -1)), tol=1e-10, maxit=150)
    A = oasm.assemble(omega, c, n)
    precs = [osw.preconditioner(omega, c, n, N, nm, A=A).apply for nm in names]
    ref = omp.mpgmres(A, precs, b, tol=1e-10, maxit=150)
    print(f"[mpgmres] {'+'.join(names)}: {st[0]['iterations']} iterations (oracle "
          f"{ref.iterations}), res_true {st[0]['res_true']:.2e}", flush=True)
    assert rc == hh.HH_OK and st[0]["converged"] == 1
    assert st[0]["iterations"] == ref.iterations
    assert rel(host(x)[0], ref.x) < 1e-8
    assert st[0]["res_true"] < 1e-10
    pb.free()


def test_set_preconditioners_rejects_unfactored_direction():
    pb = hh.Problem(10.0, [1.0], 33)
    pb.factor_sweeps(hh.HH_DIR_X, 4, hh.HH_FP64)
    with pytest.raises(hh.HHError):
        pb.set_preconditioners(["LR", "BT"])       # y was not factored
    with pytest.raises(hh.HHError):
        pb.set_preconditioners(["LR"] * 5)         # t > 4
    with pytest.raises(hh.HHError):
        pb.set_preconditioners([7])                # unknown kind
    pb.set_preconditioners(["LR", "RL"])
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, 4, hh.HH_FP64)  # resets to LRL+BTB
    b = dev(rand((1, 33 * 33), 3))
    x, st, rc = pb.mpgmres(b, tol=1e-8, maxit=60)
    assert rc == hh.HH_OK
    pb.free()


def test_wide_sweep_gives_up_when_partners_are_late(monkeypatch):
    # a zero wait bound makes the first workgroup to arrive at a meeting give
    # up: the call reports the error instead of waiting, and the next call
    # with the normal bound is correct again
    n, N, omega, c = 64, 9, 30.0, [2.2, 1.1, 1.7, 2.9, 1.3]
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP32)
    r = rand((1, n * n), 6)
    monkeypatch.setenv("HH_SWEEP_PLAN", "1")
    monkeypatch.setenv("HH_SWEEP_WAIT_US", "0")
    with pytest.raises(hh.HHError, match="did not meet"):
        pb.sweep_apply(hh.HH_DIR_X, dev(r))
    monkeypatch.delenv("HH_SWEEP_WAIT_US")
    z = host(pb.sweep_apply(hh.HH_DIR_X, dev(r)))[0]
    A = oasm.assemble(omega, c, n)
    zr = osw.DoubleSweep(omega, c, n, N, ost.X, A=A).apply(r[0])
    z32 = osw.DoubleSweep(omega, c, n, N, ost.X, A=A, precision="fp32").apply(r[0])
    check_fp32(z, zr, z32, f"sweep after abort n={n} N={N} x")
    pb.free()


def test_sweep_single_strip_is_exact_solve():
    n, omega, c = 31, 12.0, [1.0, 2.0]
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, 1, hh.HH_FP64)
    A = oasm.assemble(omega, c, n)
    r = rand(n * n, 3)
    for d in (hh.HH_DIR_X, hh.HH_DIR_Y):
        z = host(pb.sweep_apply(d, dev(r.reshape(1, -1))))[0]
        assert rel(A @ z, r) < 1e-12
    pb.free()


def _oracle_solve(n, N, omega, c, b, tol, t=2):
    A = oasm.assemble(omega, c, n)
    precs = [osw.DoubleSweep(omega, c, n, N, ost.X, A=A).apply]
    if t == 2:
        precs.append(osw.DoubleSweep(omega, c, n, N, ost.Y, A=A).apply)
    return A, omp.mpgmres(A, precs, b, tol=tol)


@pytest.mark.parametrize("n,N,omega,c", CASES)
def test_mpgmres_fp64_matches_oracle(n, N, omega, c):
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64)
    f = wl.gaussian_field(n, 0.45, 0.55, 0.05)
    b = oasm.source_load(n, f)
    x, st, rc = pb.mpgmres(dev(b.reshape(1, -1)), tol=1e-10, maxit=100)
    A, ref = _oracle_solve(n, N, omega, c, b, 1e-10)
    assert rc == hh.HH_OK and st[0]["converged"] == 1
    assert st[0]["iterations"] == ref.iterations
    assert rel(host(x)[0], ref.x) < 1e-8
    assert st[0]["res_true"] < 1e-10
    assert abs(st[0]["res_est"] - ref.res_hist[-1]) < 1e-3 * ref.res_hist[-1] + 1e-14
    pb.free()


def test_mpgmres_one_direction_is_gmres():
    n, N, omega, c = 33, 4, 18.0, [1.0, 2.0, 1.5]
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X, N, hh.HH_FP64)
    b = oasm.source_load(n, wl.gaussian_field(n, 0.5, 0.5, 0.05))
    x, st, rc = pb.mpgmres(dev(b.reshape(1, -1)), tol=1e-9, maxit=100)
    A = oasm.assemble(omega, c, n)
    SX = osw.DoubleSweep(omega, c, n, N, ost.X, A=A)
    xr, its, _ = omp.gmres_right(A, SX.apply, b, tol=1e-9, maxit=100)
    assert st[0]["iterations"] == its
    assert rel(host(x)[0], xr) < 1e-7
    pb.free()


def test_mpgmres_single_strip_converges_in_one_iteration():
    n, omega, c = 31, 12.0, [1.0, 2.0]
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, 1, hh.HH_FP64)
    b = rand(n * n, 8)
    x, st, rc = pb.mpgmres(dev(b.reshape(1, -1)), tol=1e-10, maxit=10)
    assert rc == hh.HH_OK and st[0]["iterations"] == 1
    assert st[0]["res_true"] < 1e-11
    assert st[0]["deflated"] >= 1
    pb.free()


def test_batched_rhs_equal_to_single():
    n, N, omega, c = 41, 5, 25.0, [1.0, 1.7]
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP32)
    pos = wl.source_positions(11, 4)
    f = np.stack([wl.gaussian_field(n, x0, y0, 0.03) for x0, y0 in pos])
    b = pb.load_vector(dev(f))
    xb, stb, _ = pb.mpgmres(b, tol=1e-8, maxit=100)
    for v in range(4):
        xs, sts, _ = pb.mpgmres(b[v:v + 1].contiguous(), tol=1e-8, maxit=100)
        assert sts[0]["iterations"] == stb[v]["iterations"]
        assert rel(host(xs)[0], host(xb)[v]) <= 1e-14
    pb.free()


def test_zero_rhs_and_maxit():
    n, N, omega, c = 33, 4, 18.0, [1.0]
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64)
    z = torch.zeros((1, n * n), dtype=torch.complex128, device="cuda")
    x, st, rc = pb.mpgmres(z, tol=1e-6, maxit=5)
    assert rc == hh.HH_OK and st[0]["iterations"] == 0 and torch.all(x == 0)
    b = dev(rand((1, n * n), 4))
    x, st, rc = pb.mpgmres(b, tol=1e-14, maxit=1)
    assert rc == hh.HH_ENOCONV and st[0]["iterations"] == 1 and st[0]["converged"] == 0
    pb.free()


def test_invalid_factorisation_arguments():
    pb = hh.Problem(10.0, [1.0], 33)
    with pytest.raises(hh.HHError):
        pb.factor_sweeps(3, 5, hh.HH_FP64)        # 32 not divisible by 5
    with pytest.raises(hh.HHError):
        pb.factor_sweeps(3, 32, hh.HH_FP64)       # one interval per strip
    with pytest.raises(hh.HHError):
        pb.factor_sweeps(4, 4, hh.HH_FP64)        # unknown direction bits
    with pytest.raises(hh.HHError):
        pb.mpgmres(torch.zeros((1, 33 * 33), dtype=torch.complex128, device="cuda"))  # not factored
    pb.free()
