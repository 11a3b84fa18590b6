"""Strips wider than the one-wave LU window (band half-width kl > 63): the
blocked band LU with matrix-core trailing updates and the lane-major
substitution with two or three window slots (Sec. 2 and Sec. 4 set-up; the
strips of Table 5 with N = 4 and 8 at h = 2^-9 have kl = 132 and 68).

Bars as in test_gpu_parity.py: strip solves against LAPACK on the oracle's
strip matrices and sweeps against the oracle at 1e-12 in FP64 and the
complex64 bar in FP32; MPGMRES by exact iteration count and x to 1e-8."""
import numpy as np
import pytest

from oracle import assemble as oasm
from oracle import mpgmres as omp
from oracle import strips as ost
from oracle import sweep as osw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hh = pytest.importorskip("paper_2408_11929_amd")

from _parity import check_fp32, check_fp64  # noqa: E402

# (n, N, omega, c): kl = 67 (two slots) with ragged ns = 129 * 66; kl = 131
# (three slots); an under-resolved mesh whose factorisation interchanges rows
# inside the blocked elimination
BANDS = [
    (129, 2, 60.0, [1.0, 1.5]),
    (257, 2, 90.0, [1.2, 0.8, 1.0]),
    (129, 2, 420.0, [1.0]),
]


def rand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("prec", [hh.HH_FP64, hh.HH_FP32])
@pytest.mark.parametrize("n,N,omega,c", BANDS)
def test_wide_strip_solves_match_lapack(n, N, omega, c, prec):
    pb = hh.Problem(omega, c, n)
    print(f"[wideband] strip solves n={n} N={N} omega={omega} prec={prec}", flush=True)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, prec)
    for d, dname in ((hh.HH_DIR_X, ost.X), (hh.HH_DIR_Y, ost.Y)):
        for s in range(1, N + 1):
            a, w, kl = pb.strip_info(d, s)
            assert kl == ost.band_width(n, N, s) and kl > 63
            As = ost.strip_matrix(omega, c, n, N, dname, s)
            rhs = rand(As.shape[0], 10 * s + d)
            x = host(pb.strip_solve(d, s, dev(rhs)))
            ref = osw.StripSolver(As, kl)
            xr = ref.solve(rhs)
            if prec == hh.HH_FP32:
                x32 = osw.StripSolver(As, kl, np.complex64).solve(rhs)
                check_fp32(x, xr, x32, f"wide strip solve n={n} N={N} {dname}{s}", cond=ref.cond1())
            else:
                check_fp64(x, xr, f"wide strip solve n={n} N={N} {dname}{s}")
    pb.free()


@pytest.mark.parametrize("prec", [hh.HH_FP64, hh.HH_FP32])
@pytest.mark.parametrize("n,N,omega,c", BANDS[:2])
def test_wide_sweeps_match_oracle(n, N, omega, c, prec):
    pb = hh.Problem(omega, c, n)
    print(f"[wideband] sweeps n={n} N={N} prec={prec}", flush=True)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, prec)
    A = oasm.assemble(omega, c, n)
    r = rand((2, n * n), 5)
    for d, dname in ((hh.HH_DIR_X, ost.X), (hh.HH_DIR_Y, ost.Y)):
        z = host(pb.sweep_apply(d, dev(r)))
        S = osw.DoubleSweep(omega, c, n, N, dname, A=A)
        S32 = osw.DoubleSweep(omega, c, n, N, dname, A=A, precision="fp32") if prec == hh.HH_FP32 else None
        for v in range(2):
            ref = S.apply(r[v])
            if prec == hh.HH_FP32:
                check_fp32(z[v], ref, S32.apply(r[v]), f"wide sweep n={n} N={N} {dname} v{v}")
            else:
                check_fp64(z[v], ref, f"wide sweep n={n} N={N} {dname} v{v}")
    pb.free()


def test_wide_single_sweeps_match_oracle():
    n, N, omega, c = BANDS[0]
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64)
    A = oasm.assemble(omega, c, n)
    r = rand((1, n * n), 9)
    for kind, name in ((hh.HH_PRE_LR, "LR"), (hh.HH_PRE_TB, "TB")):
        z = host(pb.precond_apply(kind, dev(r)))
        ref = osw.preconditioner(omega, c, n, N, name, A=A).apply(r[0])
        check_fp64(z[0], ref, f"wide single sweep {name}")
    pb.free()


def test_wide_mpgmres_matches_oracle():
    n, N, omega, c = BANDS[0]
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64)
    A = oasm.assemble(omega, c, n)
    b = rand(n * n, 11)
    x, st, rc = pb.mpgmres(dev(b[None]), tol=1e-8, maxit=60)
    precs = [osw.DoubleSweep(omega, c, n, N, d, A=A).apply for d in (ost.X, ost.Y)]
    ref = omp.mpgmres(A, precs, b, tol=1e-8, maxit=60)
    print(f"[wideband] mpgmres gpu {st[0]['iterations']} oracle {ref.iterations}", flush=True)
    assert rc == hh.HH_OK and st[0]["iterations"] == ref.iterations
    xg = host(x)[0]
    assert np.linalg.norm(xg - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
    pb.free()


def test_bands_beyond_the_lane_major_window_are_refused():
    pb = hh.Problem(10.0, [1.0], 513)  # N = 2: kl = 259 > 191
    with pytest.raises(hh.HHError, match="band half-width"):
        pb.factor_sweeps(hh.HH_DIR_X, 2, hh.HH_FP32)
    pb.free()


def test_wide_five_point_sweeps_match_oracle():
    # the strips of Table 5's N = 4 column at a smaller size: five-point
    # scheme, kl = 67, against the oracle's five-point sweep
    n, N, omega = 129, 2, 60.0
    f = torch.zeros(n * n, dtype=torch.complex128, device="cuda")
    pb = hh.Problem.from_field(omega, [1.0], n, f=f, scheme="fd5")
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64)
    A = oasm.assemble(omega, [1.0], n, scheme="fd5")
    r = rand((1, n * n), 12)
    for d, dname in ((hh.HH_DIR_X, ost.X), (hh.HH_DIR_Y, ost.Y)):
        z = host(pb.sweep_apply(d, dev(r)))
        ref = osw.DoubleSweep(omega, [1.0], n, N, dname, A=A, scheme="fd5").apply(r[0])
        check_fp64(z[0], ref, f"wide five-point sweep {dname}")
    pb.free()
