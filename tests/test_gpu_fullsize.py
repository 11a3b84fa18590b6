"""Parity at full sizes, in the launch configuration bench.py times.

- The layered 321 x 321 medium (8 layers, k_max 200, 16 strips per
  direction): sampled strip solves and whole sweeps against the oracle's
  LAPACK solves, element by element on the same inputs.  The MPGMRES solve is
  checked on the oracle side by its FP64 residual, its error against the
  oracle's direct solve and the iteration count of the plain FP64 method.
- The 64-source batch of the same medium and the k_max = 800 media on 801^2 and
  1281^2 meshes (32 strips, 8 sources): convergence, and the FP64 residual of
  sampled right-hand sides recomputed on the CPU.

Bars: FP64 kernels 1e-12 relative; complex64 strips 1e-5 (2-norm and
element-wise) where the oracle's own complex64 LAPACK emulation meets it, else
reported as a miss and held to three times the emulation's error (see
_parity.py); solutions 1e-6 residual (1e-6 tolerance, recomputed in FP64) and
1e-5 error against the direct solve; complex64 iteration counts within
floor(1.1 x) of the plain FP64 method's.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import assemble as oasm
from oracle import direct as odr
from oracle import strips as ost
from oracle import sweep as osw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

hh = pytest.importorskip("paper_2408_11929_amd")

from _parity import check_fp32, check_fp64  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.cpu().numpy()


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.fixture(scope="module")
def bench_medium():
    cfg = wl.layered_321()
    return cfg, oasm.assemble(cfg.omega, cfg.c_layers, cfg.n)


@pytest.mark.parametrize("prec", [hh.HH_FP64, hh.HH_FP32])
def test_fullsize_strip_solves(bench_medium, prec):
    cfg, _ = bench_medium
    n, N = cfg.n, cfg.nstrips
    pb = hh.Problem(cfg.omega, cfg.c_layers, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, prec)
    for d, dname in ((hh.HH_DIR_X, ost.X), (hh.HH_DIR_Y, ost.Y)):
        for s in (1, N // 2, N):  # an end strip, an interior one, the other end
            a, w, kl = pb.strip_info(d, s)
            As = ost.strip_matrix(cfg.omega, cfg.c_layers, n, N, dname, s)
            rhs = rand(As.shape[0], 100 * s + d)
            x = host(pb.strip_solve(d, s, dev(rhs)))
            ref = osw.StripSolver(As, kl)
            xr = ref.solve(rhs)
            if prec == hh.HH_FP32:
                x32 = osw.StripSolver(As, kl, np.complex64).solve(rhs)
                check_fp32(x, xr, x32, f"strip solve {cfg.name} {dname}{s}", cond=ref.cond1())
            else:
                check_fp64(x, xr, f"strip solve {cfg.name} {dname}{s}")
    pb.free()


@pytest.mark.parametrize("plan,prec", [("", hh.HH_FP64), ("", hh.HH_FP32), ("0", hh.HH_FP32),
                                       ("2", hh.HH_FP32)])
def test_fullsize_sweeps(bench_medium, prec, plan, monkeypatch):
    # the default plan (sixteen workgroups per chain for one complex64 vector)
    # and the batch plans 0 and 2
    if plan:
        monkeypatch.setenv("HH_SWEEP_PLAN", plan)
    cfg, A = bench_medium
    n, N = cfg.n, cfg.nstrips
    pb = hh.Problem(cfg.omega, cfg.c_layers, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, prec)
    r = rand((1, n * n), 7)
    for d, dname in ((hh.HH_DIR_X, ost.X), (hh.HH_DIR_Y, ost.Y)):
        z = host(pb.sweep_apply(d, dev(r)))[0]
        S = osw.DoubleSweep(cfg.omega, cfg.c_layers, n, N, dname, A=A)
        zr = S.apply(r[0])
        if prec == hh.HH_FP32:
            S32 = osw.DoubleSweep(cfg.omega, cfg.c_layers, n, N, dname, A=A, precision="fp32")
            cond = max(sv.cond1() for sv in S.solvers)
            check_fp32(z, zr, S32.apply(r[0]), f"sweep {cfg.name} {dname} plan={plan or 'auto'}",
                       cond=cond)
        else:
            check_fp64(z, zr, f"sweep {cfg.name} {dname}")
    pb.free()


def test_fullsize_solve_accuracy(bench_medium):
    """The benchmark's solve: FP64 residual and error against the direct solve,
    both recomputed by the oracle, and the iteration count of the plain method."""
    cfg, A = bench_medium
    n, N = cfg.n, cfg.nstrips
    f = cfg.f()
    b = oasm.source_load(n, f[0])
    its = {}
    for prec in (hh.HH_FP32, hh.HH_FP64):
        pb = hh.Problem(cfg.omega, cfg.c_layers, n)
        bd = pb.load_vector(dev(f))
        assert rel(host(bd)[0], b) < 1e-13
        pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, prec)
        x, st, rc = pb.mpgmres(bd, tol=cfg.tol, maxit=cfg.maxit)
        assert rc == hh.HH_OK and st[0]["converged"] == 1
        xh = host(x)[0]
        res = np.linalg.norm(b - A @ xh) / np.linalg.norm(b)
        assert res <= cfg.tol and abs(res - st[0]["res_true"]) <= 1e-3 * res
        if prec == hh.HH_FP32:
            xd = odr.direct_solve(A, b)
            assert rel(xh, xd) <= 1e-5
        its[prec] = st[0]["iterations"]
        pb.free()
    assert its[hh.HH_FP32] <= int(1.1 * its[hh.HH_FP64])


def _sampled_residuals(cfg, f, x, picks):
    A = oasm.assemble(cfg.omega, cfg.c_layers, cfg.n)
    out = []
    for v in picks:
        b = oasm.source_load(cfg.n, f[v])
        out.append(np.linalg.norm(b - A @ x[v]) / np.linalg.norm(b))
    return out


def _batch_solve(cfg, prec=None):
    prec = hh.HH_FP32 if prec is None else prec
    f = cfg.f()
    pb = hh.Problem(cfg.omega, cfg.c_layers, cfg.n)
    b = pb.load_vector(dev(f))
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, cfg.nstrips, prec)
    x, st, rc = pb.mpgmres(b, tol=cfg.tol, maxit=cfg.maxit)
    xh = host(x)
    pb.free()
    return f, xh, st, rc


def test_batched_sources_sampled():
    cfg = wl.layered_321_batch(64)
    f, x, st, rc = _batch_solve(cfg)
    assert rc == hh.HH_OK and all(s["converged"] == 1 for s in st)
    assert max(s["res_true"] for s in st) <= cfg.tol
    picks = [0, 37, 63]
    for v, res in zip(picks, _sampled_residuals(cfg, f, x, picks)):
        assert res <= cfg.tol and abs(res - st[v]["res_true"]) <= 1e-3 * res


@pytest.mark.parametrize("n", [801, 1281])
def test_large_media_sampled(n):
    cfg = wl.large_layered(n)
    f, x, st, rc = _batch_solve(cfg)
    assert rc == hh.HH_OK and all(s["converged"] == 1 for s in st)
    picks = [0, cfg.nsrc - 1]
    for v, res in zip(picks, _sampled_residuals(cfg, f, x, picks)):
        assert res <= cfg.tol and abs(res - st[v]["res_true"]) <= 1e-3 * res
