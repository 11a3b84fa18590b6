"""The no-allocation preconditioner entry point (hh_precond_apply_noalloc),
called through the C ABI, against hh_precond_apply on the same inputs: the
same kernels on the library's static scratch, so the results must agree
bit for bit (which meets the 1e-12 / 1e-5 parity bars).  Two calls in a row,
the second on a smaller input, so that what the first left in the shared
scratch cannot leak into the second."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

hh = pytest.importorskip("paper_2408_11929_amd")


def rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def apply(pb, kind, r, noalloc):
    z = torch.full_like(r, complex(np.nan, np.nan))
    fn = hh.lib().hh_precond_apply_noalloc if noalloc else hh.lib().hh_precond_apply
    torch.cuda.synchronize()
    rc = fn(pb.handle, kind, r.shape[0], ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(z.data_ptr()))
    assert rc == hh.HH_OK, hh.lib().hh_last_error()
    return z.cpu().numpy()


@pytest.mark.parametrize("prec", [hh.HH_FP64, hh.HH_FP32])
def test_noalloc_matches_allocating_entry_point(prec):
    # first call: a larger problem and batch (nine vectors: the one-workgroup
    # plan, whose complex64 maps the allocating call builds first); second
    # call: a smaller problem and one vector (the sixteen-workgroup plan for
    # complex64 strips)
    calls = [((64, 9, 30.0, [2.2, 1.1, 1.7, 2.9, 1.3]), 9, hh.HH_PRE_LRL),
             ((33, 4, 18.0, [1.0, 2.0, 1.5]), 1, hh.HH_PRE_TB)]
    for (n, N, omega, c), nvec, kind in calls:
        pb = hh.Problem(omega, c, n)
        pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, prec)
        r = torch.from_numpy(rand((nvec, n * n), n)).to("cuda")
        z_ref = apply(pb, kind, r, noalloc=False)
        z_na = apply(pb, kind, r, noalloc=True)
        assert np.all(np.isfinite(z_na))
        assert np.array_equal(z_na, z_ref), np.abs(z_na - z_ref).max()
        pb.free()


def test_noalloc_on_wide_and_recursive_factorisations():
    # strips beyond the one-wave window (kl = 67, lane-major sweep), then a
    # factorisation with recursive strip solves, two calls in a row on the
    # shared scratch
    calls = [((129, 2, 60.0, [1.0, 1.5]), None, 2, hh.HH_PRE_LRL, hh.HH_FP32),
             ((33, 4, 18.0, [1.0, 2.0, 1.5]), 4, 1, hh.HH_PRE_BT, hh.HH_FP64)]
    for (n, N, omega, c), nsub, nvec, kind, prec in calls:
        pb = hh.Problem(omega, c, n)
        pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, prec, nsub=nsub)
        r = torch.from_numpy(rand((nvec, n * n), n + 1)).to("cuda")
        z_ref = apply(pb, kind, r, noalloc=False)
        z_na = apply(pb, kind, r, noalloc=True)
        assert np.all(np.isfinite(z_na))
        assert np.array_equal(z_na, z_ref), np.abs(z_na - z_ref).max()
        pb.free()


def test_noalloc_rejects_oversized_calls():
    n, N = 321, 16
    pb = hh.Problem(200.0, [1.0], n)
    pb.factor_sweeps(hh.HH_DIR_X, N, hh.HH_FP32)
    # 128 complex64 vectors at n = 321 need about 120 MiB of scratch
    r = torch.zeros((128, n * n), dtype=torch.complex128, device="cuda")
    z = torch.empty_like(r)
    rc = hh.lib().hh_precond_apply_noalloc(pb.handle, hh.HH_PRE_LRL, 128,
                                           ctypes.c_void_p(r.data_ptr()),
                                           ctypes.c_void_p(z.data_ptr()))
    assert rc == hh.HH_EINVAL
    assert b"scratch" in hh.lib().hh_last_error()
    pb.free()
