"""The boundary's remaining calls through the C ABI: a general speed field
with the source given at assembly (hh_assemble_field), device memory and
streams supplied by torch (hh_set_allocator, hh_set_streams).

Bars as in test_gpu_parity.py: FP64 operator 1e-13 and sweeps 1e-12 against
the oracle assembled with the same callable speed; MPGMRES by exact iteration
count and solution to 1e-8; with torch's memory and stream the benchmark
solve must be bitwise the one with the library's own."""
import gc

import numpy as np
import pytest

import workloads as wl
from oracle import assemble as oasm
from oracle import mpgmres as omp
from oracle import strips as ost
from oracle import sweep as osw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hh = pytest.importorskip("paper_2408_11929_amd")

from _parity import check_fp64, rel  # noqa: E402


def speed(x, y):
    return 1.0 + 0.5 * np.sin(3.0 * x) + 0.3 * y + 0.2 * x * y


def upper_diagonals(A, n):
    out = np.zeros((4, n * n), dtype=np.complex128)
    coo = A.tocoo()
    for r, c, v in zip(coo.row, coo.col, coo.data):
        k = {0: 0, 1: 1, n: 2, n + 1: 3}.get(c - r)
        if k is not None:
            out[k, r] += v
    return out


def test_speed_field_matches_oracle():
    n, N, omega = 33, 4, 18.0
    f = wl.gaussian_field(n, 0.4, 0.6, 0.05)
    pb = hh.Problem.from_field(omega, speed, n, f=torch.from_numpy(f).to("cuda"))
    A = oasm.assemble(omega, speed, n)
    got = pb.get_operator()
    ref = upper_diagonals(A, n)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64)
    r = np.random.default_rng(4).standard_normal((1, n * n)) + 0j
    for d, dname in ((hh.HH_DIR_X, ost.X), (hh.HH_DIR_Y, ost.Y)):
        z = pb.sweep_apply(d, torch.from_numpy(r).to("cuda")).cpu().numpy()[0]
        check_fp64(z, osw.DoubleSweep(omega, speed, n, N, dname, A=A).apply(r[0]),
                   f"field sweep {dname}")
    # the right-hand side given at assembly: b = -M f
    x, st, rc = pb.mpgmres(None, tol=1e-10, maxit=100)
    b = oasm.source_load(n, f)
    precs = [osw.DoubleSweep(omega, speed, n, N, d, A=A).apply for d in (ost.X, ost.Y)]
    ref = omp.mpgmres(A, precs, b, tol=1e-10, maxit=100)
    assert rc == hh.HH_OK and st[0]["iterations"] == ref.iterations
    assert rel(x.cpu().numpy()[0], ref.x) < 1e-8
    pb.free()


def test_speed_field_rejects_bad_speeds():
    with pytest.raises(hh.HHError) as e:
        hh.Problem.from_field(10.0, lambda x, y: -1.0 if x > 0.5 else 1.0, 17)
    assert e.value.code == hh.HH_EINVAL
    with pytest.raises(hh.HHError):
        hh.Problem.from_field(10.0, lambda x, y: float("nan"), 17)


def _bench_solve():
    cfg = wl.layered_321()
    f = torch.from_numpy(cfg.f()).to("cuda")
    pb = hh.Problem(cfg.omega, cfg.c_layers, cfg.n)
    b = pb.load_vector(f)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, cfg.nstrips, hh.HH_FP32)
    x, st, rc = pb.mpgmres(b, tol=cfg.tol, maxit=cfg.maxit)
    torch.cuda.synchronize()
    out = x.cpu().numpy(), st[0]["iterations"], rc
    pb.free()
    return out


def test_torch_memory_and_streams_give_identical_results():
    x0, it0, rc0 = _bench_solve()
    gc.collect()
    side = torch.cuda.Stream()
    try:
        with torch.cuda.stream(side):
            hh.use_torch(memory=True, streams=True)
            before = torch.cuda.memory_allocated()
            cfg = wl.layered_321()
            pb = hh.Problem(cfg.omega, cfg.c_layers, cfg.n)
            # the operator (4 n^2 complex128) came from torch's allocator
            assert torch.cuda.memory_allocated() - before >= 4 * cfg.n ** 2 * 16
            pb.free()
            x1, it1, rc1 = _bench_solve()
    finally:
        gc.collect()
        hh.use_library_defaults()
    assert rc0 == rc1 == hh.HH_OK and it0 == it1
    assert np.array_equal(x0, x1)


def test_allocator_cannot_change_while_memory_is_held():
    pb = hh.Problem(10.0, [1.0], 17)
    with pytest.raises(hh.HHError) as e:
        hh.use_torch(memory=True, streams=False)
    assert e.value.code == hh.HH_EINVAL
    pb.free()
