"""The segment-plan autotuner: with tuning on, the first launch of a shape
times the plans that fit and keeps the fastest; the solves stay within the
parity bars; a saved choice, loaded into a run with tuning off, replays the
same plan and so the same results bit for bit."""
import json

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


def solve(n, N, omega, c, f, tol):
    pb = hh.Problem(omega, c, n)
    b = pb.load_vector(torch.from_numpy(f).to("cuda"))
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP32)
    x, st, rc = pb.mpgmres(b, tol=tol, maxit=100)
    out = x.cpu().numpy(), [s["iterations"] for s in st], rc
    pb.free()
    return out


def test_tuned_plan_is_replayed_from_json(tmp_path):
    n, N, omega, c = 65, 8, 30.0, [1.0, 1.8, 2.6, 1.2]
    pos = wl.source_positions(17, 6)
    f = np.stack([wl.gaussian_field(n, x0, y0, 0.03) for x0, y0 in pos])
    hh.hh_tune_clear()
    hh.hh_autotune(True)
    try:
        x1, its1, rc1 = solve(n, N, omega, c, f, 1e-8)   # measures, then solves
        x2, its2, rc2 = solve(n, N, omega, c, f, 1e-8)   # reuses the choice
        path = tmp_path / "tune.json"
        hh.hh_tune_save(path)
    finally:
        hh.hh_autotune(False)
    assert rc1 == rc2 == hh.HH_OK and its1 == its2
    assert np.array_equal(x1, x2)
    entries = json.loads(path.read_text())["entries"]
    assert entries and all(e["plan"] in (0, 1, 2, 3) for e in entries)
    for e in entries:
        timed = [m for m in e["ms"] if m > 0]
        assert e["ms"][e["plan"]] == min(timed)
    print(f"[tune] {entries}", flush=True)
    # a fresh table loaded from the file, tuning off: the same plan, the same bits
    hh.hh_tune_clear()
    hh.hh_tune_load(path)
    x3, its3, rc3 = solve(n, N, omega, c, f, 1e-8)
    assert its3 == its2 and np.array_equal(x3, x2)
    hh.hh_tune_clear()
    # and the tuned solve is the method: each RHS against the oracle
    A = oasm.assemble(omega, c, n)
    SX = osw.DoubleSweep(omega, c, n, N, ost.X, A=A)
    SY = osw.DoubleSweep(omega, c, n, N, ost.Y, A=A)
    for v in (0, 5):
        b = oasm.source_load(n, f[v])
        ref = omp.mpgmres(A, [SX.apply, SY.apply], b, tol=1e-8, maxit=100)
        res = np.linalg.norm(b - A @ x1[v]) / np.linalg.norm(b)
        assert res < 1e-8 * 1.01 and abs(its1[v] - ref.iterations) <= max(1, ref.iterations // 10)
