"""The five-point scheme of Sec. 4 on the GPU (hh_assemble_field with
HH_SCHEME_FD5): operator, sweeps and MPGMRES against the oracle's five-point
scheme (1e-13, 1e-12, exact iteration count), then the paper-shaped runs of
Table 5 (h = 2^-9, k = 50 and 100, N = 16, 32, 64) with their iteration counts
printed beside the paper's.  Those counts are parity unpinned: the paper does
not give the discrete form of its transmission operator; LRL+BTB is checked
against a loose band around the printed values."""
import os

import numpy as np

import workloads as wl
import pytest

from oracle import assemble as oasm
from oracle import mpgmres as omp
from oracle import strips as ost
from oracle import sweep as osw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hh = pytest.importorskip("paper_2408_11929_amd")

from _parity import check_fp64, rel  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def paper_source(n, k):
    return wl.paper_point_source(n, k)


def upper_diagonals(A, n):
    out = np.zeros((4, n * n), dtype=np.complex128)
    coo = A.tocoo()
    for r, c, v in zip(coo.row, coo.col, coo.data):
        k = {0: 0, 1: 1, n: 2, n + 1: 3}.get(c - r)
        if k is not None:
            out[k, r] += v
    return out


@pytest.mark.parametrize("c", [[1.0], [1.0, 2.1, 1.4]])
def test_fd5_matches_oracle(c):
    n, N, omega = 33, 4, 18.0
    f = paper_source(n, 20.0)
    pb = hh.Problem.from_field(omega, c, n, f=torch.from_numpy(f).to("cuda"), scheme="fd5")
    A = oasm.assemble(omega, c, n, scheme="fd5")
    ref = upper_diagonals(A, n)
    assert np.abs(pb.get_operator() - ref).max() <= 1e-13 * np.abs(ref).max()
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64)
    r = np.random.default_rng(5).standard_normal((1, n * n)) + 0j
    S = {}
    for d, dname in ((hh.HH_DIR_X, ost.X), (hh.HH_DIR_Y, ost.Y)):
        S[dname] = osw.DoubleSweep(omega, c, n, N, dname, A=A, scheme="fd5")
        z = pb.sweep_apply(d, torch.from_numpy(r).to("cuda")).cpu().numpy()[0]
        check_fp64(z, S[dname].apply(r[0]), f"fd5 sweep {dname}")
    b = oasm.source_load(n, f, scheme="fd5")
    x, st, rc = pb.mpgmres(None, tol=1e-10, maxit=100)
    ref = omp.mpgmres(A, [S[ost.X].apply, S[ost.Y].apply], b, tol=1e-10, maxit=100)
    assert rc == hh.HH_OK and st[0]["iterations"] == ref.iterations
    assert rel(x.cpu().numpy()[0], ref.x) < 1e-8
    pb.free()


def test_table5_paper_shaped_runs():
    rows = [list(map(int, ln.split())) for ln in open(os.path.join(GOLD, "table5_h2m9.txt"))
            if ln.strip() and not ln.startswith("#")]
    n = 513
    out = []
    for k, N, lrl_p, both_p in rows:
        # N = 4 and 8 (band half-widths 132 and 68) take the blocked MFMA LU
        # and the lane-major sweep, whose iterations cost about 0.35 s here:
        # LRL alone, which does not converge in this construction (see the
        # Table 4 check in test_golden.py), is run on N >= 16 only
        f = torch.from_numpy(paper_source(n, float(k))).to("cuda")
        pb = hh.Problem.from_field(float(k), [1.0], n, f=f, scheme="fd5")
        pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64)
        x, st, rc = pb.mpgmres(None, tol=1e-6, maxit=200)
        both = st[0]["iterations"]
        assert rc == hh.HH_OK and st[0]["res_true"] <= 1e-6
        one = None
        if N >= 16:
            pb.set_preconditioners(["LRL"])
            x, st1, rc1 = pb.mpgmres(None, tol=1e-6, maxit=200)
            one = st1[0]["iterations"]
        pb.free()
        out.append((k, N, one, lrl_p, both, both_p))
        print(f"[table5] k={k} N={N}: LRL {one} (paper {lrl_p}), LRL+BTB {both} (paper {both_p})",
              flush=True)
    for k, N, one, lrl_p, both, both_p in out:
        assert 0.5 * both_p <= both <= 1.5 * both_p, (k, N, both, both_p)
