"""Recursive strip solves through the C ABI (hh_factor_sweeps_inner, Sec. 4
closing discussion): every strip solve of a sweep is an inner double sweep
over sub-blocks along the strip, checked against oracle/recursive.py.

Bars as in test_gpu_parity.py: FP64 sweeps 1e-12, complex64 against the
oracle's complex64 emulation, MPGMRES by exact iteration count and x to 1e-8."""
import numpy as np
import pytest

from oracle import assemble as oasm
from oracle import mpgmres as omp
from oracle import recursive as orc
from oracle import strips as ost
from oracle import sweep as osw

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hh = pytest.importorskip("paper_2408_11929_amd")

from _parity import check_fp32, check_fp64  # noqa: E402

# (n, N, N2, omega, c): sub-blocks across the strip fastest (w <= len); along
# it (a wide strip, w = 34 against len 10-11); a strip too wide for the
# one-wave LU (kl = 67) whose sub-blocks have kl = 20
CASES = [
    (33, 4, 4, 18.0, [1.0, 2.0, 1.5]),
    (65, 2, 8, 30.0, [1.0, 1.6]),
    (129, 2, 8, 60.0, [1.0, 1.5]),
]


def rand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("prec", [hh.HH_FP64, hh.HH_FP32])
@pytest.mark.parametrize("n,N,N2,omega,c", CASES)
def test_recursive_sweeps_match_oracle(n, N, N2, omega, c, prec):
    pb = hh.Problem(omega, c, n)
    print(f"[recursive] sweeps n={n} N={N} N2={N2} prec={prec}", flush=True)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, prec, nsub=N2)
    A = oasm.assemble(omega, c, n)
    r = rand((2, n * n), 7)
    for d, dname in ((hh.HH_DIR_X, ost.X), (hh.HH_DIR_Y, ost.Y)):
        z = host(pb.sweep_apply(d, dev(r)))
        S = orc.RecursiveSweep(omega, c, n, N, dname, N2, A=A)
        S32 = (orc.RecursiveSweep(omega, c, n, N, dname, N2, A=A, precision="fp32")
               if prec == hh.HH_FP32 else None)
        for v in range(2):
            ref = S.apply(r[v])
            label = f"recursive sweep n={n} N={N} N2={N2} {dname} v{v}"
            if prec == hh.HH_FP32:
                check_fp32(z[v], ref, S32.apply(r[v]), label)
            else:
                check_fp64(z[v], ref, label)
    pb.free()


def test_recursive_single_sweep_matches_oracle():
    n, N, N2, omega, c = CASES[0]
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64, nsub=N2)
    A = oasm.assemble(omega, c, n)
    r = rand((1, n * n), 8)
    for kind, name, d, order in ((hh.HH_PRE_RL, "RL", ost.X, "reverse"),
                                 (hh.HH_PRE_BT, "BT", ost.Y, "forward")):
        z = host(pb.precond_apply(kind, dev(r)))
        ref_op = osw.SingleSweep(omega, c, n, N, d, order=order, A=A)
        ref_op.solvers = [orc.InnerSweep(omega, c, n, N, d, s, N2, ref_op.As[s - 1])
                          for s in range(1, N + 1)]
        check_fp64(z[0], ref_op.apply(r[0]), f"recursive single sweep {name}")
    pb.free()


def test_one_sub_block_matches_the_exact_factorisation():
    n, N, _, omega, c = CASES[0]
    r = rand((1, n * n), 9)
    pa = hh.Problem(omega, c, n)
    pa.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64)
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64, nsub=1)
    for d in (hh.HH_DIR_X, hh.HH_DIR_Y):
        za = host(pa.sweep_apply(d, dev(r)))
        zb = host(pb.sweep_apply(d, dev(r)))
        check_fp64(zb[0], za[0], f"nsub=1 against the exact strip solves, dir {d}")
    pa.free()
    pb.free()


@pytest.mark.parametrize("n,N,N2,omega,c", CASES[:2])
def test_recursive_mpgmres_matches_oracle(n, N, N2, omega, c):
    pb = hh.Problem(omega, c, n)
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64, nsub=N2)
    A = oasm.assemble(omega, c, n)
    b = rand(n * n, 10)
    x, st, rc = pb.mpgmres(dev(b[None]), tol=1e-8, maxit=100)
    precs = [orc.RecursiveSweep(omega, c, n, N, d, N2, A=A).apply for d in (ost.X, ost.Y)]
    ref = omp.mpgmres(A, precs, b, tol=1e-8, maxit=100)
    print(f"[recursive] mpgmres n={n} N2={N2}: gpu {st[0]['iterations']} oracle {ref.iterations}",
          flush=True)
    assert rc == hh.HH_OK and st[0]["iterations"] == ref.iterations
    xg = host(x)[0]
    assert np.linalg.norm(xg - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
    pb.free()


def test_recursive_factorisation_refusals():
    pb = hh.Problem(10.0, [1.0], 33)
    with pytest.raises(hh.HHError, match="nsub"):
        pb.factor_sweeps(hh.HH_DIR_X, 4, hh.HH_FP64, nsub=5)   # 32 % 5 != 0
    with pytest.raises(hh.HHError, match="sub-block needs"):
        pb.factor_sweeps(hh.HH_DIR_X, 4, hh.HH_FP64, nsub=32)  # one interval each
    pb.factor_sweeps(hh.HH_DIR_X, 4, hh.HH_FP64, nsub=4)
    with pytest.raises(hh.HHError, match="inner sweeps"):
        pb.strip_solve(hh.HH_DIR_X, 1, torch.zeros(33 * 11, dtype=torch.complex128, device="cuda"))
    pb.free()


def test_recursive_five_point_sweeps_match_oracle():
    n, N, N2, omega = 65, 2, 8, 30.0
    f = torch.zeros(n * n, dtype=torch.complex128, device="cuda")
    pb = hh.Problem.from_field(omega, [1.0], n, f=f, scheme="fd5")
    pb.factor_sweeps(hh.HH_DIR_X | hh.HH_DIR_Y, N, hh.HH_FP64, nsub=N2)
    A = oasm.assemble(omega, [1.0], n, scheme="fd5")
    r = rand((1, n * n), 13)
    for d, dname in ((hh.HH_DIR_X, ost.X), (hh.HH_DIR_Y, ost.Y)):
        z = host(pb.sweep_apply(d, dev(r)))
        ref = orc.RecursiveSweep(omega, [1.0], n, N, dname, N2, A=A, scheme="fd5").apply(r[0])
        check_fp64(z[0], ref, f"recursive five-point sweep {dname}")
    pb.free()
