"""Serving loop (continuous batching) through the C ABI: each result is the same
alone and in the mix, admission respects the HBM budget, and a request that
fails to converge does not disturb the others.

The server runs every sweep on one workgroup per chain (segment plan 0); a
lone solve would take the wide plan for a single complex64 right-hand side,
which is the same method in another rounding order, so the lone reference
is pinned to plan 0 (HH_SWEEP_PLAN=0) for the bitwise comparison."""
import os
import time

import numpy as np
import pytest

import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hh = pytest.importorskip("paper_2408_11929_amd")

MIX = [
    # n, N, omega, layers, nsrc, precision
    (33, 4, 15.0, [1.0, 2.0], 2, hh.HH_FP64),
    (41, 5, 22.0, [1.4, 1.1, 2.5], 1, hh.HH_FP32),
    (65, 8, 30.0, [1.0, 1.8, 2.6, 1.2], 3, hh.HH_FP32),
    (49, 6, 18.0, [2.0], 2, hh.HH_FP64),
    # a request of the serving stream's smallest size (n = 161, 16 strips, 10
    # points per wavelength at the slowest of 5 layers)
    (161, 16, wl.ppwl_wavenumber(161) * 1.2, [1.2, 2.4, 1.9, 2.8, 1.5], 2, hh.HH_FP32),
]


def sources(n, nsrc, seed):
    pos = wl.source_positions(seed, nsrc)
    f = np.stack([wl.gaussian_field(n, x0, y0, 0.04) for x0, y0 in pos])
    return torch.from_numpy(f).to("cuda")


def alone(n, N, omega, c, f, prec, tol, maxit, dirs=hh.HH_DIR_X | hh.HH_DIR_Y):
    """The request solved on its own, with the server's segment plan."""
    old = os.environ.get("HH_SWEEP_PLAN")
    os.environ["HH_SWEEP_PLAN"] = "0"
    try:
        pb = hh.Problem(omega, c, n)
        b = pb.load_vector(f)
        pb.factor_sweeps(dirs, N, prec)
        x, st, rc = pb.mpgmres(b, tol=tol, maxit=maxit)
        pb.free()
    finally:
        if old is None:
            del os.environ["HH_SWEEP_PLAN"]
        else:
            os.environ["HH_SWEEP_PLAN"] = old
    return x.cpu().numpy(), st, rc


def wait_all(srv, tickets, timeout=60.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        assert time.time() - t0 < timeout, "serving loop made no progress"
        time.sleep(0.002)
    return out


def test_results_identical_alone_and_in_the_mix():
    srv = hh.Server(hbm_budget=8 << 30, max_active=8)
    tickets, xs, refs = [], [], []
    for k, (n, N, omega, c, nsrc, prec) in enumerate(MIX):
        f = sources(n, nsrc, 20 + k)
        x = torch.empty_like(f)
        tickets.append(srv.submit(n, omega, c, f, x, nstrips=N, precision=prec, tol=1e-8, maxit=100))
        xs.append(x)
        refs.append(alone(n, N, omega, c, f, prec, 1e-8, 100))
    res = wait_all(srv, tickets)
    for t, x, (xr, st, rc) in zip(tickets, xs, refs):
        r = res[t]
        assert r["status"] == hh.HH_OK
        assert r["iterations_max"] == max(s["iterations"] for s in st)
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
        got = x.cpu().numpy()
        assert np.array_equal(got, xr), np.abs(got - xr).max()
    srv.destroy()


def test_admission_limits_and_oversized_request_is_refused():
    n, N, omega, c = 33, 4, 15.0, [1.0]
    f = sources(n, 1, 3)
    x1, x2 = torch.empty_like(f), torch.empty_like(f)
    srv = hh.Server(hbm_budget=64 << 20, max_active=1)  # one request at a time
    t1 = srv.submit(n, omega, c, f, x1, nstrips=N, precision=hh.HH_FP32, tol=1e-8, maxit=50)
    t2 = srv.submit(n, omega, c, f, x2, nstrips=N, precision=hh.HH_FP32, tol=1e-8, maxit=50)
    res = wait_all(srv, [t1, t2])
    assert res[t1]["status"] == hh.HH_OK and res[t2]["status"] == hh.HH_OK
    assert res[t2]["t_admit"] >= res[t1]["t_done"]
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    big = sources(321, 4, 4)
    xb = torch.empty_like(big)
    with pytest.raises(hh.HHError) as e:
        srv.submit(321, 100.0, c, big, xb, nstrips=16, precision=hh.HH_FP64, tol=1e-6, maxit=50)
    assert e.value.code == hh.HH_EBUDGET
    srv.destroy()


def test_failing_request_does_not_disturb_others():
    srv = hh.Server(hbm_budget=8 << 30, max_active=8)
    n, N, omega, c = 41, 5, 22.0, [1.0, 2.0]
    f = sources(n, 2, 7)
    good, bad = torch.empty_like(f), torch.empty_like(f)
    tg = srv.submit(n, omega, c, f, good, nstrips=N, precision=hh.HH_FP32, tol=1e-8, maxit=100)
    tb = srv.submit(n, omega, c, f, bad, nstrips=N, precision=hh.HH_FP32, tol=1e-14, maxit=2)
    res = wait_all(srv, [tg, tb])
    assert res[tb]["status"] == hh.HH_ENOCONV
    assert res[tg]["status"] == hh.HH_OK
    xr, st, rc = alone(n, N, omega, c, f, hh.HH_FP32, 1e-8, 100)
    assert np.array_equal(good.cpu().numpy(), xr)
    with pytest.raises(hh.HHError):
        srv.submit(40, omega, c, f, good, nstrips=N)  # (n-1) not divisible by N
    srv.destroy()


def _footprint(n, N, omega, c, f, x, prec, maxit):
    """Smallest HBM budget that admits the request alone (bisection on HH_EBUDGET)."""
    lo, hi = 1 << 20, 64 << 30
    while hi - lo > (1 << 16):
        mid = (lo + hi) // 2
        srv = hh.Server(hbm_budget=mid, max_active=1)
        try:
            srv.submit(n, omega, c, f, x, nstrips=N, precision=prec, tol=1.0, maxit=maxit)
            ok = True
        except hh.HHError as e:
            assert e.code == hh.HH_EBUDGET
            ok = False
        srv.destroy()
        if ok:
            hi = mid
        else:
            lo = mid
    return hi


def test_long_solve_grows_within_budget_next_to_others():
    # one request (the x double sweep alone, i.e. GMRES, on a medium where it
    # needs many iterations) runs past 34 iterations, so that its bases grow
    # twice past the 32 iterations charged at admission, next to a short one;
    # both match their lone runs bit for bit
    srv = hh.Server(hbm_budget=8 << 30, max_active=8)
    n, N, omega, c = 65, 8, 30.0, [1.0, 2.6, 1.3]
    f = sources(n, 1, 9)
    xl, xs = torch.empty_like(f), torch.empty_like(f)
    tl = srv.submit(n, omega, c, f, xl, nstrips=N, dirs=hh.HH_DIR_X, precision=hh.HH_FP64,
                    tol=1e-13, maxit=60)
    ts = srv.submit(n, omega, c, f, xs, nstrips=N, precision=hh.HH_FP32, tol=1e-8, maxit=100)
    res = wait_all(srv, [tl, ts])
    print(f"[serving] long solve: {res[tl]['iterations_max']} iterations, status {res[tl]['status']}")
    assert res[tl]["status"] in (hh.HH_OK, hh.HH_ENOCONV) and res[tl]["iterations_max"] > 34
    assert res[ts]["status"] == hh.HH_OK
    rl = alone(n, N, omega, c, f, hh.HH_FP64, 1e-13, 60, dirs=hh.HH_DIR_X)
    rs = alone(n, N, omega, c, f, hh.HH_FP32, 1e-8, 100)
    assert np.array_equal(xl.cpu().numpy(), rl[0])
    assert np.array_equal(xs.cpu().numpy(), rs[0])
    srv.destroy()


def test_growth_beyond_the_budget_stops_that_request():
    # the budget admits the request (charged for 32 iterations of Krylov
    # memory) but not the growth of its bases at iteration 17: it stops there
    # with HH_EBUDGET; the server then serves the next request normally
    n, N, omega, c = 41, 5, 22.0, [1.0, 2.0]
    f = sources(n, 1, 10)
    xl, xs = torch.empty_like(f), torch.empty_like(f)
    fl = _footprint(n, N, omega, c, f, xl, hh.HH_FP64, 60)
    srv = hh.Server(hbm_budget=fl, max_active=8)
    tl = srv.submit(n, omega, c, f, xl, nstrips=N, precision=hh.HH_FP64, tol=1e-30, maxit=60)
    res = wait_all(srv, [tl])
    assert res[tl]["status"] == hh.HH_EBUDGET and res[tl]["iterations_max"] == 16
    assert np.all(np.isfinite(xl.cpu().numpy()))
    ts = srv.submit(n, omega, c, f, xs, nstrips=N, precision=hh.HH_FP64, tol=1e-6, maxit=16)
    res = wait_all(srv, [ts])
    assert res[ts]["status"] == hh.HH_OK
    rs = alone(n, N, omega, c, f, hh.HH_FP64, 1e-6, 16)
    assert np.array_equal(xs.cpu().numpy(), rs[0])
    srv.destroy()
