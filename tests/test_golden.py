"""Checks against numbers the paper prints (fixtures under tests/golden/)."""
import os

import numpy as np
import pytest

import workloads as wl
from oracle import assemble as asm
from oracle import mpgmres as mp
from oracle import strips as st
from oracle import sweep as sw

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as fh:
        return [list(map(float, ln.split())) for ln in fh if ln.strip() and not ln.startswith("#")]


def test_table3_wavenumbers_from_ppwl_rule():
    for p, k in _rows("table3_ppwl.txt"):
        n = 2 ** int(p) + 1
        assert round(wl.ppwl_wavenumber(n, 10.0), 1) == pytest.approx(k, abs=1e-9)


def test_sec4_quoted_ppwl():
    for p, k, ppwl, tol in _rows("sec4_ppwl_text.txt"):
        h = 2.0 ** -p
        assert 2 * np.pi / (k * h) == pytest.approx(ppwl, abs=ppwl * tol + 0.1)


def test_sec3_inner_product_counts_from_oracle_counter():
    # the oracle counts the inner products it performs; with one CGS pass and
    # one MGS pass the count must equal the paper's printed values
    n, omega, c = 17, 15.0, [1.0, 2.0, 1.5]
    A = asm.assemble(omega, c, n)
    b = np.random.default_rng(0).standard_normal(n * n) + 0j
    all_precs = [sw.DoubleSweep(omega, c, n, N, d, A=A).apply
                 for N, d in ((2, st.X), (2, st.Y), (4, st.X), (4, st.Y))]
    table = {(int(k), int(t)): int(cnt) for k, t, cnt in _rows("sec3_inner_products.txt")}
    for t in (1, 2, 3, 4):
        res = mp.mpgmres(A, all_precs[:t], b, tol=1e-14, maxit=3, cgs_passes=1, block_passes=1)
        for k in range(1, 4):
            assert res.kept_per_iter[k - 1] == t
            assert res.ip_per_iter[k - 1] == table[(k, t)]


@pytest.mark.slow
def test_table4_band_parity_unpinned():
    # paper benchmark source f = 3e4 exp(-200 k r^2) at the centre, k = 50, N = 8
    for p, lrl, lrlbtb in _rows("table4_k50_lrlbtb.txt"):
        n = 2 ** int(p) + 1
        k = 50.0
        A = asm.assemble(k, [1.0], n)
        h = 1.0 / (n - 1)
        x = np.arange(n) * h
        X, Y = np.meshgrid(x, x, indexing="xy")
        f = 3e4 * np.exp(-200 * k * ((X - 0.5) ** 2 + (Y - 0.5) ** 2))
        b = asm.source_load(n, f.ravel())
        SX = sw.DoubleSweep(k, [1.0], n, 8, st.X, A=A)
        SY = sw.DoubleSweep(k, [1.0], n, 8, st.Y, A=A)
        res = mp.mpgmres(A, [SX.apply, SY.apply], b, tol=1e-6)
        assert res.converged
        assert 0.5 * lrlbtb <= res.iterations <= 1.5 * lrlbtb
        one = mp.mpgmres(A, [SX.apply], b, tol=1e-6, maxit=300)
        assert one.converged
        if p <= 7:
            # LRL alone follows the paper's column on the coarser meshes
            assert 0.5 * lrl <= one.iterations <= 1.5 * lrl
        else:
            # a known deviation at h = 2^-8, also with 5-point differences:
            # far above the paper's 15 while LRL+BTB stays in its band; the
            # paper does not give the discrete form of its transmission
            # operator, which is what differs
            assert one.iterations > 3 * lrl
