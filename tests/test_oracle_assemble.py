"""Pins of the oracle's P1 assembly (eq. (1)) against closed forms and invariants."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import assemble as asm


def test_complex_symmetric_not_hermitian():
    # eq. (1) with impedance BC gives a complex symmetric, non-Hermitian matrix
    n, k = 9, 7.0
    A = asm.assemble(k, [1.0], n)
    assert abs(A - A.T).max() == 0.0
    assert abs(A - A.conj().T).max() > 0.1
    # the imaginary part lives on boundary rows only (the impedance term)
    im = abs(A.imag).sum(axis=1).A.ravel().reshape(n, n)
    assert np.all(im[1:-1, 1:-1] == 0.0)
    assert np.all(im[0, :] > 0) and np.all(im[-1, :] > 0)
    assert np.all(im[:, 0] > 0) and np.all(im[:, -1] > 0)


def test_constant_mode_sums():
    # K 1 = 0; 1' M 1 = area = 1; 1' M_Gamma 1 = perimeter = 4  =>  1' A 1 = -k^2 - 4 i k
    n, k = 13, 3.5
    K, Mk2, Mg = asm.operator_parts(k, [1.0], n)
    one = np.ones(n * n)
    assert np.abs(K @ one).max() < 1e-12
    assert one @ Mk2 @ one == pytest.approx(k * k, rel=1e-13)
    assert one @ Mg @ one == pytest.approx(4 * k, rel=1e-13)
    A = asm.assemble(k, [1.0], n)
    assert one @ A @ one == pytest.approx(-k * k - 4j * k, rel=1e-13)


def test_interior_rows_match_textbook_stencils():
    # P1 on right isosceles triangles: stiffness = 5-point Laplacian, mass = 7-point
    n = 11
    h = 1.0 / (n - 1)
    K, M, _ = asm.operator_parts(1.0, [1.0], n)
    i, j = 5, 4
    p = asm.node_id(n, i, j)
    rowK = dict(zip(K[p].indices, K[p].data))
    expect = {p: 4.0, p - 1: -1.0, p + 1: -1.0, p - n: -1.0, p + n: -1.0}
    assert set(k for k, v in rowK.items() if abs(v) > 1e-14) == set(expect)
    for q, v in expect.items():
        assert rowK[q] == pytest.approx(v, abs=1e-13)
    rowM = dict(zip(M[p].indices, M[p].data))
    nb = [p - 1, p + 1, p - n, p + n, p + n + 1, p - n - 1]   # "/" diagonal neighbours
    assert set(k for k, v in rowM.items() if abs(v) > 0) == set(nb + [p])
    assert rowM[p] == pytest.approx(h * h / 2, rel=1e-13)
    for q in nb:
        assert rowM[q] == pytest.approx(h * h / 12, rel=1e-13)


def _exact_layer(y_frac, L):
    return min(int(y_frac * L), L - 1)


def test_layer_classification_exact():
    # centroid heights (3j+1)h/3 and (3j+2)h/3, edge heights jh and (j+1/2)h,
    # classified with exact rational arithmetic
    n, L = 11, 3
    for P in range(0, 6 * (n - 1) + 1):
        y = Fraction(P, 6 * (n - 1))
        assert asm.layer_of(P, n, L) == _exact_layer(y, L)


def test_layered_medium_weighted_sums():
    # layers aligned with grid lines: 1' M_{k^2} 1 = (1/L) sum k_l^2,
    # 1' M_Gamma 1 = 2 (1/L) sum k_l + k_0 + k_{L-1}
    n, L = 17, 4
    c = np.array([1.0, 2.0, 1.5, 3.0])
    omega = 9.0
    kl = omega / c
    _, Mk2, Mg = asm.operator_parts(omega, c, n)
    one = np.ones(n * n)
    assert one @ Mk2 @ one == pytest.approx((kl ** 2).sum() / L, rel=1e-13)
    assert one @ Mg @ one == pytest.approx(2 * kl.sum() / L + kl[0] + kl[-1], rel=1e-13)


def test_source_load_integrates_constant():
    n = 9
    b = asm.source_load(n, np.ones(n * n))
    assert b.sum() == pytest.approx(-1.0, rel=1e-13)


def _plane_wave_error(n, k):
    d = np.array([np.cos(np.pi / 6), np.sin(np.pi / 6)])
    u = lambda x, y: np.exp(1j * k * (d[0] * x + d[1] * y))
    g = lambda x, y, nx, ny: 1j * k * (d[0] * nx + d[1] * ny - 1.0) * u(x, y)
    A = asm.assemble(k, [1.0], n)
    b = asm.impedance_load(n, g)
    uh = spla.spsolve(A.tocsc(), b)
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    e = uh - u(X, Y).ravel()
    M = asm.mass_matrix(n)
    return np.sqrt(abs(np.vdot(e, M @ e)))


@pytest.mark.slow
def test_plane_wave_converges_second_order():
    # u = exp(i k d.x) solves eq. (1a) with f = 0 and du/dn - i k u = i k (d.n - 1) u
    k = 10.0
    ns = [33, 65, 129, 257]
    errs = [_plane_wave_error(n, k) for n in ns]
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] > 1.9 and orders[-1] < 2.1, orders
    assert all(o > 1.7 for o in orders), orders


# ---------------------------------------------------------------- speed fields
# A callable c(x, y) in place of the layer list, sampled at the triangle
# centroids and edge midpoints.

def _grid_transpose(n):
    p = np.arange(n * n)
    i, j = p % n, p // n
    return sp.csr_matrix((np.ones(n * n), (p, i * n + j)), shape=(n * n, n * n))


def test_callable_field_reproduces_layers_off_interfaces():
    # n - 1 = 32 and 5 layers: no centroid or edge midpoint lies on a layer
    # interface, so floor(5 y) classifies every sample point as the exact
    # integer rule does and the two operators are identical
    n, omega, cl = 33, 17.0, [1.0, 2.3, 1.4, 2.9, 1.7]
    Q = 6 * (n - 1)
    assert all((q * Q) % 5 != 0 for q in range(1, 5))
    A = asm.assemble(omega, cl, n)
    Af = asm.assemble(omega, lambda x, y: cl[min(int(5 * y), 4)], n)
    assert abs(A - Af).max() == 0.0
    Ac = asm.assemble(omega, lambda x, y: 1.6, n)
    assert abs(asm.assemble(omega, [1.6], n) - Ac).max() == 0.0


def test_callable_field_transposes_with_the_grid():
    # the "/" triangulation, its centroids and edge midpoints map onto
    # themselves under x <-> y, so A[c] = T A[c^T] T with c^T(x, y) = c(y, x);
    # a swapped or shifted sample coordinate breaks this for a field that is
    # not symmetric
    n, omega = 21, 14.0

    def c(x, y):
        return 1.0 + 0.5 * np.sin(3.0 * x) + 0.2 * y + 0.1 * x * y

    A = asm.assemble(omega, c, n)
    At = asm.assemble(omega, lambda x, y: c(y, x), n)
    T = _grid_transpose(n)
    assert abs(A - T @ At @ T.T).max() < 1e-13 * abs(A).max()
    assert abs(A - At).max() > 1e-3 * abs(A).max()
    # still complex symmetric with K 1 = 0
    assert abs(A - A.T).max() == 0.0
    K, _, _ = asm.operator_parts(omega, c, n)
    assert np.abs(K @ np.ones(n * n)).max() < 1e-12


# ---------------------------------------------------------------- five-point scheme
# Sec. 4's discretisation: five-point differences, the impedance condition
# through eliminated ghost nodes, rows scaled by h^2 times the node weight.

def _fd5_by_ghosts(omega, n):
    """The five-point operator written out node by node: -(Laplacian) - k^2 on
    each node, a ghost value u_out = u_in + 2 i k h u at each boundary side
    (central difference of du/dn = i k u), then the row times h^2 w."""
    h = 1.0 / (n - 1)
    A = np.zeros((n * n, n * n), dtype=complex)
    for j in range(n):
        for i in range(n):
            p = j * n + i
            row = {p: 4.0 / h ** 2 - omega ** 2}
            for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                ii, jj = i + di, j + dj
                if 0 <= ii < n and 0 <= jj < n:
                    q = jj * n + ii
                    row[q] = row.get(q, 0) - 1.0 / h ** 2
                else:  # ghost: mirror neighbour plus 2 i k h u_p
                    q = (j - dj) * n + (i - di)
                    row[q] = row.get(q, 0) - 1.0 / h ** 2
                    row[p] -= 2j * omega * h / h ** 2
            w = (0.5 if i in (0, n - 1) else 1.0) * (0.5 if j in (0, n - 1) else 1.0)
            for q, v in row.items():
                A[p, q] = v * h * h * w
    return A


def test_fd5_rows_follow_from_ghost_elimination():
    n, omega = 9, 10.0
    A = asm.assemble(omega, [1.0], n, scheme="fd5").toarray()
    assert np.abs(A - _fd5_by_ghosts(omega, n)).max() < 1e-13
    assert np.abs(A - A.T).max() == 0.0                      # complex symmetric
    assert np.abs(A - A.conj().T).max() > 0.1                # not Hermitian


def test_fd5_is_second_order_consistent_inside():
    # a plane wave solves the Helmholtz equation: the scaled interior rows
    # applied to it shrink like h^4 (h^2 truncation error times the h^2 scale)
    omega, d = 10.0, (np.cos(0.4), np.sin(0.4))
    res = []
    for n in (33, 65, 129):
        h = 1.0 / (n - 1)
        p = np.arange(n * n)
        x, y = (p % n) * h, (p // n) * h
        u = np.exp(1j * omega * (d[0] * x + d[1] * y))
        A = asm.assemble(omega, [1.0], n, scheme="fd5")
        inner = ((p % n) > 0) & ((p % n) < n - 1) & ((p // n) > 0) & ((p // n) < n - 1)
        res.append(np.abs((A @ u)[inner]).max())
    assert 14.0 < res[0] / res[1] < 18.0 and 14.0 < res[1] / res[2] < 18.0


def test_fd5_sweep_one_strip_is_exact_and_load_is_weighted():
    from oracle import strips as st
    from oracle import sweep as sw
    n, omega, c = 17, 12.0, [1.0, 2.0]
    S = sw.DoubleSweep(omega, c, n, 1, st.X, scheme="fd5")
    r = np.random.default_rng(3).standard_normal(n * n) + 0j
    assert np.linalg.norm(S.A @ S.apply(r) - r) < 1e-12 * np.linalg.norm(r)
    f = np.ones(n * n)
    b = asm.source_load(n, f, scheme="fd5")
    h = 1.0 / (n - 1)
    assert abs(b.sum() + h * h * (n - 1) ** 2) < 1e-12      # sum of weights = area / h^2
