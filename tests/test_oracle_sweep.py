"""Pins of the oracle's strips, transmission data and double sweep (Sec. 2, eqs. (2)-(4))."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import assemble as asm
from oracle import strips as st
from oracle import sweep as sw


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_strip_geometry():
    # N strips, one extra mesh line per internal boundary -> overlap 2h (Sec. 4)
    n, N = 25, 4
    m = (n - 1) // N
    prev = None
    covered = np.zeros(n, dtype=bool)
    for s in range(1, N + 1):
        a, b = st.strip_lines(n, N, s)
        w = b - a + 1
        assert w == (m + 2 if s in (1, N) else m + 3)
        covered[a:b + 1] = True
        if prev is not None:
            assert prev[1] - a == 2            # overlap of two cells (2h)
        prev = (a, b)
    assert covered.all()
    with pytest.raises(ValueError):
        st.strip_lines(25, 5, 1)               # (n-1) not divisible
    with pytest.raises(ValueError):
        st.strip_lines(25, 24, 1)              # one interval per strip


def test_strip_matrix_band_and_interior_rows():
    n, N, omega, c = 19, 3, 11.0, [1.0, 2.5, 1.7]
    A = asm.assemble(omega, c, n)
    for d in (st.X, st.Y):
        for s in range(1, N + 1):
            As = st.strip_matrix(omega, c, n, N, d, s)
            kl = st.band_width(n, N, s)
            coo = As.tocoo()
            assert np.max(np.abs(coo.row - coo.col)) == kl
            idx = st.strip_nodes(n, N, d, s)
            z = _rand(n * n, s)
            diff = As @ z[idx] - (A @ z)[idx]
            gamma = np.concatenate([st.interface_rows(n, N, s, 1), st.interface_rows(n, N, s, 2)])
            interior = np.setdiff1d(np.arange(len(idx)), gamma)
            assert np.abs(diff[interior]).max() < 1e-12 * np.abs(diff).max() + 1e-14
            if len(gamma):
                assert np.abs(diff[gamma]).max() > 1e-3


# --- independent stencil form of the transmission data -----------------------------

def _tri_rows(n, omega, c, ci, cj, h):
    """Tabulated element matrices of the two triangles of cell (ci, cj):
    stiffness 1/2 [[1,-1,0],[-1,2,-1],[0,-1,1]] (right angle at the middle vertex),
    mass h^2/24 [[2,1,1],[1,2,1],[1,1,2]] k^2 at the centroid."""
    out = []
    Ks = 0.5 * np.array([[1, -1, 0], [-1, 2, -1], [0, -1, 1]], dtype=float)
    Ms = h * h / 24.0 * np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]], dtype=float)
    for verts, P in (([(ci, cj), (ci + 1, cj), (ci + 1, cj + 1)], 6 * cj + 2),
                     ([(ci, cj), (ci, cj + 1), (ci + 1, cj + 1)], 6 * cj + 4)):
        k = asm.wavenumber(omega, c, n, P)
        out.append((verts, Ks - k * k * Ms))
    return out


def _edge_form(n, omega, c, v0, v1, P, h):
    k = asm.wavenumber(omega, c, n, P)
    return [v0, v1], -1j * k * h / 6.0 * np.array([[2, 1], [1, 2]])


def _stencil_g(n, omega, c, N, s, side, z):
    """g on Gamma_{s,side} of an x-strip from the outside cells and the interface edges."""
    h = 1.0 / (n - 1)
    a, b = st.strip_lines(n, N, s)
    col = a if side == 1 else b
    out_ci = a - 1 if side == 1 else b           # cell column on the other side
    Z = z.reshape(n, n)                           # Z[j, i]
    g = np.zeros(n, dtype=complex)
    for j in range(n):
        node = (col, j)
        acc = 0.0
        # + impedance edges of the interface (inside the strip's operator)
        for jj in (j - 1, j):
            if 0 <= jj <= n - 2:
                verts, E = _edge_form(n, omega, c, (col, jj), (col, jj + 1), 6 * jj + 3, h)
                r = verts.index(node)
                acc += sum(E[r, q] * Z[verts[q][1], verts[q][0]] for q in range(2))
        # - triangles of the outside cell column
        for cj in (j - 1, j):
            if 0 <= cj <= n - 2:
                for verts, E in _tri_rows(n, omega, c, out_ci, cj, h):
                    if node in verts:
                        r = verts.index(node)
                        acc -= sum(E[r, q] * Z[verts[q][1], verts[q][0]] for q in range(3))
        # - physical impedance edge of the outside cell on the bottom/top boundary
        for jb in (0, n - 1):
            if j == jb:
                verts, E = _edge_form(n, omega, c, (out_ci, jb), (out_ci + 1, jb), 6 * jb, h)
                r = verts.index(node)
                acc -= sum(E[r, q] * Z[verts[q][1], verts[q][0]] for q in range(2))
        g[j] = acc
    return g


def test_transmission_matches_stencil_form():
    n, N, omega, c = 19, 3, 13.0, [1.0, 2.5, 1.7]
    S = sw.DoubleSweep(omega, c, n, N, st.X)
    z = _rand(n * n, 7)
    for s in range(N):
        for side in (1, 2):
            rows = st.interface_rows(n, N, s + 1, side)
            g = S.transmission(s, side, z)
            if len(rows) == 0:
                assert np.abs(g).max() == 0
                continue
            ref = _stencil_g(n, omega, c, N, s + 1, side, z)
            assert np.allclose(g[rows], ref, rtol=1e-12, atol=1e-12)
            mask = np.ones(len(g), dtype=bool)
            mask[rows] = False
            assert np.abs(g[mask]).max() == 0


def test_exact_solution_solves_every_local_problem():
    # A_s (R_s u*) = R_s r + g_s(u*) for u* = A^{-1} r
    n, N, omega, c = 21, 4, 17.0, [1.3, 2.2]
    S = sw.DoubleSweep(omega, c, n, N, st.Y)
    r = _rand(n * n, 3)
    u = spla.spsolve(S.A.tocsc(), r)
    for s in range(N):
        rhs = r[S.idx[s]] + S.transmission(s, 1, u) + S.transmission(s, 2, u)
        w = S.solvers[s].solve(rhs)
        assert np.linalg.norm(w - u[S.idx[s]]) < 1e-10 * np.linalg.norm(u)


def test_strip_solve_matches_dense():
    n, N, omega, c = 13, 3, 9.0, [1.0]
    for d in (st.X, st.Y):
        for s in range(1, N + 1):
            As = st.strip_matrix(omega, c, n, N, d, s)
            solver = sw.StripSolver(As, st.band_width(n, N, s))
            rhs = _rand(As.shape[0], s)
            x = solver.solve(rhs)
            xd = np.linalg.solve(As.toarray(), rhs)
            assert np.linalg.norm(x - xd) < 1e-12 * np.linalg.norm(xd)


def test_single_strip_sweep_is_exact_inverse():
    n, omega, c = 15, 12.0, [1.0, 2.0, 1.4]
    for d in (st.X, st.Y):
        S = sw.DoubleSweep(omega, c, n, 1, d)
        r = _rand(n * n, 11)
        z = S.apply(r)
        assert np.linalg.norm(S.A @ z - r) < 1e-12 * np.linalg.norm(r)


def _transpose(v, n):
    return v.reshape(n, n).T.ravel()


def test_btb_is_transposed_lrl_for_constant_speed():
    n, N, omega = 17, 4, 10.0
    SX = sw.DoubleSweep(omega, [1.0], n, N, st.X)
    SY = sw.DoubleSweep(omega, [1.0], n, N, st.Y)
    for s in range(N):
        assert abs(SX.As[s] - SY.As[s]).max() == 0.0
    r = _rand(n * n, 5)
    zy = SY.apply(r)
    zx = _transpose(SX.apply(_transpose(r, n)), n)
    assert np.linalg.norm(zy - zx) < 1e-13 * np.linalg.norm(zy)


def test_sweep_is_linear():
    n, N, omega, c = 13, 3, 8.0, [1.0, 2.0]
    S = sw.DoubleSweep(omega, c, n, N, st.X)
    a, b = _rand(n * n, 1), _rand(n * n, 2)
    al = 0.3 - 1.1j
    lhs = S.apply(a + al * b)
    rhs = S.apply(a) + al * S.apply(b)
    assert np.linalg.norm(lhs - rhs) < 1e-12 * np.linalg.norm(lhs)


def _block_system_sweep(S, r):
    """Eqs. (2)-(3) written as one block lower-triangular system in the unknowns
    (v_1..v_N, u_1..u_{N-1}), solved at once by a sparse direct solver."""
    N, n = S.N, S.n
    sizes = [len(i) for i in S.idx]
    nv = sum(sizes)
    offs_v = np.cumsum([0] + sizes)
    offs_u = nv + np.cumsum([0] + sizes[:-1])
    total = nv + sum(sizes[:-1])

    def G(s, side):
        # matrix of z -> g_{s,side}(z) acting on the global vector (n^2 columns)
        rows = S.rows1[s] if side == 1 else S.rows2[s]
        full = S.As[s] @ sp.identity(n * n, format="csr")[S.idx[s]] - S.A[S.idx[s]]
        keep = sp.diags(np.isin(np.arange(len(S.idx[s])), rows).astype(float))
        return (keep @ full).tocsr()

    def ext(s):
        # extension by zero of strip s's vector to the global grid
        m = len(S.idx[s])
        return sp.csr_matrix((np.ones(m), (S.idx[s], np.arange(m))), shape=(n * n, m))

    blocks = {}
    rhs = np.zeros(total, dtype=complex)
    for s in range(N):                               # forward: v_s
        blocks[("v", s, "v", s)] = S.As[s]
        if s > 0:
            blocks[("v", s, "v", s - 1)] = -(G(s, 1) @ ext(s - 1))
        rhs[offs_v[s]:offs_v[s + 1]] = r[S.idx[s]]
    for s in range(N - 1):                           # backward: u_s, with u_N = v_N
        blocks[("u", s, "u", s)] = S.As[s]
        if s > 0:
            blocks[("u", s, "v", s - 1)] = -(G(s, 1) @ ext(s - 1))
        nxt = ("v", N - 1) if s + 1 == N - 1 else ("u", s + 1)
        blocks[("u", s) + nxt] = -(G(s, 2) @ ext(s + 1))
        rhs[offs_u[s]:offs_u[s] + sizes[s]] = r[S.idx[s]]

    def off(kind, s):
        return offs_v[s] if kind == "v" else offs_u[s]

    big = sp.lil_matrix((total, total), dtype=complex)
    for (k1, s1, k2, s2), B in blocks.items():
        B = sp.coo_matrix(B)
        big[off(k1, s1) + B.row, off(k2, s2) + B.col] = B.data
    sol = spla.spsolve(big.tocsc(), rhs)
    z = np.zeros(n * n, dtype=complex)
    owner = np.full(n * n, -1)
    for s in range(N):                               # lowest-index strip wins
        free = owner[S.idx[s]] < 0
        owner[S.idx[s][free]] = s
    for s in range(N):
        part = sol[offs_u[s]:offs_u[s] + sizes[s]] if s < N - 1 else sol[offs_v[s]:offs_v[s + 1]]
        sel = owner[S.idx[s]] == s
        z[S.idx[s][sel]] = part[sel]
    return z


@pytest.mark.parametrize("direction,N", [(st.X, 2), (st.X, 3), (st.Y, 4)])
def test_sweep_matches_block_triangular_system(direction, N):
    n, omega, c = 13, 9.0, [1.0, 2.2, 1.6]
    S = sw.DoubleSweep(omega, c, n, N, direction)
    for seed in range(2):
        r = _rand(n * n, 20 + seed)
        z = S.apply(r)
        zb = _block_system_sweep(S, r)
        assert np.linalg.norm(z - zb) < 1e-11 * np.linalg.norm(zb)


def test_recomputed_left_data_differs_from_stored():
    # reading c8: the flag switches between eq. (3b) as stated and the recomputed form
    n, N, omega = 13, 3, 9.0
    r = _rand(n * n, 4)
    zs = sw.DoubleSweep(omega, [1.0], n, N, st.X).apply(r)
    zr = sw.DoubleSweep(omega, [1.0], n, N, st.X, backward_left="recomputed").apply(r)
    assert np.linalg.norm(zs - zr) > 1e-6 * np.linalg.norm(zs)


EPS32 = 2.0 ** -24   # unit roundoff of IEEE single precision


def test_complex64_strip_solver_matches_dense_complex64_solve():
    # The complex64 emulation that sets the complex64 parity bars: its band LU
    # (cgbtrf/cgbtrs) must agree with an independent dense complex64 solve
    # (cgesv through numpy) and with the FP64 solve within the error bound
    # kappa_1(A_s) * eps32 (times a small constant); its error must also be
    # that of single precision, not of double.
    n, N, omega, c = 13, 3, 9.0, [1.0, 2.4, 1.6]
    for d in (st.X, st.Y):
        for s in range(1, N + 1):
            As = st.strip_matrix(omega, c, n, N, d, s)
            kl = st.band_width(n, N, s)
            dense = As.toarray()
            kappa = np.linalg.cond(dense, 1)
            rhs = _rand(As.shape[0], 50 + s)
            x64 = np.linalg.solve(dense, rhs)
            x32 = sw.StripSolver(As, kl, np.complex64).solve(rhs)
            xd32 = np.linalg.solve(dense.astype(np.complex64), rhs.astype(np.complex64))
            assert x32.dtype == np.complex64 and xd32.dtype == np.complex64
            e = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
            ed = np.linalg.norm(xd32 - x64) / np.linalg.norm(x64)
            assert 1e-10 < e < 8 * kappa * EPS32, (d, s, e, kappa)
            assert ed < 8 * kappa * EPS32
            assert np.linalg.norm(x32 - xd32) / np.linalg.norm(x64) < 16 * kappa * EPS32
            # the LAPACK-free condition estimate used in the GPU tests' reports
            est = sw.StripSolver(As, kl).cond1()
            assert kappa / 3 <= est <= kappa * (1 + 1e-8)


def test_complex64_sweep_is_single_precision_within_bound():
    # N = 1: the complex64 sweep is a complex64 solve of A (dense cgesv as the
    # independent reference); N > 1: its error against the FP64 sweep stays
    # within (2N - 1) * max_s kappa_1(A_s) * eps32 times a small constant.
    n, omega, c = 17, 12.0, [1.0, 2.0]
    A = asm.assemble(omega, c, n)
    r = _rand(n * n, 9)
    z1 = sw.DoubleSweep(omega, c, n, 1, st.X, A=A, precision="fp32").apply(r)
    dense = A.toarray()
    zd = np.linalg.solve(dense.astype(np.complex64), r.astype(np.complex64))
    x64 = np.linalg.solve(dense, r)
    kappa = np.linalg.cond(dense, 1)
    assert z1.dtype == np.complex64
    assert np.linalg.norm(z1 - zd) / np.linalg.norm(x64) < 16 * kappa * EPS32
    n, N, omega = 33, 4, 20.0
    A = asm.assemble(omega, c, n)
    r = _rand(n * n, 10)
    S = sw.DoubleSweep(omega, c, n, N, st.X, A=A)
    z64 = S.apply(r)
    z32 = sw.DoubleSweep(omega, c, n, N, st.X, A=A, precision="fp32").apply(r)
    assert z32.dtype == np.complex64
    kmax = max(np.linalg.cond(a.toarray(), 1) for a in S.As)
    err = np.linalg.norm(z32 - z64) / np.linalg.norm(z64)
    assert 1e-10 < err < 8 * (2 * N - 1) * kmax * EPS32, (err, kmax)


# ---------------------------------------------------------------- single sweeps
# LR / RL / BT / TB of Sec. 4 (Table 1): one pass of eq. (2) in either order.

@pytest.mark.parametrize("direction", [st.X, st.Y])
@pytest.mark.parametrize("order", ["forward", "reverse"])
def test_single_sweep_one_strip_is_exact_inverse(direction, order):
    n, omega, c = 13, 11.0, [1.0, 1.7, 2.3]
    S = sw.SingleSweep(omega, c, n, 1, direction, order=order)
    r = _rand(n * n, 31)
    z = S.apply(r)
    assert np.linalg.norm(S.A @ z - r) < 1e-12 * np.linalg.norm(r)


def _block_system_single(S, r):
    """One pass of eq. (2) as a block lower-triangular system in v_1..v_N (in the
    sweep's order), solved at once by a sparse direct solver; each node then
    takes the value of the last strip in the sweep's order that contains it."""
    N, n = S.N, S.n
    order = list(range(N)) if S.order == "forward" else list(range(N - 1, -1, -1))
    side = 1 if S.order == "forward" else 2
    sizes = [len(S.idx[s]) for s in order]
    offs = np.cumsum([0] + sizes)
    big = sp.lil_matrix((offs[-1], offs[-1]), dtype=complex)
    rhs = np.zeros(offs[-1], dtype=complex)
    eye = sp.identity(n * n, format="csr")
    for k, s in enumerate(order):
        B = sp.coo_matrix(S.As[s])
        big[offs[k] + B.row, offs[k] + B.col] = B.data
        rhs[offs[k]:offs[k + 1]] = r[S.idx[s]]
        if k > 0:
            prev = order[k - 1]
            rows = S.rows1[s] if side == 1 else S.rows2[s]
            keep = sp.diags(np.isin(np.arange(len(S.idx[s])), rows).astype(float))
            full = S.As[s] @ eye[S.idx[s]] - S.A[S.idx[s]]
            m = len(S.idx[prev])
            ext = sp.csr_matrix((np.ones(m), (S.idx[prev], np.arange(m))), shape=(n * n, m))
            C = sp.coo_matrix(-(keep @ full @ ext))
            big[offs[k] + C.row, offs[k - 1] + C.col] = C.data
    sol = spla.spsolve(big.tocsc(), rhs)
    z = np.zeros(n * n, dtype=complex)
    for k, s in enumerate(order):                    # later strips overwrite
        z[S.idx[s]] = sol[offs[k]:offs[k + 1]]
    return z


@pytest.mark.parametrize("direction,N,order", [(st.X, 3, "forward"), (st.X, 3, "reverse"),
                                               (st.Y, 4, "forward"), (st.Y, 2, "reverse")])
def test_single_sweep_matches_block_triangular_system(direction, N, order):
    n, omega, c = 13, 9.0, [1.0, 2.2, 1.6]
    S = sw.SingleSweep(omega, c, n, N, direction, order=order)
    for seed in range(2):
        r = _rand(n * n, 40 + seed)
        z = S.apply(r)
        zb = _block_system_single(S, r)
        assert np.linalg.norm(z - zb) < 1e-11 * np.linalg.norm(zb)


@pytest.mark.parametrize("direction", [st.X, st.Y])
def test_reverse_sweep_is_rotated_forward_sweep(direction):
    # The half-turn (i, j) -> (n-1-i, n-1-j) maps the "/" triangulation, the
    # impedance boundary and, for a constant speed, the operator onto
    # themselves, and strip s onto strip N+1-s with its two interfaces
    # exchanged: RL = Rot o LR o Rot (Rot reverses the node order).
    n, N, omega = 17, 4, 10.0
    F = sw.SingleSweep(omega, [1.0], n, N, direction, order="forward")
    B = sw.SingleSweep(omega, [1.0], n, N, direction, order="reverse")
    r = _rand(n * n, 6)
    zb = B.apply(r)
    zf = F.apply(r[::-1])[::-1]
    assert np.linalg.norm(zb - zf) < 1e-12 * np.linalg.norm(zb)
    # and the reverse sweep is a different operator from the forward one
    assert np.linalg.norm(zb - F.apply(r)) > 1e-3 * np.linalg.norm(zb)


def test_preconditioner_names():
    n, N, omega = 13, 3, 8.0
    r = _rand(n * n, 8)
    for name, cls, d in [("LRL", sw.DoubleSweep, st.X), ("BTB", sw.DoubleSweep, st.Y),
                         ("LR", sw.SingleSweep, st.X), ("RL", sw.SingleSweep, st.X),
                         ("BT", sw.SingleSweep, st.Y), ("TB", sw.SingleSweep, st.Y)]:
        P = sw.preconditioner(omega, [1.0], n, N, name)
        assert type(P) is cls and P.direction == d
        assert P.strip_solve_count() == (2 * N - 1 if cls is sw.DoubleSweep else N)
        assert np.all(np.isfinite(P.apply(r)))
