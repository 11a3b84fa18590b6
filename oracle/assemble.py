"""P1 assembly of the impedance Helmholtz problem (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The model problem is eq. (1): Delta u + k^2 u = f in the unit square, with the
impedance condition du/dn - i k u = 0 on its boundary, and k = omega / c
(Sec. 1, directly after eq. (1)).  The paper discretises with the 5-point
finite-difference stencil (Sec. 4); this oracle uses continuous P1 triangles
instead, which is the discretisation this library targets.

Mesh (the "/" diagonal in every cell): nodes (i, j) at (i h, j h),
h = 1/(n-1), global index p = j n + i (x fastest).  Each cell
[i, i+1] x [j, j+1] is cut by its "/" diagonal into
    T_lo = {(i,j), (i+1,j), (i+1,j+1)}   and   T_up = {(i,j), (i+1,j+1), (i,j+1)}.

Weak form: multiply eq. (1a) by a test function v, integrate by parts and
insert du/dn = i k u + g on the boundary:
    (K - M_{k^2} - i M_{Gamma,k}) u = G - F,
with K the stiffness matrix, M_{k^2} the mass matrix weighted by k^2,
M_{Gamma,k} the boundary mass matrix weighted by k, F = M f (nodal f,
unweighted mass) and G the boundary load of the impedance data g (g = 0 in
eq. (1b); nonzero only for the manufactured-solution pin).

Variable wave speed (reading c3): c is piecewise constant on L equal
horizontal layers, layer 0 at the bottom.  The element wave number is taken
at the triangle centroid, the edge wave number at the edge midpoint.  A
sample height y = P / (6 (n-1)) lies in layer min(floor(P L / (6(n-1))), L-1),
evaluated in exact integer arithmetic so that a height on a layer interface
is classified without rounding.  A general speed field c(x, y) (a Python
callable in place of the layer list) is sampled at the same points: the
triangle centroids and the edge midpoints, k = omega / c there.

The element matrices are computed here from the vertex coordinates (gradients
of the barycentric functions), not from the tabulated right-triangle forms.
"""
import numpy as np
import scipy.sparse as sp


def node_id(n, i, j):
    """Global node index p = j n + i (x fastest)."""
    return j * n + i


def layer_of(P, n, nlayers):
    """Layer index of the sample height y = P / (6 (n-1)) (reading c3)."""
    Q = 6 * (n - 1)
    P = np.asarray(P, dtype=np.int64)
    return np.minimum((P * nlayers) // Q, nlayers - 1)


def wavenumber(omega, c_layers, n, P):
    """k = omega / c at sample heights y = P / (6 (n-1)) (eq. (1), k = omega/c)."""
    c = np.asarray(c_layers, dtype=np.float64)
    return omega / c[layer_of(P, n, len(c))]


def sampled_wavenumber(omega, c_field, n, P, pts):
    """k = omega / c at the sample points pts (S, 2) in units of h: a layer list
    is read at the heights y = P / (6 (n-1)), a callable c(x, y) at the points."""
    if not callable(c_field):
        return wavenumber(omega, c_field, n, P)
    h = 1.0 / (n - 1)
    c = np.array([float(c_field(x * h, y * h)) for x, y in pts], dtype=np.float64)
    if np.any(~np.isfinite(c)) or np.any(c <= 0):
        raise ValueError("the speed field must be positive and finite")
    return omega / c


def _cells(n, window):
    cx0, cx1, cy0, cy1 = window
    ci, cj = np.meshgrid(np.arange(cx0, cx1), np.arange(cy0, cy1), indexing="xy")
    return ci.ravel().astype(np.int64), cj.ravel().astype(np.int64)


def triangles(n, window=None):
    """Triangles of the cells [cx0, cx1) x [cy0, cy1).

    Returns (tri, P): tri is (T, 3, 2) integer vertex coordinates (i, j) and
    P is the integer numerator of each centroid height y = P / (6 (n-1)).
    """
    if window is None:
        window = (0, n - 1, 0, n - 1)
    ci, cj = _cells(n, window)
    lo = np.stack([np.stack([ci, cj], -1), np.stack([ci + 1, cj], -1),
                   np.stack([ci + 1, cj + 1], -1)], axis=1)
    up = np.stack([np.stack([ci, cj], -1), np.stack([ci + 1, cj + 1], -1),
                   np.stack([ci, cj + 1], -1)], axis=1)
    tri = np.concatenate([lo, up], axis=0)
    # centroid heights: lower triangle (3j+1)h/3, upper triangle (3j+2)h/3
    P = np.concatenate([6 * cj + 2, 6 * cj + 4])
    return tri, P


def boundary_edges(n, window=None):
    """Edges on the four sides of the window rectangle.

    Returns (e, P, normal): e is (E, 2, 2) integer vertex coordinates, P the
    numerator of the midpoint height y = P / (6 (n-1)), normal the outward
    unit normal of the rectangle on that edge.
    """
    if window is None:
        window = (0, n - 1, 0, n - 1)
    cx0, cx1, cy0, cy1 = window
    out_e, out_P, out_n = [], [], []
    ii = np.arange(cx0, cx1)
    jj = np.arange(cy0, cy1)
    for jrow, ny in ((cy0, -1.0), (cy1, 1.0)):            # bottom, top
        e = np.stack([np.stack([ii, np.full_like(ii, jrow)], -1),
                      np.stack([ii + 1, np.full_like(ii, jrow)], -1)], axis=1)
        out_e.append(e)
        out_P.append(np.full(len(ii), 6 * jrow, dtype=np.int64))
        out_n.append(np.tile([0.0, ny], (len(ii), 1)))
    for icol, nx in ((cx0, -1.0), (cx1, 1.0)):            # left, right
        e = np.stack([np.stack([np.full_like(jj, icol), jj], -1),
                      np.stack([np.full_like(jj, icol), jj + 1], -1)], axis=1)
        out_e.append(e)
        out_P.append(6 * jj + 3)
        out_n.append(np.tile([nx, 0.0], (len(jj), 1)))
    return (np.concatenate(out_e).astype(np.int64), np.concatenate(out_P),
            np.concatenate(out_n))


def element_matrices(tri, h):
    """Stiffness and unit-weight mass matrices of each triangle.

    K_e[a, b] = area * grad(phi_a) . grad(phi_b), with the barycentric
    gradients obtained by inverting [[1, x, y]] at the three vertices;
    M_e[a, b] = area / 12 * (1 + delta_ab) (exact P1 mass).
    """
    xy = tri.astype(np.float64) * h                       # (T, 3, 2)
    T = xy.shape[0]
    Mx = np.concatenate([np.ones((T, 3, 1)), xy], axis=2)  # rows [1, x, y]
    C = np.linalg.inv(Mx)                                  # phi_a = C[:, a] . [1, x, y]
    grads = np.transpose(C[:, 1:3, :], (0, 2, 1))          # (T, 3, 2)
    d1 = xy[:, 1] - xy[:, 0]
    d2 = xy[:, 2] - xy[:, 0]
    area = 0.5 * np.abs(d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])
    K = area[:, None, None] * np.einsum("tad,tbd->tab", grads, grads)
    base = (np.ones((3, 3)) + np.eye(3)) / 12.0
    M = area[:, None, None] * base[None]
    return K, M


def edge_mass(e, h):
    """Unit-weight P1 mass matrix of each edge: length / 6 * [[2, 1], [1, 2]]."""
    d = (e[:, 1] - e[:, 0]).astype(np.float64) * h
    length = np.sqrt((d ** 2).sum(1))
    base = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
    return length[:, None, None] * base[None]


def _scatter(n, idx, vals):
    """Sum element matrices vals (E, a, a) with node ids idx (E, a) into CSR."""
    a = idx.shape[1]
    rows = np.repeat(idx, a, axis=1).ravel()
    cols = np.tile(idx, (1, a)).ravel()
    return sp.coo_matrix((vals.ravel(), (rows, cols)), shape=(n * n, n * n)).tocsr()


def operator_parts(omega, c_layers, n, window=None):
    """(K, M_{k^2}, M_{Gamma,k}) assembled over the window's triangles.

    c_layers: the layer speeds, or a callable speed field c(x, y).

    The boundary term covers all four sides of the window rectangle with the
    impedance edge form, whether the side is part of the physical boundary or
    an artificial strip interface (eq. (4) uses the same zeroth-order
    operator du/dn - i k u on internal boundaries as eq. (1b) on the outer
    one).  Rows and columns of nodes outside the window are empty.
    """
    h = 1.0 / (n - 1)
    tri, Pt = triangles(n, window)
    ids = node_id(n, tri[..., 0], tri[..., 1])
    Ke, Me = element_matrices(tri, h)
    kt = sampled_wavenumber(omega, c_layers, n, Pt, tri.mean(axis=1))      # centroids
    K = _scatter(n, ids, Ke)
    Mk2 = _scatter(n, ids, Me * (kt ** 2)[:, None, None])
    e, Pe, _ = boundary_edges(n, window)
    eids = node_id(n, e[..., 0], e[..., 1])
    ke = sampled_wavenumber(omega, c_layers, n, Pe, e.mean(axis=1))        # midpoints
    Mg = _scatter(n, eids, edge_mass(e, h) * ke[:, None, None])
    return K, Mk2, Mg


def fd5_weights(n, window=None):
    """Node weights of the five-point scheme on the window rectangle: 1 inside,
    1/2 on a side, 1/4 at a corner (0 outside the window), and the indicator
    of the window's boundary nodes."""
    if window is None:
        window = (0, n - 1, 0, n - 1)
    cx0, cx1, cy0, cy1 = window
    p = np.arange(n * n)
    i, j = p % n, p // n
    inside = (i >= cx0) & (i <= cx1) & (j >= cy0) & (j <= cy1)
    wx = np.where((i == cx0) | (i == cx1), 0.5, 1.0)
    wy = np.where((j == cy0) | (j == cy1), 0.5, 1.0)
    side = inside & ((i == cx0) | (i == cx1) | (j == cy0) | (j == cy1))
    return np.where(inside, wx * wy, 0.0), side.astype(np.float64)


def node_wavenumber(omega, c_field, n):
    """k = omega / c at the mesh nodes (five-point scheme): a layer list is read
    at the node heights y = 6 j / (6 (n-1)), a callable c(x, y) at the nodes."""
    p = np.arange(n * n)
    i, j = p % n, p // n
    if callable(c_field):
        h = 1.0 / (n - 1)
        c = np.array([float(c_field(a * h, b * h)) for a, b in zip(i, j)])
        return omega / c
    return wavenumber(omega, c_field, n, 6 * j)


def assemble(omega, c_layers, n, window=None, scheme="p1"):
    """A = K - M_{k^2} - i M_{Gamma,k} (complex symmetric, non-Hermitian).

    scheme "p1": weak form of eq. (1) with P1 elements; see the module
    docstring.  scheme "fd5": the standard five-point finite differences of
    Sec. 4 on the same grid, the impedance condition imposed through a ghost
    node outside each boundary node (central difference of du/dn, the ghost
    eliminated) and every row scaled by h^2 times its node weight (1/2 on a
    side, 1/4 at a corner) so that the matrix is complex symmetric:
        A = K - h^2 diag(k^2 w) - i h diag(k [node on the boundary]),
    with K the five-point Laplacian in that scaling (which is the P1 stiffness
    of this mesh) and k taken at the nodes.
    """
    if scheme == "fd5":
        h = 1.0 / (n - 1)
        K, _, _ = operator_parts(omega, [1.0], n, window)
        w, side = fd5_weights(n, window)
        k = node_wavenumber(omega, c_layers, n)
        return (K.astype(np.complex128) - sp.diags(h * h * k * k * w)
                - 1j * sp.diags(h * k * side)).tocsr()
    K, Mk2, Mg = operator_parts(omega, c_layers, n, window)
    return (K.astype(np.complex128) - Mk2 - 1j * Mg).tocsr()


def mass_matrix(n):
    """Unit-weight P1 mass matrix M (used for the load F = M f)."""
    h = 1.0 / (n - 1)
    tri, _ = triangles(n)
    ids = node_id(n, tri[..., 0], tri[..., 1])
    _, Me = element_matrices(tri, h)
    return _scatter(n, ids, Me)


def source_load(n, f_nodal, scheme="p1"):
    """Right-hand side of eq. (1) for the nodal source f and g = 0: b = -M f
    (P1), or b = -h^2 w f in the five-point scheme's row scaling."""
    f = np.asarray(f_nodal, dtype=np.complex128)
    if scheme == "fd5":
        h = 1.0 / (n - 1)
        return -(h * h) * fd5_weights(n)[0] * f
    return -(mass_matrix(n) @ f)


def impedance_load(n, gfun):
    """Boundary load G for impedance data du/dn - i k u = g on the boundary.

    g is given as gfun(x, y, nx, ny) (it depends on the outward normal, which
    differs on the two sides of a corner).  Per boundary edge, g is
    interpolated linearly between the edge's end points:
    G_e = length / 6 * [[2, 1], [1, 2]] [g(p), g(q)].
    """
    h = 1.0 / (n - 1)
    e, _, nrm = boundary_edges(n)
    eids = node_id(n, e[..., 0], e[..., 1])
    xy = e.astype(np.float64) * h
    g = np.stack([gfun(xy[:, a, 0], xy[:, a, 1], nrm[:, 0], nrm[:, 1])
                  for a in range(2)], axis=1).astype(np.complex128)
    Ge = np.einsum("eab,eb->ea", edge_mass(e, h), g)
    out = np.zeros(n * n, dtype=np.complex128)
    np.add.at(out, eids.ravel(), Ge.ravel())
    return out
