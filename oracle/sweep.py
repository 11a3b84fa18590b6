"""Double-sweep preconditioners with Robin transmission (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 2, eqs. (2)-(4).  Forward sweep, eq. (2): for s = 1..N solve on Omega_s
with the transmission data of v_{s-1} on Gamma_{s,1} (s >= 2) and zero data on
Gamma_{s,2}.  Backward sweep, eq. (3): for s = N-1..1 solve on Omega_s with
the data of v_{s-1} on Gamma_{s,1} and the data of u_{s+1} on Gamma_{s,2};
u_N = v_N, so the last strip is solved once (2N - 1 strip solves).  In the
overlaps, the values of the most recent strip solve are kept (no partition
of unity), so at the end every node holds u of the lowest-index strip that
contains it.  Seen discretely (Sec. 2, opening paragraph) this is a
forward/backward block substitution with approximate Schur complements.

Discrete transmission data (reading c7): for a global vector z,
    g_s(z) = A_s R_s z - R_s A z,
kept on the rows of Gamma_{s,1} (-> g_{s,1}) and of Gamma_{s,2}
(-> g_{s,2}) and zero elsewhere.  It is the discrete form of the integral of
(dz/dn_s - i k z) phi_i over the interface, eq. (4): A_s carries the
impedance edge terms on the interface, A carries the triangles on the other
side instead.  The exact solution u* = A^{-1} r therefore satisfies every
local problem A_s (R_s u*) = R_s r + g_s(u*).

Reading c8: the backward solve on strip s reuses the g_{s,1} that was formed
from v_{s-1} in the forward sweep, as eq. (3b) states.  The alternative
(recomputing it from the current global vector) is kept behind a flag.

Single sweeps (Sec. 4, the LR, RL, BT and TB preconditioners of Table 1):
one pass of eq. (2) only.  The forward order (LR in x, BT in y) solves
s = 1..N with the data of the previous solve on Gamma_{s,1} and zero data on
Gamma_{s,2}; the reverse order (RL, TB) solves s = N..1 with the data of the
previous solve on Gamma_{s,2} and zero data on Gamma_{s,1}.  Each is N strip
solves, and in the overlaps the most recent solve wins (the highest-index
strip for the forward order, the lowest for the reverse order).

Strip solves use LAPACK band LU with partial pivoting (zgbtrf / zgbtrs, or
cgbtrf / cgbtrs for the complex64 diagnostic), standing in for the sparse
direct solver of Sec. 4.
"""
import numpy as np
import scipy.sparse.linalg as spla
from scipy.linalg import lapack

from . import assemble as asm
from . import strips as st


def to_lapack_band(A, kl, ku, dtype):
    """LAPACK general-band storage: ab[kl + ku + i - j, j] = A[i, j]."""
    coo = A.tocoo()
    if coo.nnz and (np.max(coo.row - coo.col) > kl or np.max(coo.col - coo.row) > ku):
        raise ValueError("matrix entries outside the declared band")
    ab = np.zeros((2 * kl + ku + 1, A.shape[0]), dtype=dtype, order="F")
    ab[kl + ku + coo.row - coo.col, coo.col] = coo.data
    return ab


class StripSolver:
    """Band LU with partial pivoting of one strip matrix (LAPACK gbtrf)."""

    def __init__(self, A_s, kl, dtype=np.complex128):
        self.kl = self.ku = kl
        self.dtype = dtype
        self.A = A_s.astype(dtype)
        ab = to_lapack_band(self.A, kl, kl, dtype)
        trf = lapack.zgbtrf if dtype == np.complex128 else lapack.cgbtrf
        self.lu, self.piv, info = trf(ab, kl, kl)
        if info > 0:
            raise ZeroDivisionError(f"exactly singular strip matrix (pivot {info})")
        if info < 0:
            raise ValueError(f"gbtrf argument error {info}")

    def solve(self, rhs):
        trs = lapack.zgbtrs if self.dtype == np.complex128 else lapack.cgbtrs
        b = np.asarray(rhs, dtype=self.dtype)
        one = b.ndim == 1
        x, info = trs(self.lu, self.kl, self.ku, b.reshape(b.shape[0], -1), self.piv)
        if info != 0:
            raise ValueError(f"gbtrs error {info}")
        return x[:, 0] if one else x

    def cond1(self):
        """LAPACK-free estimate of the 1-norm condition number of A_s."""
        n = self.A.shape[0]
        inv = spla.LinearOperator((n, n), matvec=self.solve,
                                  rmatvec=lambda v: np.conj(self._solve_h(np.conj(v))),
                                  dtype=self.dtype)
        anorm = abs(self.A).sum(axis=0).max()
        return float(anorm * spla.onenormest(inv))

    def _solve_h(self, v):
        trs = lapack.zgbtrs if self.dtype == np.complex128 else lapack.cgbtrs
        x, _ = trs(self.lu, self.kl, self.ku, np.asarray(v, self.dtype).reshape(-1, 1),
                   self.piv, trans=2)
        return np.conj(x[:, 0])


class DoubleSweep:
    """M^{-1} of one double sweep: LRL (direction 'x') or BTB ('y').

    precision 'fp64': everything complex128 (the oracle proper).
    precision 'fp32': strip matrices, their LU, the transmission data and the
    strip solves in complex64; the input is rounded to complex64 and the
    output is returned exactly (a diagnostic of the error attainable with
    complex64 strips, not a parity reference).
    """

    def __init__(self, omega, c_layers, n, N, direction, A=None, precision="fp64",
                 backward_left="stored", scheme="p1"):
        st.check_decomposition(n, N)
        self.n, self.N, self.direction = n, N, direction
        self.dtype = np.complex128 if precision == "fp64" else np.complex64
        self.backward_left = backward_left
        A = asm.assemble(omega, c_layers, n, scheme=scheme) if A is None else A
        self.A = A.astype(self.dtype)
        self.idx, self.As, self.solvers, self.rows1, self.rows2 = [], [], [], [], []
        for s in range(1, N + 1):
            A_s = st.strip_matrix(omega, c_layers, n, N, direction, s, scheme=scheme)
            kl = st.band_width(n, N, s)
            self.idx.append(st.strip_nodes(n, N, direction, s))
            self.As.append(A_s.astype(self.dtype))
            self.solvers.append(StripSolver(A_s, kl, self.dtype))
            self.rows1.append(st.interface_rows(n, N, s, 1))
            self.rows2.append(st.interface_rows(n, N, s, 2))

    def transmission(self, s, side, z):
        """g_{s,side}(z) = (A_s R_s z - R_s A z) on the interface rows (0-based s)."""
        idx = self.idx[s]
        rows = self.rows1[s] if side == 1 else self.rows2[s]
        full = self.As[s] @ z[idx] - (self.A @ z)[idx]
        g = np.zeros(len(idx), dtype=self.dtype)
        g[rows] = full[rows]
        return g

    def apply(self, r):
        """z = M^{-1} r by the forward sweep, eq. (2), then the backward sweep, eq. (3)."""
        N = self.N
        r = np.asarray(r).astype(self.dtype)
        z = np.zeros(self.n * self.n, dtype=self.dtype)
        g1 = [None] * N
        for s in range(N):                                   # forward: v_s
            g1[s] = self.transmission(s, 1, z)
            z[self.idx[s]] = self.solvers[s].solve(r[self.idx[s]] + g1[s])
        for s in range(N - 2, -1, -1):                       # backward: u_s
            left = g1[s] if self.backward_left == "stored" else self.transmission(s, 1, z)
            rhs = r[self.idx[s]] + left + self.transmission(s, 2, z)
            z[self.idx[s]] = self.solvers[s].solve(rhs)
        return z

    def strip_solve_count(self):
        return 2 * self.N - 1

    def dense(self):
        """Dense matrix of M^{-1} (apply to unit vectors); tiny n only."""
        m = self.n * self.n
        out = np.zeros((m, m), dtype=self.dtype)
        for p in range(m):
            e = np.zeros(m, dtype=self.dtype)
            e[p] = 1
            out[:, p] = self.apply(e)
        return out


class SingleSweep(DoubleSweep):
    """M^{-1} of one single sweep (Sec. 4, Table 1): order 'forward' is LR
    (direction 'x') or BT ('y'), order 'reverse' is RL ('x') or TB ('y').
    Same strips, strip matrices and transmission data as the double sweep."""

    def __init__(self, omega, c_layers, n, N, direction, order="forward", A=None,
                 precision="fp64", scheme="p1"):
        if order not in ("forward", "reverse"):
            raise ValueError("order must be 'forward' or 'reverse'")
        super().__init__(omega, c_layers, n, N, direction, A=A, precision=precision,
                         scheme=scheme)
        self.order = order

    def apply(self, r):
        """z = M^{-1} r: N strip solves in the sweep's order, each with the
        transmission data of the previous solve on the interface it faces."""
        N = self.N
        r = np.asarray(r).astype(self.dtype)
        z = np.zeros(self.n * self.n, dtype=self.dtype)
        if self.order == "forward":
            for s in range(N):            # Gamma_{s,1} data of v_{s-1}, zero on Gamma_{s,2}
                z[self.idx[s]] = self.solvers[s].solve(r[self.idx[s]] + self.transmission(s, 1, z))
        else:
            for s in range(N - 1, -1, -1):  # Gamma_{s,2} data of v_{s+1}, zero on Gamma_{s,1}
                z[self.idx[s]] = self.solvers[s].solve(r[self.idx[s]] + self.transmission(s, 2, z))
        return z

    def strip_solve_count(self):
        return self.N


def preconditioner(omega, c_layers, n, N, name, A=None, precision="fp64"):
    """The preconditioner named as in Sec. 4: LRL, BTB (double sweeps), LR, RL,
    BT, TB (single sweeps)."""
    table = {"LRL": (st.X, None), "BTB": (st.Y, None),
             "LR": (st.X, "forward"), "RL": (st.X, "reverse"),
             "BT": (st.Y, "forward"), "TB": (st.Y, "reverse")}
    if name not in table:
        raise ValueError(f"unknown preconditioner {name!r}")
    d, order = table[name]
    if order is None:
        return DoubleSweep(omega, c_layers, n, N, d, A=A, precision=precision)
    return SingleSweep(omega, c_layers, n, N, d, order=order, A=A, precision=precision)
