"""Selective multipreconditioned GMRES (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 3: with t preconditioners M_1..M_t, selective MPGMRES enlarges the
search space by t vectors per iteration and picks the iterate that minimises
the Euclidean norm of the residual over it; with one preconditioner it is
right-preconditioned GMRES.  Its k-th iteration needs t products with A, t
preconditioner solves and (k - 1/2) t^2 + (3/2) t inner products when each
new block is orthogonalised once against the previous basis and then among
itself (modified Gram-Schmidt, t norms included).

Sec. 4 fixes the selection: for two preconditioners, each is applied to the
new basis vector that came from the *other* preconditioner; for more than
two, each is applied to the sum of all new basis vectors of the previous
iteration.

Readings taken where the paper is silent:
  * x0 = 0, no restart, default maxit = 200, relative residual tolerance
    measured in the 2-norm against ||b||.
  * The new block W = A Z_k is orthogonalised against the basis V with
    block classical Gram-Schmidt (``cgs_passes`` passes, default 2), then its
    columns are orthonormalised in order by modified Gram-Schmidt
    (``block_passes`` passes, default 2).  Column c is deflated (adds no
    basis vector) when its norm after orthogonalisation is at most
    ``deflate_tol`` times ||A z_c||; its Z column is kept.
  * The V column produced by W's column c "corresponds" to preconditioner c.
    If only one column survives, every preconditioner is applied to it; if
    none survives the iteration has broken down (the space is invariant).
  * The small least-squares problem min_y ||beta e1 - Hbar y|| is solved
    afresh each iteration with ``numpy.linalg.lstsq`` (minimum-norm
    solution), and its residual is the convergence estimate.
"""
import numpy as np


class Result:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def _as_op(A):
    return A if callable(A) else (lambda v: A @ v)


def mpgmres(A, precs, b, tol=1e-6, maxit=200, cgs_passes=2, block_passes=2,
            deflate_tol=1e-12):
    """Selective MPGMRES (Sec. 3) with the selection rule of Sec. 4.

    A      matrix or callable v -> A v
    precs  list of callables r -> M_i^{-1} r (t = len(precs))
    b      right-hand side (x0 = 0)
    Returns a Result with x, iterations, converged, res_hist (relative
    least-squares residual after each iteration), true_res (FP64
    ||b - A x|| / ||b||), ip_per_iter (inner products of each iteration,
    the deflation reference norms excluded) and kept_per_iter.
    """
    Aop = _as_op(A)
    t = len(precs)
    b = np.asarray(b, dtype=np.complex128)
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return Result(x=np.zeros_like(b), iterations=0, converged=True, res_hist=[],
                      true_res=0.0, ip_per_iter=[], kept_per_iter=[], breakdown=False)
    V = [b / beta]
    Z = []
    Hbar = np.zeros((1, 0), dtype=np.complex128)
    inputs = [V[0]] * t
    res_hist, ip_per_iter, kept_per_iter = [], [], []
    converged = breakdown = False
    y = np.zeros(0, dtype=np.complex128)
    for k in range(1, maxit + 1):
        Zk = [np.asarray(precs[i](inputs[i]), dtype=np.complex128) for i in range(t)]
        W = np.stack([Aop(z) for z in Zk], axis=1)
        ref = np.linalg.norm(W, axis=0)
        m = len(V)
        Vm = np.stack(V, axis=1)
        ip = 0
        h = np.zeros((m, t), dtype=np.complex128)
        for _ in range(cgs_passes):                      # block CGS against V
            hp = Vm.conj().T @ W
            ip += m * t
            W = W - Vm @ hp
            h += hp
        kept = []                                        # (column c, q_c)
        R = np.zeros((t, t), dtype=np.complex128)        # rows = kept order
        for c in range(t):                               # MGS inside the block
            w = W[:, c].copy()
            for _ in range(block_passes):
                for ki, (_, q) in enumerate(kept):
                    r = np.vdot(q, w)
                    ip += 1
                    w = w - r * q
                    R[ki, c] += r
            nrm = np.linalg.norm(w)
            ip += 1
            if nrm > deflate_tol * ref[c]:
                R[len(kept), c] = nrm
                kept.append((c, w / nrm))
        rows, cols = Hbar.shape
        Hn = np.zeros((m + len(kept), cols + t), dtype=np.complex128)
        Hn[:rows, :cols] = Hbar
        Hn[:m, cols:] = h
        Hn[m:m + len(kept), cols:] = R[:len(kept), :]
        Hbar = Hn
        V.extend(q for _, q in kept)
        Z.extend(Zk)
        rhs = np.zeros(Hbar.shape[0], dtype=np.complex128)
        rhs[0] = beta
        y = np.linalg.lstsq(Hbar, rhs, rcond=None)[0]
        res = np.linalg.norm(rhs - Hbar @ y)
        res_hist.append(res / beta)
        ip_per_iter.append(ip)
        kept_per_iter.append(len(kept))
        if res <= tol * beta:
            converged = True
            break
        if not kept:
            breakdown = True
            break
        qs = [q for _, q in kept]
        if t == 2 and len(kept) == 2:
            inputs = [qs[1], qs[0]]                      # cross rule, Sec. 4
        elif len(kept) == 1:
            inputs = [qs[0]] * t
        else:
            ssum = np.sum(np.stack(qs, axis=1), axis=1)  # sum rule, Sec. 4
            inputs = [ssum] * t
    x = np.stack(Z, axis=1) @ y
    true_res = np.linalg.norm(b - Aop(x)) / beta
    return Result(x=x, iterations=k, converged=converged, res_hist=res_hist,
                  true_res=float(true_res), ip_per_iter=ip_per_iter,
                  kept_per_iter=kept_per_iter, breakdown=breakdown)


def _givens(a, b):
    """Complex Givens rotation (c real, s complex) with [[c, s], [-conj(s), c]] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, 1.0 + 0.0j
    rho = np.hypot(abs(a), abs(b))
    return abs(a) / rho, (a / abs(a)) * np.conj(b) / rho


def gmres_right(A, Minv, b, tol=1e-6, maxit=200):
    """Textbook right-preconditioned GMRES (Arnoldi with modified Gram-Schmidt,
    Givens rotations, x0 = 0), written independently of ``mpgmres``: the
    one-preconditioner case of Sec. 3.  Returns (x, iterations, res_hist)."""
    Aop = _as_op(A)
    b = np.asarray(b, dtype=np.complex128)
    beta = np.linalg.norm(b)
    V = [b / beta]
    Z = []
    H = np.zeros((maxit + 1, maxit), dtype=np.complex128)
    cs = np.zeros(maxit)
    sn = np.zeros(maxit, dtype=np.complex128)
    g = np.zeros(maxit + 1, dtype=np.complex128)
    g[0] = beta
    res_hist = []
    j = 0
    for j in range(maxit):
        z = np.asarray(Minv(V[j]), dtype=np.complex128)
        Z.append(z)
        w = Aop(z)
        for i in range(j + 1):
            H[i, j] = np.vdot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        V.append(w / H[j + 1, j] if H[j + 1, j] != 0 else w)
        for i in range(j):
            a, bb = H[i, j], H[i + 1, j]
            H[i, j] = cs[i] * a + sn[i] * bb
            H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * bb
        cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
        a, bb = H[j, j], H[j + 1, j]
        H[j, j] = cs[j] * a + sn[j] * bb
        H[j + 1, j] = 0.0
        g[j + 1] = -np.conj(sn[j]) * g[j]
        g[j] = cs[j] * g[j]
        res_hist.append(abs(g[j + 1]) / beta)
        if abs(g[j + 1]) <= tol * beta:
            break
    kk = j + 1
    y = np.zeros(kk, dtype=np.complex128)
    for i in range(kk - 1, -1, -1):
        y[i] = (g[i] - H[i, i + 1:kk] @ y[i + 1:kk]) / H[i, i]
    x = np.stack(Z[:kk], axis=1) @ y
    return x, kk, res_hist


def inner_products_paper(k, t):
    """Inner products of iteration k with t preconditioners, as counted in Sec. 3."""
    return (k - 0.5) * t * t + 1.5 * t
