"""Full direct solve of the global P1 system (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The reference solution that solver results are compared against.  In the
x-fastest node order the global matrix of eq. (1) is banded with
kl = ku = n + 1, so for moderate n it is factored with LAPACK band LU with
partial pivoting (zgbtrf / zgbtrs).  For large n the band fill becomes
prohibitive (about 1.6 GB at n = 321, over 100 GB at n = 1281) and SuperLU
(scipy.sparse.linalg.splu) stands in; the two agree on every size where both
fit (pinned by a test).
"""
import numpy as np
import scipy.sparse.linalg as spla
from scipy.linalg import lapack

from .sweep import to_lapack_band


def direct_solve(A, b, method="auto"):
    """x = A^{-1} b for the global matrix A (n^2 x n^2, CSR)."""
    N2 = A.shape[0]
    n = int(round(np.sqrt(N2)))
    if method == "auto":
        method = "band" if n <= 161 else "splu"
    b = np.asarray(b, dtype=np.complex128)
    if method == "band":
        kl = n + 1
        ab = to_lapack_band(A.astype(np.complex128), kl, kl, np.complex128)
        lu, piv, info = lapack.zgbtrf(ab, kl, kl)
        if info != 0:
            raise ZeroDivisionError(f"zgbtrf info {info}")
        x, info = lapack.zgbtrs(lu, kl, kl, b.reshape(N2, -1), piv)
        return x[:, 0] if b.ndim == 1 else x
    lu = spla.splu(A.tocsc().astype(np.complex128))
    return lu.solve(b)
