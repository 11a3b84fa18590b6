"""Sequential overlapping strip decomposition (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 2 and Fig. 1: N sequential subdomains Omega_s, 1 <= s <= N, each
overlapping its neighbours; Gamma_{s,1} (s >= 2) is the interface facing
Omega_{s-1}, Gamma_{s,2} (s <= N-1) the one facing Omega_{s+1}.  Sec. 4: the
square is split into N regular strips in x (LRL, left to right) or in y (BTB,
bottom to top) and every internal boundary gets one extra layer of mesh
points, so neighbouring strips overlap by 2h.

Reading c6: with m = (n-1)/N intervals per strip, strip s covers node lines
a_s = max(0, (s-1) m - 1) ... b_s = min(n-1, s m + 1) across the strip and
every node line along it; its triangles are those of the cells between lines
a_s and b_s.  Strip widths are w = m + 3 (interior) and m + 2 (end strips).
m >= 2 is required so that every internal interface lies strictly inside the
square.

Local ordering inside a strip (long index, then short index):
q = long * w + short, where long runs along the strip (y for x-strips, x for
y-strips) and short across it.  The strip matrix is then banded with
kl = ku = w + 1.

The strip matrix A_s is the P1 Helmholtz operator of the sub-rectangle with
the zeroth-order impedance operator on all four of its sides: the physical
boundary keeps eq. (1b), and the internal interfaces carry the transmission
operator of eq. (4), which has the same form.
"""
import numpy as np

from . import assemble as asm

X, Y = "x", "y"


def check_decomposition(n, N):
    if n < 3:
        raise ValueError("need n >= 3")
    if N < 1 or (n - 1) % N != 0:
        raise ValueError("(n-1) must be divisible by the strip count")
    if N > 1 and (n - 1) // N < 2:
        raise ValueError("each strip needs at least 2 intervals")


def strip_lines(n, N, s):
    """Node-line range [a_s, b_s] of strip s (1-based), reading c6."""
    check_decomposition(n, N)
    m = (n - 1) // N
    return max(0, (s - 1) * m - 1), min(n - 1, s * m + 1)


def strip_window(n, N, direction, s):
    """Cell window (cx0, cx1, cy0, cy1) of strip s in the given direction."""
    a, b = strip_lines(n, N, s)
    if direction == X:
        return (a, b, 0, n - 1)
    return (0, n - 1, a, b)


def strip_nodes(n, N, direction, s):
    """Global node ids of strip s in local order q = long * w + short."""
    a, b = strip_lines(n, N, s)
    w = b - a + 1
    long = np.arange(n)[:, None]
    short = np.arange(w)[None, :]
    if direction == X:
        p = asm.node_id(n, a + short, long)
    else:
        p = asm.node_id(n, long, a + short)
    return p.ravel()


def strip_matrix(omega, c_layers, n, N, direction, s, scheme="p1"):
    """A_s in local order (sparse CSR, complex128): the operator of the strip's
    rectangle with the impedance condition on all four of its sides."""
    win = strip_window(n, N, direction, s)
    A_win = asm.assemble(omega, c_layers, n, window=win, scheme=scheme)
    idx = strip_nodes(n, N, direction, s)
    return A_win[idx][:, idx].tocsr()


def interface_rows(n, N, s, side):
    """Local rows of Gamma_{s,1} (side 1, short index 0, s >= 2) or
    Gamma_{s,2} (side 2, short index w-1, s <= N-1); empty otherwise."""
    a, b = strip_lines(n, N, s)
    w = b - a + 1
    if side == 1:
        if s == 1:
            return np.zeros(0, dtype=np.int64)
        return np.arange(n) * w
    if s == N:
        return np.zeros(0, dtype=np.int64)
    return np.arange(n) * w + (w - 1)


def band_width(n, N, s):
    a, b = strip_lines(n, N, s)
    w = b - a + 1
    return w + 1
