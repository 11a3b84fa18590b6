"""Seeded synthetic inputs for the solver, its tests and its benchmark.

This module holds none of the method's arithmetic: it only draws layer wave
speeds, source positions and request arrival times from
``numpy.random.default_rng(seed)`` and samples Gaussian source fields at the
mesh nodes.  Both the HIP library (through its tests and benchmark) and the
CPU oracle consume exactly these arrays.

The paper (Sec. 4) evaluates on a synthetic benchmark, a unit square with a
Gaussian point source in the centre; there is no dataset to stand in for.
The workloads below keep that shape and add the layered media, the source
batches and the request streams of the batched and serving forms.

Draw order within a workload: layer speeds, then source positions, then
arrival times.
"""
import math

import numpy as np

TWO_PI = 2.0 * math.pi


def layer_speeds(seed, nlayers, lo=1.0, hi=3.0):
    """Wave speeds of nlayers equal horizontal layers (bottom first), U[lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=nlayers)


def source_positions(seed, count, skip_layers=0):
    """Source centres uniform in the unit square.  ``skip_layers`` draws that
    many layer speeds first, so that a medium and its sources can share a
    seed in the documented draw order."""
    rng = np.random.default_rng(seed)
    if skip_layers:
        rng.uniform(size=skip_layers)
    return rng.uniform(0.0, 1.0, size=(count, 2))


def gaussian_field(n, x0, y0, sigma, amplitude=1.0):
    """Nodal source f(x, y) = A exp(-((x-x0)^2 + (y-y0)^2) / (2 sigma^2)),
    x-fastest (index j n + i at (i h, j h)), complex128."""
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    f = amplitude * np.exp(-((X - x0) ** 2 + (Y - y0) ** 2) / (2.0 * sigma * sigma))
    return f.ravel().astype(np.complex128)


def ppwl_wavenumber(n, ppwl=10.0):
    """Wave number giving ``ppwl`` points per wavelength on h = 1/(n-1):
    2 pi / (k h) = ppwl (the relation behind Sec. 4's 10-ppwl study)."""
    return TWO_PI * (n - 1) / ppwl


def poisson_arrivals(seed, rate, count):
    """Arrival times (s) of a Poisson process with the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))


class Problem:
    """One solve request: medium, mesh, strips, sources and tolerances."""

    def __init__(self, name, n, omega, c_layers, nstrips, sources, sigma,
                 tol=1e-6, maxit=200):
        self.name, self.n, self.omega = name, n, float(omega)
        self.c_layers = np.asarray(c_layers, dtype=np.float64)
        self.nstrips = nstrips
        self.sources = np.asarray(sources, dtype=np.float64).reshape(-1, 2)
        self.sigma, self.tol, self.maxit = sigma, tol, maxit

    @property
    def nsrc(self):
        return len(self.sources)

    def f(self, which=None):
        """Nodal source fields, shape (nsrc, n*n) (or one field)."""
        if which is not None:
            x0, y0 = self.sources[which]
            return gaussian_field(self.n, x0, y0, self.sigma)
        return np.stack([gaussian_field(self.n, x0, y0, self.sigma)
                         for x0, y0 in self.sources])

    def describe(self):
        return {"workload": self.name, "n": self.n, "omega": self.omega,
                "layers": len(self.c_layers), "nstrips": self.nstrips,
                "nsrc": self.nsrc, "sigma": self.sigma, "tol": self.tol}


def paper_point_source(n, k):
    """The source of Sec. 4's experiments: f = 3e4 exp(-200 k r^2) about the
    centre of the unit square, nodal values (complex) on the n x n grid."""
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    X, Y = np.meshgrid(x, x, indexing="xy")
    return (3e4 * np.exp(-200.0 * k * ((X - 0.5) ** 2 + (Y - 0.5) ** 2))).ravel().astype(complex)


def homogeneous_small():
    """Constant c = 1, k = 20, 101 x 101 nodes, centre Gaussian (sigma 0.02),
    4 strips per direction: the small case the oracle finishes in seconds."""
    return Problem("homogeneous k=20 n=101 N=4", 101, 20.0, [1.0], 4,
                   [[0.5, 0.5]], 0.02)


def layered_321():
    """8 layers, c ~ U[1, 3] (seed 2), omega = 200 min c (k_max = 200),
    321 x 321 nodes (about 10 points per wavelength), 16 strips, centre
    Gaussian (sigma 0.02)."""
    c = layer_speeds(2, 8)
    return Problem("layered 8 layers k_max=200 n=321 N=16", 321, 200.0 * c.min(), c,
                   16, [[0.5, 0.5]], 0.02)


def layered_321_batch(nsrc=64):
    """The 321 x 321 layered medium with nsrc Gaussian sources (sigma 0.01)
    at seeded uniform positions (seed 3)."""
    c = layer_speeds(2, 8)
    pos = source_positions(3, nsrc)
    return Problem(f"layered 8 layers k_max=200 n=321 N=16, {nsrc} sources", 321,
                   200.0 * c.min(), c, 16, pos, 0.01)


def large_layered(n=1281, nsrc=8):
    """k_max = 800 layered medium (8 layers, seed 5) on an n x n mesh,
    32 strips, nsrc sources (sigma 0.01, seed 5 after the layer draws)."""
    c = layer_speeds(5, 8)
    pos = source_positions(5, nsrc, skip_layers=8)
    return Problem(f"layered k_max=800 n={n} N=32, {nsrc} sources", n, 800.0 * c.min(),
                   c, 32, pos, 0.01)


def serving_stream(count=256, seed=4, sizes=(161, 321, 641), nstrips=16, sigma=0.01):
    """Request mix for the serving loop: n uniform over ``sizes``, 4-12 layers
    with c ~ U[1, 3], omega for 10 points per wavelength at the slowest
    layer, 1-16 sources.  Arrival times are drawn separately (poisson_arrivals)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for r in range(count):
        n = int(rng.choice(sizes))
        L = int(rng.integers(4, 13))
        c = rng.uniform(1.0, 3.0, size=L)
        nsrc = int(rng.integers(1, 17))
        pos = rng.uniform(0.0, 1.0, size=(nsrc, 2))
        omega = ppwl_wavenumber(n) * c.min()
        reqs.append(Problem(f"serve#{r} n={n}", n, omega, c, nstrips, pos, sigma))
    return reqs
