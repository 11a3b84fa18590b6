"""MI355X-native multipreconditioned sweeping solver for 2D Helmholtz problems.

Python binding of the C ABI in ``include/hh.h`` (Bootland & Rees, arXiv
2408.11929: selective MPGMRES over directional double-sweep preconditioners
for the impedance Helmholtz problem, discretised with P1 triangles).  The
functions carry the C names; vectors are torch tensors on the GPU
(complex128, contiguous) whose device pointers are handed to the library.
Nothing here computes: it marshals arguments and raises on error codes.
"""
import atexit
import ctypes

import numpy as np

from . import _lib
from ._lib import (HH_DIR_X, HH_DIR_Y, HH_EBUDGET, HH_EDEVICE, HH_EINVAL, HH_ENOCONV,
                   HH_ENOMEM, HH_ESINGULAR, HH_FP32, HH_FP64, HH_OK, HH_PENDING, HH_PRE_BT,
                   HH_PRE_BTB, HH_PRE_LR, HH_PRE_LRL, HH_PRE_RL, HH_PRE_TB, PRE_KINDS, HHError)

_L = None


def lib():
    """The loaded libhh.so (raises ImportError if it has not been built)."""
    global _L
    if _L is None:
        _L = _lib.load()
    return _L


def _check(rc, allowed=(HH_OK,)):
    if rc not in allowed:
        raise HHError(rc, lib().hh_last_error().decode(errors="replace"))
    return rc


def _dev(t, what="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{what} must be a torch tensor on the GPU")
    if t.dtype != torch.complex128 or not t.is_contiguous():
        raise TypeError(f"{what} must be contiguous complex128")
    return ctypes.c_void_p(t.data_ptr())


def _empty_like_vecs(nvec, nn, device):
    import torch
    return torch.empty((nvec, nn), dtype=torch.complex128, device=device)


def _sync():
    import torch
    torch.cuda.synchronize()


class Problem:
    """Handle of an assembled problem (``hh_problem``)."""

    def __init__(self, omega, c_layers, n):
        c = np.ascontiguousarray(np.asarray(c_layers, dtype=np.float64).ravel())
        h = ctypes.c_void_p()
        _check(lib().hh_assemble(float(omega), len(c),
                                 c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(n),
                                 ctypes.byref(h)))
        self._h = h
        self.n = int(n)
        self.omega = float(omega)
        self.c_layers = c

    @classmethod
    def from_field(cls, omega, speed, n, f=None, scheme="p1"):
        """hh_assemble_field: speed is a callable c(x, y) (sampled by the library at
        the triangle centroids, edge midpoints and nodes) or a list of layer
        speeds; f an optional nodal source (device tensor of n*n complex128)
        whose right-hand side the problem keeps; scheme "p1" or "fd5"."""
        sc = {"p1": _lib.HH_SCHEME_P1, "fd5": _lib.HH_SCHEME_FD5}[scheme]
        if callable(speed):
            fn = _lib.SPEED_FN(lambda x, y, ctx: float(speed(x, y)))
            field = _lib.hh_cfield(fn, None, 0, None, sc)
        else:
            c = np.ascontiguousarray(np.asarray(speed, dtype=np.float64).ravel())
            field = _lib.hh_cfield(_lib.SPEED_FN(), None, len(c),
                                   c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), sc)
        h = ctypes.c_void_p()
        fp = _dev(f, "f") if f is not None else None
        _sync()
        _check(lib().hh_assemble_field(float(omega), ctypes.byref(field), int(n), fp,
                                       ctypes.byref(h)))
        self = cls.__new__(cls)
        self._h = h
        self.n = int(n)
        self.omega = float(omega)
        self.c_layers = None
        return self

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("problem has been freed")
        return self._h

    def free(self):
        if getattr(self, "_h", None) is not None:
            lib().hh_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # -- assembly
    def load_vector(self, f, b=None):
        nvec = f.shape[0] if f.dim() == 2 else 1
        if b is None:
            b = _empty_like_vecs(nvec, self.n * self.n, f.device).reshape(f.shape)
        _sync()
        _check(lib().hh_load_vector(self.handle, nvec, _dev(f, "f"), _dev(b, "b")))
        return b

    def get_operator(self):
        out = np.zeros((4, self.n * self.n), dtype=np.complex128)
        _check(lib().hh_get_operator(self.handle, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    # -- strips
    def factor_sweeps(self, dirs=HH_DIR_X | HH_DIR_Y, nstrips=4, precision=HH_FP64, nsub=None):
        """hh_factor_sweeps, or with nsub hh_factor_sweeps_inner (every strip solve
        an inner double sweep over nsub sub-blocks along the strip)."""
        if nsub is None:
            _check(lib().hh_factor_sweeps(self.handle, int(dirs), int(nstrips), int(precision)))
        else:
            _check(lib().hh_factor_sweeps_inner(self.handle, int(dirs), int(nstrips), int(nsub),
                                                int(precision)))
        self.dirs, self.nstrips, self.precision = int(dirs), int(nstrips), int(precision)

    def strip_info(self, direction, s):
        a, w, kl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().hh_strip_info(self.handle, int(direction), int(s), ctypes.byref(a),
                                   ctypes.byref(w), ctypes.byref(kl)))
        return a.value, w.value, kl.value

    def strip_solve(self, direction, s, rhs, x=None):
        if x is None:
            x = rhs.new_empty(rhs.shape)
        _sync()
        _check(lib().hh_strip_solve(self.handle, int(direction), int(s), _dev(rhs, "rhs"),
                                    _dev(x, "x")))
        return x

    def sweep_apply(self, direction, r, z=None):
        nvec = r.shape[0] if r.dim() == 2 else 1
        if z is None:
            z = r.new_empty(r.shape)
        _sync()
        _check(lib().hh_sweep_apply(self.handle, int(direction), nvec, _dev(r, "r"), _dev(z, "z")))
        return z

    def precond_apply(self, kind, r, z=None):
        """z = M^{-1} r for a preconditioner kind (HH_PRE_* or its name, e.g. "RL")."""
        kind = PRE_KINDS[kind] if isinstance(kind, str) else int(kind)
        nvec = r.shape[0] if r.dim() == 2 else 1
        if z is None:
            z = r.new_empty(r.shape)
        _sync()
        _check(lib().hh_precond_apply(self.handle, kind, nvec, _dev(r, "r"), _dev(z, "z")))
        return z

    def set_preconditioners(self, kinds):
        """The preconditioners M_1..M_t combined by mpgmres, e.g. ["LR", "BT", "RL", "TB"]."""
        ks = [PRE_KINDS[k] if isinstance(k, str) else int(k) for k in kinds]
        arr = (ctypes.c_int * len(ks))(*ks)
        _check(lib().hh_set_preconditioners(self.handle, len(ks), arr))

    # -- operator and solver
    def spmv(self, x, y=None):
        nvec = x.shape[0] if x.dim() == 2 else 1
        if y is None:
            y = x.new_empty(x.shape)
        _sync()
        _check(lib().hh_spmv(self.handle, nvec, _dev(x, "x"), _dev(y, "y")))
        return y

    def mpgmres(self, b, tol=1e-6, maxit=200, x=None, x0=None):
        """Returns (x, stats, rc) with stats a list of dicts, rc HH_OK or HH_ENOCONV.
        b None: the right-hand side given to from_field.  x0: starting guess of
        b's shape (hh_mpgmres_x0); it may be x itself to resume in place."""
        import torch
        nrhs = 1 if b is None else (b.shape[0] if b.dim() == 2 else 1)
        if x is None:
            x = (torch.empty((1, self.n * self.n), dtype=torch.complex128, device="cuda")
                 if b is None else b.new_empty(b.shape))
        st = (_lib.hh_stats * nrhs)()
        _sync()
        bp = None if b is None else _dev(b, "b")
        if x0 is not None and x0.numel() != nrhs * self.n * self.n:
            raise ValueError("x0 must hold one n*n vector per right-hand side")
        x0p = None if x0 is None else _dev(x0, "x0")
        rc = _check(lib().hh_mpgmres_x0(self.handle, nrhs, bp, x0p, float(tol), int(maxit),
                                        _dev(x, "x"), st), allowed=(HH_OK, HH_ENOCONV))
        stats = [{k: getattr(s, k) for k, _ in _lib.hh_stats._fields_} for s in st]
        return x, stats, rc


# -- device memory and streams from torch (hh_set_allocator, hh_set_streams)
_torch_hooks = None


def use_torch(memory=True, streams=True):
    """Routes the library's device memory through torch's caching allocator and
    its work onto torch's current stream (for problems created afterwards).
    Memory can only be switched while the library holds none."""
    global _torch_hooks
    import torch
    if memory:
        def _alloc(size, ctx):
            return torch.cuda.caching_allocator_alloc(int(size), device=torch.cuda.current_device())

        def _free(p, ctx):
            torch.cuda.caching_allocator_delete(p)

        hooks = (_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free))
        _check(lib().hh_set_allocator(hooks[0], hooks[1], None))
        _torch_hooks = hooks            # the callbacks must outlive their use
    if streams:
        s = torch.cuda.current_stream().cuda_stream
        _check(lib().hh_set_streams(ctypes.c_void_p(s), ctypes.c_void_p(s)))


def use_library_defaults(memory=True, streams=True):
    """Undoes use_torch: the library's own allocator cache and streams."""
    global _torch_hooks
    if memory:
        _check(lib().hh_set_allocator(_lib.ALLOC_FN(), _lib.FREE_FN(), None))
        _torch_hooks = None
    if streams:
        _check(lib().hh_set_streams(None, None))


def hh_autotune(on=True):
    _check(lib().hh_autotune(1 if on else 0))


def hh_tune_save(path):
    _check(lib().hh_tune_save(str(path).encode()))


def hh_tune_load(path):
    _check(lib().hh_tune_load(str(path).encode()))


def hh_tune_clear():
    _check(lib().hh_tune_clear())


def hh_release_caches():
    _check(lib().hh_release_caches())


@atexit.register
def _release_at_exit():
    # hand the cached device blocks and timing events back while the runtime
    # is still up, rather than leaving them to process teardown
    if _L is not None:
        try:
            _L.hh_release_caches()
        except Exception:
            pass


# C-named entry points
def hh_assemble(omega, c_layers, n):
    return Problem(omega, c_layers, n)


def hh_assemble_field(omega, speed, n, f=None):
    return Problem.from_field(omega, speed, n, f)


def hh_set_streams(x, y):
    _check(lib().hh_set_streams(ctypes.c_void_p(x) if x else None, ctypes.c_void_p(y) if y else None))


def hh_load_vector(pb, f, b=None):
    return pb.load_vector(f, b)


def hh_factor_sweeps(pb, dirs, nstrips, precision):
    return pb.factor_sweeps(dirs, nstrips, precision)


def hh_sweep_apply(pb, direction, r, z=None):
    return pb.sweep_apply(direction, r, z)


def hh_precond_apply(pb, kind, r, z=None):
    return pb.precond_apply(kind, r, z)


def hh_set_preconditioners(pb, kinds):
    return pb.set_preconditioners(kinds)


def hh_strip_solve(pb, direction, s, rhs, x=None):
    return pb.strip_solve(direction, s, rhs, x)


def hh_strip_info(pb, direction, s):
    return pb.strip_info(direction, s)


def hh_spmv(pb, x, y=None):
    return pb.spmv(x, y)


def hh_get_operator(pb):
    return pb.get_operator()


def hh_mpgmres(pb, b, tol=1e-6, maxit=200, x=None):
    return pb.mpgmres(b, tol, maxit, x)


def hh_free(pb):
    pb.free()


def hh_timing_enable(on=True):
    _check(lib().hh_timing_enable(1 if on else 0))


def hh_timing_reset():
    _check(lib().hh_timing_reset())


def hh_timing_get(family):
    n, ms, by = ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
    _check(lib().hh_timing_get(family.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return {"launches": n.value, "ms": ms.value, "bytes": by.value}


from .serving import Server, hh_server_create  # noqa: E402,F401
