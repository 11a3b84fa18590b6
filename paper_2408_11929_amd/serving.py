"""Binding of the serving loop (hh_server_* in include/hh.h)."""
import ctypes

import numpy as np

from . import _lib


class Server:
    """Continuous-batching request server (``hh_server``)."""

    def __init__(self, hbm_budget, max_active=64):
        from . import _check, lib
        h = ctypes.c_void_p()
        _check(lib().hh_server_create(int(hbm_budget), int(max_active), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, n, omega, c_layers, f, x, nstrips=16, dirs=3, precision=1, tol=1e-6,
               maxit=200):
        """f, x: GPU complex128 tensors (nsrc, n*n) kept alive until completion."""
        from . import _check, _dev, _sync, lib
        c = np.ascontiguousarray(np.asarray(c_layers, dtype=np.float64).ravel())
        req = _lib.hh_request()
        req.n = int(n)
        req.omega = float(omega)
        req.nlayers = len(c)
        req.c_layers = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        req.nsrc = f.shape[0] if f.dim() == 2 else 1
        req.f = _dev(f, "f").value
        req.x = _dev(x, "x").value
        req.nstrips = int(nstrips)
        req.dirs = int(dirs)
        req.precision = int(precision)
        req.tol = float(tol)
        req.maxit = int(maxit)
        ticket = ctypes.c_uint64()
        _sync()
        _check(lib().hh_submit(self._h, ctypes.byref(req), ctypes.byref(ticket)))
        self._keep[ticket.value] = (f, x)
        return ticket.value

    def poll(self, ticket):
        """None while pending, else a dict of the hh_result fields."""
        from . import _check, lib
        res = _lib.hh_result()
        rc = _check(lib().hh_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(res)),
                    allowed=(_lib.HH_OK, _lib.HH_PENDING))
        if rc == _lib.HH_PENDING:
            return None
        self._keep.pop(ticket, None)
        return {k: getattr(res, k) for k, _ in _lib.hh_result._fields_}

    def clock(self):
        from . import lib
        return lib().hh_server_clock(self._h)

    def destroy(self):
        from . import lib
        if self._h is not None:
            lib().hh_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def hh_server_create(hbm_budget, max_active=64):
    return Server(hbm_budget, max_active)
