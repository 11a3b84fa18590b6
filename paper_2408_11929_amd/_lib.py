"""ctypes binding of libhh.so (the C ABI in include/hh.h).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  The library must have been built (``__graft_entry__.build()`` or
``python paper_2408_11929_amd/build.py``); importing this module without it
raises ``ImportError`` rather than falling back to anything else.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhh.so")

HH_OK = 0
HH_PENDING = 1
HH_EINVAL = -1
HH_ENOMEM = -2
HH_ESINGULAR = -3
HH_ENOCONV = -4
HH_EDEVICE = -5
HH_EBUDGET = -6
HH_DIR_X = 1
HH_DIR_Y = 2
HH_FP64 = 0
HH_FP32 = 1
HH_PRE_LRL = 1
HH_PRE_BTB = 2
HH_PRE_LR = 3
HH_PRE_RL = 4
HH_PRE_BT = 5
HH_PRE_TB = 6
PRE_KINDS = {"LRL": HH_PRE_LRL, "BTB": HH_PRE_BTB, "LR": HH_PRE_LR, "RL": HH_PRE_RL,
             "BT": HH_PRE_BT, "TB": HH_PRE_TB}

ERROR_NAMES = {HH_EINVAL: "HH_EINVAL", HH_ENOMEM: "HH_ENOMEM", HH_ESINGULAR: "HH_ESINGULAR",
               HH_ENOCONV: "HH_ENOCONV", HH_EDEVICE: "HH_EDEVICE", HH_EBUDGET: "HH_EBUDGET"}


class hh_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int),
                ("res_est", ctypes.c_double), ("res_true", ctypes.c_double),
                ("basis_size", ctypes.c_int), ("deflated", ctypes.c_int)]


class hh_request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("omega", ctypes.c_double), ("nlayers", ctypes.c_int),
                ("c_layers", ctypes.POINTER(ctypes.c_double)), ("nsrc", ctypes.c_int),
                ("f", ctypes.c_void_p), ("x", ctypes.c_void_p), ("nstrips", ctypes.c_int),
                ("dirs", ctypes.c_uint), ("precision", ctypes.c_int), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int)]


SPEED_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_void_p)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class hh_cfield(ctypes.Structure):
    _fields_ = [("speed", SPEED_FN), ("ctx", ctypes.c_void_p), ("nlayers", ctypes.c_int),
                ("c_layers", ctypes.POINTER(ctypes.c_double)), ("scheme", ctypes.c_int)]


HH_SCHEME_P1 = 0
HH_SCHEME_FD5 = 1


class hh_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations_max", ctypes.c_int),
                ("res_true_max", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


P = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double
U = ctypes.c_uint

# name -> (restype, argtypes); the full exported surface of include/hh.h
PROTOTYPES = {
    "hh_assemble": (I, [D, I, ctypes.POINTER(D), I, ctypes.POINTER(P)]),
    "hh_assemble_field": (I, [D, ctypes.POINTER(hh_cfield), I, P, ctypes.POINTER(P)]),
    "hh_set_allocator": (I, [ALLOC_FN, FREE_FN, P]),
    "hh_set_streams": (I, [P, P]),
    "hh_release_caches": (I, []),
    "hh_autotune": (I, [I]),
    "hh_tune_save": (I, [ctypes.c_char_p]),
    "hh_tune_load": (I, [ctypes.c_char_p]),
    "hh_tune_clear": (I, []),
    "hh_load_vector": (I, [P, I, P, P]),
    "hh_factor_sweeps": (I, [P, U, I, I]),
    "hh_factor_sweeps_inner": (I, [P, U, I, I, I]),
    "hh_sweep_apply": (I, [P, U, I, P, P]),
    "hh_precond_apply": (I, [P, I, I, P, P]),
    "hh_precond_apply_noalloc": (I, [P, I, I, P, P]),
    "hh_set_preconditioners": (I, [P, I, ctypes.POINTER(I)]),
    "hh_strip_solve": (I, [P, U, I, P, P]),
    "hh_strip_info": (I, [P, U, I, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
    "hh_spmv": (I, [P, I, P, P]),
    "hh_get_operator": (I, [P, P]),
    "hh_mpgmres": (I, [P, I, P, D, I, P, ctypes.POINTER(hh_stats)]),
    "hh_mpgmres_x0": (I, [P, I, P, P, D, I, P, ctypes.POINTER(hh_stats)]),
    "hh_free": (I, [P]),
    "hh_last_error": (ctypes.c_char_p, []),
    "hh_timing_enable": (I, [I]),
    "hh_timing_reset": (I, []),
    "hh_timing_get": (I, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_longlong),
                          ctypes.POINTER(D), ctypes.POINTER(D)]),
    "hh_server_create": (I, [ctypes.c_size_t, I, ctypes.POINTER(P)]),
    "hh_submit": (I, [P, ctypes.POINTER(hh_request), ctypes.POINTER(ctypes.c_uint64)]),
    "hh_poll": (I, [P, ctypes.c_uint64, ctypes.POINTER(hh_result)]),
    "hh_server_clock": (D, [P]),
    "hh_server_destroy": (I, [P]),
}


def load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


class HHError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code
