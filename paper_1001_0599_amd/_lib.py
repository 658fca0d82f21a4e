"""ctypes binding of libcbct (include/cbct.h): argument marshalling only.

Every step of the reconstruction runs in the HIP library; this module converts
torch tensors to device pointers and the current HIP stream, and turns status
codes into exceptions.  It fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcbct.so")

_lock = threading.Lock()
_lib = None


class CbctError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status


STATUS_NAMES = {0: "CBCT_OK", 1: "CBCT_ERR_INVALID_ARG", 2: "CBCT_ERR_OUT_OF_MEMORY", 3: "CBCT_ERR_BUDGET",
                4: "CBCT_ERR_HIP", 5: "CBCT_ERR_NONFINITE", 6: "CBCT_ERR_NOT_FOUND", 7: "CBCT_ERR_INTERNAL"}


class GeometryDesc(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("hx", C.c_double), ("hy", C.c_double), ("hz", C.c_double),
                ("nu", C.c_int), ("nv", C.c_int), ("pu", C.c_double), ("pv", C.c_double),
                ("sad", C.c_double), ("sdd", C.c_double), ("n_views", C.c_int),
                ("angles", C.POINTER(C.c_double)), ("sample_ratio", C.c_double)]


class SolveParams(C.Structure):
    _fields_ = [("lam", C.c_double), ("iters", C.POINTER(C.c_int)), ("levels", C.c_int), ("step", C.c_double),
                ("tv_eps", C.c_double), ("armijo_c", C.c_double), ("backtrack", C.c_double),
                ("rof_tol", C.c_double), ("rof_max_iter", C.c_int), ("rof_max_backtrack", C.c_int),
                ("replay", C.POINTER(C.c_int)), ("replay_len", C.c_int), ("step1_eq6", C.c_int),
                ("conv_tol", C.c_double), ("projector", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("trace", C.POINTER(C.c_int)), ("trace_cap", C.c_int), ("trace_len", C.c_int),
                ("rof_e", C.POINTER(C.c_double)), ("energy", C.POINTER(C.c_double)), ("energy_cap", C.c_int),
                ("energy_len", C.c_int), ("t_used", C.c_double * 8), ("seconds", C.c_double),
                ("replay_used", C.c_int)]


# (name, restype, argtypes) of every exported entry point declared in include/cbct.h
_VP = C.c_void_p
_SIG = [
    ("cbct_context_create", C.c_int, [C.c_int, C.POINTER(_VP)]),
    ("cbct_context_destroy", None, [_VP]),
    ("cbct_context_device", C.c_int, [_VP, C.POINTER(C.c_int)]),
    ("cbct_plan_create", C.c_int, [_VP, C.POINTER(GeometryDesc), C.c_int, C.c_int, C.POINTER(_VP)]),
    ("cbct_plan_destroy", None, [_VP]),
    ("cbct_plan_level_dims", C.c_int, [_VP, C.c_int, C.POINTER(C.c_int)]),
    ("cbct_forward_workspace_size", C.c_int, [_VP, C.c_int, C.POINTER(C.c_size_t)]),
    ("cbct_forward", C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_size_t, _VP]),
    ("cbct_forward_columns", C.c_int, [_VP, C.c_int, _VP, _VP, _VP]),
    ("cbct_backproject_eq6", C.c_int, [_VP, C.c_int, _VP, _VP, _VP]),
    ("cbct_forward_siddon", C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_size_t, _VP]),
    ("cbct_adjoint_siddon_workspace_size", C.c_int, [_VP, C.c_int, C.POINTER(C.c_size_t)]),
    ("cbct_adjoint_siddon", C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_size_t, _VP]),
    ("cbct_adjoint_workspace_size", C.c_int, [_VP, C.c_int, C.POINTER(C.c_size_t)]),
    ("cbct_adjoint", C.c_int, [_VP, C.c_int, _VP, _VP, _VP, C.c_size_t, _VP]),
    ("cbct_solve_params_default", None, [C.POINTER(SolveParams)]),
    ("cbct_reconstruct_workspace_size", C.c_int, [_VP, C.POINTER(SolveParams), C.POINTER(C.c_size_t)]),
    ("cbct_reconstruct", C.c_int, [_VP, C.POINTER(SolveParams), _VP, _VP, _VP, _VP, C.c_size_t, _VP,
                                   C.POINTER(SolveStats)]),
    ("cbct_tv_prox_workspace_size", C.c_int, [_VP, C.c_int, C.POINTER(C.c_size_t)]),
    ("cbct_tv_prox", C.c_int, [_VP, C.c_int, C.POINTER(SolveParams), _VP, _VP, _VP, C.c_size_t, _VP,
                               C.POINTER(SolveStats)]),
    ("cbct_tv_energy_grad_workspace_size", C.c_int, [_VP, C.POINTER(C.c_size_t)]),
    ("cbct_tv_energy_grad", C.c_int, [_VP, C.c_int, C.c_double, _VP, _VP, C.POINTER(C.c_double), _VP, C.c_size_t,
                                      _VP]),
    ("cbct_tv_energy_grad_noalloc", C.c_int, [_VP, C.c_int, C.c_double, _VP, _VP, C.POINTER(C.c_double), _VP]),
    ("cbct_prolong", C.c_int, [_VP, C.c_int, _VP, _VP, _VP]),
    ("cbct_restrict", C.c_int, [_VP, C.c_int, _VP, _VP, _VP]),
    ("cbct_bin_detector", C.c_int, [_VP, C.c_int, _VP, _VP, _VP]),
    ("cbct_server_create", C.c_int, [_VP, C.c_size_t, C.c_int, C.POINTER(_VP)]),
    ("cbct_server_submit", C.c_int, [_VP, C.POINTER(GeometryDesc), C.POINTER(SolveParams), _VP, C.c_int, _VP,
                                     C.POINTER(C.c_uint64)]),
    ("cbct_server_poll", C.c_int, [_VP, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    ("cbct_server_request_times", C.c_int, [_VP, C.c_uint64, C.POINTER(C.c_double)]),
    ("cbct_server_wait_all", C.c_int, [_VP]),
    ("cbct_server_stats", C.c_int, [_VP, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), C.POINTER(C.c_int),
                                    C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_uint64)]),
    ("cbct_server_batch_stats", C.c_int, [_VP, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    ("cbct_server_destroy", None, [_VP]),
    ("cbct_server_create_simulated", C.c_int, [C.c_size_t, C.c_int, C.POINTER(_VP)]),
    ("cbct_server_submit_simulated", C.c_int, [_VP, C.POINTER(GeometryDesc), C.POINTER(SolveParams), C.c_double,
                                               C.POINTER(C.c_uint64)]),
    ("cbct_status_string", C.c_char_p, [C.c_int]),
    ("cbct_last_error", C.c_char_p, []),
]


def exported_names():
    return [n for n, _, _ in _SIG]


def lib():
    """Load libcbct.so (built in-tree by build.py); raises if it is missing."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError("libcbct.so is not built (run python paper_1001_0599_amd/build.py); "
                                  "there is no fallback path")
            L = C.CDLL(LIB_PATH)
            for name, res, args in _SIG:
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


_contexts = {}


def context(device: int):
    """The library context of HIP device `device` (cbct_context_create), made once per process
    and kept until it ends (plans and servers made from it may live as long)."""
    with _lock:
        h = _contexts.get(int(device))
    if h is None:
        h = C.c_void_p()
        check(lib().cbct_context_create(int(device), C.byref(h)))
        with _lock:
            h = _contexts.setdefault(int(device), h)
    return h


def check(status: int) -> None:
    if status != 0:
        msg = lib().cbct_last_error()
        raise CbctError(int(status), msg.decode() if msg else "")
