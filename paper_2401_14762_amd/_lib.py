"""ctypes declarations of include/csrec.h and the loader of libcsrec.so.

Argument marshalling only: every step of every solver runs in the HIP
kernels of the shared library.  Loading fails loudly when the library has
not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcsrec.so")

CSREC_ABI_VERSION = 2

OK, E_INVAL, E_SHAPE, E_WORKSPACE, E_DEVICE, E_UNSUPPORTED, E_BUDGET = 0, -1, -2, -3, -4, -5, -6
PREC = {"f32": 0, "bf16": 1, "f16": 2}
FLAG_CONVERGED, FLAG_ITER_CAP, FLAG_FP64_FALLBACK, FLAG_NONFINITE, FLAG_FP32_LIMIT = 1, 2, 4, 8, 16
SOLVER_FISTA, SOLVER_GOMP, SOLVER_COSAMP, SOLVER_BIHT, SOLVER_ADMM = 0, 1, 2, 3, 4
SOLVER_FISTA_COMPLEX, SOLVER_FISTA_HERMITIAN, SOLVER_ADMM_HERMITIAN, SOLVER_ADMM_COMPLEX = 5, 6, 7, 8
SOLVER_GOMP_HERMITIAN, SOLVER_COSAMP_HERMITIAN, SOLVER_BIHT_HERMITIAN = 9, 10, 11
ADMM_THR = {"paper": 0, "standard": 1}
PRUNE = {"each": 0, "final": 1}
BIHT_MODE = {"real": 0, "one_bit": 1}
MAX_N = 256


class Problem(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("M", ctypes.c_int32),
        ("N", ctypes.c_int32),
        ("P", ctypes.c_int64),
        ("A", ctypes.c_void_p),
        ("Y", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class PixelStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("resid", ctypes.c_float), ("delta", ctypes.c_float)]


class FistaParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("lambda_", ctypes.c_double),
        ("L", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("X0", ctypes.c_void_p),
        ("prec", ctypes.c_int32),
        ("correction_iters", ctypes.c_int32),
    ]


class AdmmParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("lambda_", ctypes.c_double),
        ("alpha", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("X0", ctypes.c_void_p),
        ("threshold", ctypes.c_int32),
    ]


class GompParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("S", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("res_tol", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("prune", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("pivot_fallback", ctypes.c_double),
        ("redo_tol", ctypes.c_double),
    ]


class CosampParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("eps", ctypes.c_double),
        ("res_tol", ctypes.c_double),
        ("prec", ctypes.c_int32),
    ]


class BihtParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("mu", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("res_tol", ctypes.c_double),
        ("mode", ctypes.c_int32),
        ("Ysign", ctypes.c_void_p),
        ("prec", ctypes.c_int32),
    ]


class ServerCfg(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("device", ctypes.c_int32),
        ("hbm_budget_bytes", ctypes.c_size_t),
        ("batch_pixels", ctypes.c_int64),
        ("chunk_pixels", ctypes.c_int64),
        ("gomp", GompParams),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("tag", ctypes.c_uint64),
        ("status", ctypes.c_int32),
        ("dict_id", ctypes.c_int32),
        ("P", ctypes.c_int64),
        ("N", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("X", ctypes.c_void_p),
        ("support", ctypes.c_void_p),
        ("stats", ctypes.c_void_p),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("tiles_submitted", ctypes.c_int64),
        ("tiles_finished", ctypes.c_int64),
        ("batches", ctypes.c_int64),
        ("pixels_launched", ctypes.c_int64),
        ("host_in_pageable", ctypes.c_int64),
        ("host_out_pageable", ctypes.c_int64),
        ("elapsed_s", ctypes.c_double),
        ("busy_s", ctypes.c_double),
        ("mean_pixels_in_flight", ctypes.c_double),
        ("mean_pool_bytes", ctypes.c_double),
    ]


# every symbol the header declares, with (restype, argtypes)
_P = ctypes.POINTER
SIGNATURES = {
    "csrec_abi_version": (ctypes.c_int32, []),
    "csrec_strerror": (ctypes.c_char_p, [ctypes.c_int32]),
    "csrec_last_hip_error": (ctypes.c_int32, []),
    "csrec_workspace_bytes": (ctypes.c_int32, [ctypes.c_int32, _P(Problem), ctypes.c_void_p,
                                               _P(ctypes.c_size_t)]),
    "csrec_fista": (ctypes.c_int32, [_P(Problem), _P(FistaParams), ctypes.c_void_p, ctypes.c_void_p]),
    "csrec_fista_complex": (ctypes.c_int32, [_P(Problem), _P(FistaParams), ctypes.c_void_p, ctypes.c_void_p]),
    "csrec_fista_hermitian": (ctypes.c_int32, [_P(Problem), _P(FistaParams), ctypes.c_void_p, ctypes.c_void_p]),
    "csrec_gomp": (ctypes.c_int32, [_P(Problem), _P(GompParams), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "csrec_gomp_noalloc": (ctypes.c_int32, [_P(Problem), _P(GompParams), ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "csrec_gomp_hermitian": (ctypes.c_int32, [_P(Problem), _P(GompParams), ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "csrec_cosamp_hermitian": (ctypes.c_int32, [_P(Problem), _P(CosampParams), ctypes.c_void_p, ctypes.c_void_p,
                                                ctypes.c_void_p]),
    "csrec_biht_hermitian": (ctypes.c_int32, [_P(Problem), _P(BihtParams), ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "csrec_cosamp": (ctypes.c_int32, [_P(Problem), _P(CosampParams), ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "csrec_biht": (ctypes.c_int32, [_P(Problem), _P(BihtParams), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "csrec_admm": (ctypes.c_int32, [_P(Problem), _P(AdmmParams), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p]),
    "csrec_admm_hermitian": (ctypes.c_int32, [_P(Problem), _P(AdmmParams), ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "csrec_admm_complex": (ctypes.c_int32, [_P(Problem), _P(AdmmParams), ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "csrec_sparsify": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "csrec_sparsify_dft": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int32,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "csrec_lipschitz": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "csrec_server_create": (ctypes.c_int32, [_P(ServerCfg), _P(ctypes.c_void_p)]),
    "csrec_server_add_dict": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                               ctypes.c_int32, _P(ctypes.c_int32)]),
    "csrec_server_submit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.c_int64, _P(GompParams), ctypes.c_uint64]),
    "csrec_server_poll": (ctypes.c_int32, [ctypes.c_void_p, _P(Result), ctypes.c_int32,
                                           _P(ctypes.c_int32)]),
    "csrec_server_release": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64]),
    "csrec_server_drain": (ctypes.c_int32, [ctypes.c_void_p]),
    "csrec_server_get_stats": (ctypes.c_int32, [ctypes.c_void_p, _P(ServerStats)]),
    "csrec_server_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
}

_lib = None


class CsrecError(RuntimeError):
    def __init__(self, code: int, what: str):
        lib = _lib
        msg = lib.csrec_strerror(code).decode() if lib is not None else str(code)
        extra = ""
        if code == E_DEVICE and lib is not None:
            extra = f" (hip error {lib.csrec_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{code}]{extra}")
        self.code = code


def load(path: str = LIB_PATH):
    """Load libcsrec.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_2401_14762_amd.build); there is no CPU fallback")
    # PyTorch ships its own libamdhip64.so.7.  Loaded first, this library would
    # map the system copy as well, and a second HIP runtime in the process
    # shares neither devices nor pointers with torch's.  With torch imported
    # first, the library binds to the runtime that owns the tensors it gets.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.csrec_abi_version() != CSREC_ABI_VERSION:
        raise RuntimeError("libcsrec ABI version mismatch")
    _lib = lib
    return lib


def check(code: int, what: str) -> None:
    if code != OK:
        raise CsrecError(code, what)
