"""ctypes binding of liblbmgnn.so: the same entry points as include/lbmgnn.h.

Arguments are marshalled only; every computation runs in the HIP library.
Importing this module never falls back to anything else: if the library is
missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmgnn.so")

LBM_WS_MOMENTS = 0
LBM_WS_GNN_STEP = 1
LBM_WS_GNN_FORWARD = 2
LBM_WS_GNN_SAVED = 3
LBM_WS_GNN_BACKWARD = 4
LBM_WS_MSE = 5
LBM_WS_SIMPLE = 6
LBM_NOALLOC_MAX_NODES = 65536   # lattice nodes lbm_step_gnn_noalloc's static scratch holds

EXPORTS = [
    "lbm_last_error", "lbm_init", "lbm_init_f64", "lbm_step_bgk", "lbm_step_bgk_f64",
    "lbm_stream", "lbm_init_ce", "lbm_init_ce_f64",
    "lbm_step_channel", "lbm_step_channel_f64", "lbm_channel_profile",
    "lbm_moments", "lbm_restrict", "lbm_copy", "gnn_param_count", "gnn_blob_len",
    "lbm_step_gnn", "lbm_step_gnn_noalloc", "gnn_forward", "gnn_backward", "gnn_mse",
    "gnn_mse_weighted", "gnn_adam",
    "lbm_step_simple", "lbm_step_simple_channel", "simple_forward", "gnn_gelu_rate",
    "lbm_workspace_bytes",
]


class LbmTgv(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("u0", "kx", "ky", "x0", "y0", "nu", "t")]


class LbmFallback(ctypes.Structure):
    _fields_ = [("drift_threshold", ctypes.c_double),
                ("flags", ctypes.c_void_p),
                ("n_fallback", ctypes.c_void_p),
                ("mass", ctypes.c_void_p)]


class LbmError(RuntimeError):
    pass


_lib = None


def load(path: str = LIB_PATH):
    """Load the library and declare every signature (raises if missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise LbmError(f"{path} is not built; run paper_2504_14494_amd/build.py "
                       "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(path)
    vp, i, f, d, sz = (ctypes.c_void_p, ctypes.c_int, ctypes.c_float,
                       ctypes.c_double, ctypes.c_size_t)
    sig = {
        "lbm_last_error": ([], ctypes.c_char_p),
        "lbm_init": ([vp, i, i, vp, vp, vp, vp], i),
        "lbm_init_f64": ([vp, i, i, vp, vp, vp, vp], i),
        "lbm_step_bgk": ([vp, vp, i, i, f, vp], i),
        "lbm_step_bgk_f64": ([vp, vp, i, i, d, vp], i),
        "lbm_stream": ([vp, vp, i, i, i, vp], i),
        "lbm_step_channel": ([vp, vp, i, i, f, f, vp], i),
        "lbm_step_channel_f64": ([vp, vp, i, i, d, d, vp], i),
        "lbm_channel_profile": ([vp, i, i, f, vp, vp], i),
        "lbm_init_ce": ([vp, i, i, vp, vp, vp, f, vp], i),
        "lbm_init_ce_f64": ([vp, i, i, vp, vp, vp, d, vp], i),
        "lbm_moments": ([vp, i, i, vp, vp, vp, ctypes.POINTER(LbmTgv), vp, vp, sz, vp], i),
        "lbm_restrict": ([vp, i, i, i, d, d, i, i, vp, vp], i),
        "lbm_copy": ([vp, vp, sz, vp], i),
        "gnn_gelu_rate": ([vp, i, i, vp], i),
        "gnn_param_count": ([i], sz),
        "gnn_blob_len": ([i], sz),
        "lbm_step_gnn": ([vp, vp, i, i, f, vp, i, ctypes.POINTER(LbmFallback), vp, sz, vp], i),
        "lbm_step_gnn_noalloc": ([vp, vp, i, i, f, vp, i, ctypes.POINTER(LbmFallback), vp], i),
        "gnn_forward": ([vp, vp, i, i, i, vp, vp, i, vp, vp, sz, vp, sz, vp], i),
        "gnn_backward": ([vp, vp, vp, i, i, i, vp, vp, i, vp, vp, sz, vp], i),
        "gnn_mse": ([vp, vp, i, i, i, d, vp, vp, vp, sz, vp], i),
        "gnn_mse_weighted": ([vp, vp, i, i, i, ctypes.POINTER(ctypes.c_double), d, vp, vp, vp,
                              sz, vp], i),
        "gnn_adam": ([vp, vp, vp, vp, sz, f, f, f, f, i, vp], i),
        "lbm_step_simple": ([vp, vp, i, i, f, vp, ctypes.POINTER(LbmFallback), vp, sz, vp], i),
        "lbm_step_simple_channel": ([vp, vp, i, i, f, f, vp, ctypes.POINTER(LbmFallback), vp, sz,
                                     vp], i),
        "simple_forward": ([vp, vp, i, i, i, vp, vp, vp, vp, sz, vp, sz, vp], i),
        "lbm_workspace_bytes": ([i, i, i, i, i], sz),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(rc: int, what: str) -> None:
    if rc != 0:
        msg = load().lbm_last_error().decode(errors="replace")
        raise LbmError(f"{what} failed ({rc}): {msg}")
