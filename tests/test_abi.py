"""The C-ABI library loads and exports every symbol include/lbmgnn.h declares
(no GPU: nothing is computed)."""
import ctypes
import os
import re

from paper_2504_14494_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EINVAL = -1   # LBM_EINVAL in lbmgnn.h


def _declared():
    text = open(os.path.join(ROOT, "include", "lbmgnn.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"^\s*(?:const\s+)?(?:int|size_t|char|void)\s*\**\s*(\w+)\s*\(",
                          text, flags=re.M))


def test_header_lists_the_boundary():
    names = _declared()
    for n in ("lbm_init", "lbm_step_bgk", "lbm_step_gnn", "gnn_forward", "gnn_backward",
              "lbm_moments"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(_lib.EXPORTS) == names


def test_host_side_queries_need_no_gpu():
    L = _lib.load()
    assert L.gnn_param_count(2) == 38922
    assert L.gnn_blob_len(2) == 38922 + 25
    assert L.lbm_workspace_bytes(_lib.LBM_WS_MOMENTS, 1, 64, 64, 0) == 16 * 8 * 8
    assert L.lbm_workspace_bytes(99, 1, 64, 64, 0) == 0
    assert L.lbm_last_error() is not None


def test_channel_step_rejects_bad_arguments_before_any_device_work():
    L = _lib.load()
    a = ctypes.create_string_buffer(9 * 4 * 4 * 8)
    b = ctypes.create_string_buffer(9 * 4 * 4 * 8)
    pa, pb = ctypes.addressof(a), ctypes.addressof(b)
    assert L.lbm_step_channel(None, pb, 4, 4, 0.8, 1e-6, None) == EINVAL
    assert L.lbm_step_channel(pa, pb, 0, 4, 0.8, 1e-6, None) == EINVAL
    assert L.lbm_step_channel(pa, pb, 4, 4, 0.5, 1e-6, None) == EINVAL
    assert b"tau" in L.lbm_last_error()
    assert L.lbm_step_channel(pa, pa, 4, 4, 0.8, 1e-6, None) == EINVAL
    assert b"overlap" in L.lbm_last_error()
    assert L.lbm_step_channel_f64(pa, pb, 4, 4, 0.3, 0.0, None) == EINVAL
    assert L.lbm_channel_profile(pa, 4, 4, 0.0, None, None) == EINVAL
