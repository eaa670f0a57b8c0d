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


EWORKSPACE = -2   # LBM_EWORKSPACE


def test_every_entry_point_rejects_bad_arguments_before_device_work():
    """The documented error codes, returned before anything touches a GPU
    (host buffers stand in for device pointers and are never read)."""
    L = _lib.load()
    bufs = [ctypes.create_string_buffer(4096) for _ in range(6)]
    p = [ctypes.addressof(b) for b in bufs]
    a, b, c, d, e, f = p
    cases = [
        ("lbm_init", (None, 4, 4, b, c, d, None), EINVAL),
        ("lbm_init_f64", (a, 0, 4, b, c, d, None), EINVAL),
        ("lbm_init_ce", (a, 4, 4, b, c, d, 0.0, None), EINVAL),
        ("lbm_step_bgk", (a, a, 4, 4, 0.8, None), EINVAL),
        ("lbm_step_bgk", (a, b, 4, 4, 0.0, None), EINVAL),
        ("lbm_step_bgk_f64", (a, b, 4, -1, 0.8, None), EINVAL),
        ("lbm_stream", (a, b, 4, 4, 0, None), EINVAL),
        ("lbm_moments", (a, 4, 4, None, None, None, None, b, c, 0, None), EWORKSPACE),
        ("lbm_restrict", (a, 10, 8, 4, 0.8, 0.6, 1, 0, b, None), EINVAL),
        ("lbm_copy", (a + 4, b, 16, None), EINVAL),
        ("gnn_gelu_rate", (a, 0, 10, None), EINVAL),
        ("lbm_step_gnn", (a, b, 4, 4, 0.7, c, 2, None, d, 16, None), EWORKSPACE),
        ("lbm_step_gnn", (a, b, 4, 4, -1.0, c, 2, None, d, 1 << 30, None), EINVAL),
        ("gnn_forward", (a, a, 1, 4, 4, b, c, 2, None, None, 0, d, 1 << 30, None), EINVAL),
        ("gnn_backward", (a, b, c, 1, 4, 4, d, e, -1, f, a, 1 << 30, None), EINVAL),
        ("gnn_mse", (a, b, 0, 4, 4, 1.0, c, d, e, 1 << 30, None), EINVAL),
        ("gnn_adam", (a, b, c, d, 16, 1e-3, 0.9, 0.999, 1e-8, 0, None), EINVAL),
        ("lbm_step_simple", (a, b, 4, 4, -1.0, c, None, d, 1 << 30, None), EINVAL),
        ("lbm_step_simple_channel", (a, b, 4, 4, 0.7, float("nan"), c, None, d, 1 << 30, None),
         EINVAL),
        ("lbm_step_simple_channel", (a, a, 4, 4, 0.7, 1e-4, c, None, d, 1 << 30, None), EINVAL),
        ("lbm_step_simple_channel", (a, b, 4, 4, 0.7, 1e-4, c, None, d, 16, None), EWORKSPACE),
        ("simple_forward", (a, a, 1, 4, 4, b, c, None, None, 0, d, 1 << 30, None), EINVAL),
        ("simple_forward", (a, b, 1, 4, 4, b, c, None, e, 16, d, 1 << 30, None), EWORKSPACE),
        ("lbm_step_gnn_noalloc", (a, b, 4, 4, -1.0, c, 2, None, None), EINVAL),
        ("lbm_step_gnn_noalloc", (a, b, 4, 4, 0.7, c, 0, None, None), EINVAL),
        ("lbm_step_gnn_noalloc", (a, a, 4, 4, 0.7, c, 2, None, None), EINVAL),
    ]
    for name, args, code in cases:
        rc = getattr(L, name)(*args)
        assert rc == code, (name, rc, L.lbm_last_error())
        # the thread-local message names the entry point that failed
        assert L.lbm_last_error().decode().startswith(name.split("_f64")[0]), name


def test_noalloc_step_rejects_lattices_beyond_its_static_scratch():
    """lbm_step_gnn_noalloc holds at most LBM_NOALLOC_MAX_NODES nodes; larger
    lattices are refused before any device work (the addresses below are
    never dereferenced)."""
    L = _lib.load()
    a, b, c = 1 << 40, 2 << 40, 3 << 40
    assert L.lbm_step_gnn_noalloc(a, b, 256, 256 + 1, 0.7, c, 2, None, None) == EINVAL
    assert b"static scratch" in L.lbm_last_error()
    assert L.lbm_step_gnn_noalloc(a, b, _lib.LBM_NOALLOC_MAX_NODES + 1, 1, 0.7, c, 2, None,
                                  None) == EINVAL
    text = open(os.path.join(ROOT, "include", "lbmgnn.h")).read()
    assert f"#define LBM_NOALLOC_MAX_NODES {_lib.LBM_NOALLOC_MAX_NODES}" in text
