"""The allocation-free corrected step, lbm_step_gnn_noalloc (for callers that
cannot allocate device memory), called through the C ABI and compared with
the workspace entry point lbm_step_gnn on the same inputs.

Both run the same kernels, so the outputs, gate flags, fallback counts and
recorded masses must agree value for value.  Calls follow one another on one
GPU, each on a smaller lattice than the one before, so the static scratch
still holds the previous call's larger contents when the next call starts."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2504_14494_amd import _lib, gnn, inputs

pytestmark = pytest.mark.gpu

R = 2
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)[:, None, None]


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _noalloc(src, dst, tau, blob, fb):
    ny, nx = int(src.shape[0]), int(src.shape[2])
    fbs = ctypes.byref(fb.struct()) if fb is not None else None
    return _lib.load().lbm_step_gnn_noalloc(_vp(src), _vp(dst), nx, ny, tau, _vp(blob), R, fbs,
                                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


# (ny, nx), seed, drift threshold (negative forces the fallback), gate on
CASES = [((256, 256), 1, 1e-6, True),    # the largest lattice the static scratch holds
         ((96, 130), 2, -1.0, True),     # smaller, ragged tiles, forced fallback
         ((40, 56), 3, 1e-6, False),     # smaller still, no gate
         ((5, 7), 4, 1e-6, True)]        # a lattice smaller than one tile


def test_noalloc_step_equals_the_workspace_step_call_after_call():
    # the inference correction scale: no population goes negative, so only
    # the forced case falls back
    blob = torch.as_tensor(inputs.gnn_blob(21, R, s_delta=1e-4), device="cuda")
    for (ny, nx), seed, thr, gate in CASES:
        print(f"lbm_step_gnn_noalloc {ny}x{nx} seed {seed} threshold {thr} gate {gate}",
              flush=True)
        post = inputs.random_shifted_state((9, ny, nx), 3e-3, seed=seed)
        src = torch.as_tensor(inputs.planes_to_rows(post), device="cuda")
        mass0 = float((post.astype(np.float64) + W).sum())
        fa = gnn.Fallback(mass0, thr) if gate else None
        fb = gnn.Fallback(mass0, thr) if gate else None
        a = torch.full_like(src, float("nan"))
        b = torch.full_like(src, float("nan"))
        assert _noalloc(src, a, 0.7, blob, fa) == 0, _lib.load().lbm_last_error()
        gnn.lbm_step_gnn(src, b, 0.7, blob, R, fallback=fb)
        torch.cuda.synchronize()
        assert torch.isfinite(a).all()
        assert torch.equal(a, b), (ny, nx)
        if gate:
            assert int(fa.flags.item()) == int(fb.flags.item())
            assert int(fa.n_fallback.item()) == int(fb.n_fallback.item())
            assert fa.mass.item() == fb.mass.item()
            assert int(fa.flags.item()) == (2 if thr < 0 else 0)
            assert int(fa.n_fallback.item()) == (1 if thr < 0 else 0)


def test_noalloc_step_rejects_a_lattice_beyond_its_scratch():
    L = _lib.load()
    src = torch.zeros((257, 9, 256), device="cuda")
    dst = torch.empty_like(src)
    blob = torch.as_tensor(inputs.gnn_blob(21, R), device="cuda")
    dst.fill_(3.0)
    rc = _noalloc(src, dst, 0.7, blob, None)
    torch.cuda.synchronize()
    assert rc == -1                                   # LBM_EINVAL
    assert b"static scratch" in L.lbm_last_error()
    assert bool((dst == 3.0).all())                   # nothing was enqueued
