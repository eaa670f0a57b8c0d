"""Python face of the GNN entry points of liblbmgnn.so.

Argument marshalling only: torch supplies device memory and the current
stream, every computation runs in the HIP library.  Populations are shifted
row-interleaved tensors, [ny, 9, nx] for one lattice or [batch, ny, 9, nx]
for a batch of independent periodic lattices.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import LbmFallback, check
from .lbm import Lattice, Workspace, _need, _ptr, _stream, lbm_moments

__all__ = ["gnn_param_count", "gnn_blob_len", "saved_bytes", "gnn_forward", "lbm_step_gnn",
           "Fallback", "GnnLattice"]


def gnn_param_count(rounds: int = 2) -> int:
    return int(_lib.load().gnn_param_count(rounds))


def gnn_blob_len(rounds: int = 2) -> int:
    return int(_lib.load().gnn_blob_len(rounds))


def saved_bytes(batch: int, nx: int, ny: int, rounds: int = 2) -> int:
    return int(_lib.load().lbm_workspace_bytes(_lib.LBM_WS_GNN_SAVED, batch, nx, ny, rounds))


def _batch_dims(g: torch.Tensor):
    if g.dim() != 4 or g.shape[2] != 9:
        raise ValueError(f"batched populations must be [batch, ny, 9, nx], got {tuple(g.shape)}")
    return int(g.shape[0]), int(g.shape[3]), int(g.shape[1])


_ws = Workspace()


def _check_blob(blob: torch.Tensor, rounds: int):
    _need(blob, torch.float32, "params")
    if blob.numel() != gnn_blob_len(rounds):
        raise ValueError(f"params must hold {gnn_blob_len(rounds)} floats, got {blob.numel()}")


def gnn_forward(g_pre: torch.Tensor, tau: torch.Tensor, blob: torch.Tensor, rounds: int = 2,
                want_z: bool = False, saved: torch.Tensor = None, out: torch.Tensor = None,
                ws: Workspace = None):
    """GNN-corrected collision of a batch of pre-collision states (no
    streaming).  Returns (g_post, z or None)."""
    single = g_pre.dim() == 3
    if single:
        g_pre = g_pre.unsqueeze(0)
    _need(g_pre, torch.float32, "g_pre")
    B, nx, ny = _batch_dims(g_pre)
    _need(tau, torch.float32, "tau")
    if tau.numel() != B:
        raise ValueError("tau needs one value per lattice")
    _check_blob(blob, rounds)
    if out is None:
        out = torch.empty_like(g_pre)
    else:
        out = out.view_as(g_pre)
    _need(out, torch.float32, "g_post")
    z = torch.empty((B, ny, nx, 10), dtype=torch.float32, device=g_pre.device) if want_z else None
    if saved is not None:
        _need(saved, torch.uint8, "saved")
    L = _lib.load()
    wsb = L.lbm_workspace_bytes(_lib.LBM_WS_GNN_FORWARD, B, nx, ny, rounds)
    buf = (ws or _ws).get(wsb)
    rc = L.gnn_forward(_ptr(g_pre), _ptr(out), B, nx, ny, _ptr(tau), _ptr(blob), rounds,
                       _ptr(z), _ptr(saved), 0 if saved is None else saved.numel(),
                       _ptr(buf), buf.numel(), _stream())
    check(rc, "gnn_forward")
    if single:
        out = out[0]
        z = z[0] if z is not None else None
    return out, z


class Fallback:
    """Device state of the per-step fallback gate: sticky flag bits, number
    of steps that fell back, and the FP64 total mass of the current state."""

    def __init__(self, mass: float, threshold: float = 1e-6, device="cuda"):
        self.threshold = float(threshold)
        self.flags = torch.zeros(1, dtype=torch.int32, device=device)
        self.n_fallback = torch.zeros(1, dtype=torch.int32, device=device)
        self.mass = torch.full((1,), float(mass), dtype=torch.float64, device=device)

    def struct(self):
        return LbmFallback(self.threshold, self.flags.data_ptr(), self.n_fallback.data_ptr(),
                           self.mass.data_ptr())


def lbm_step_gnn(src: torch.Tensor, dst: torch.Tensor, tau: float, blob: torch.Tensor,
                 rounds: int = 2, fallback: Fallback = None, ws: Workspace = None):
    _need(src, torch.float32, "src")
    _need(dst, torch.float32, "dst")
    if src.dim() != 3 or src.shape[1] != 9 or src.shape != dst.shape:
        raise ValueError("src and dst must both be [ny, 9, nx]")
    _check_blob(blob, rounds)
    ny, nx = int(src.shape[0]), int(src.shape[2])
    L = _lib.load()
    wsb = L.lbm_workspace_bytes(_lib.LBM_WS_GNN_STEP, 1, nx, ny, rounds)
    buf = (ws or _ws).get(wsb)
    fb = ctypes.byref(fallback.struct()) if fallback is not None else None
    rc = L.lbm_step_gnn(_ptr(src), _ptr(dst), nx, ny, float(tau), _ptr(blob), rounds, fb,
                        _ptr(buf), buf.numel(), _stream())
    check(rc, "lbm_step_gnn")
    return dst


class GnnLattice(Lattice):
    """A/B buffers of one periodic lattice stepped with the plain BGK or the
    GNN-corrected collision, with the per-step fallback gate."""

    def __init__(self, nx: int, ny: int, blob: torch.Tensor, rounds: int = 2,
                 threshold: float = 1e-6, device="cuda"):
        super().__init__(nx, ny, torch.float32, device)
        self.blob, self.rounds = blob, rounds
        self.ws = Workspace()
        self.fallback = Fallback(float(nx * ny), threshold, device)

    @property
    def n_fallback(self):
        return self.fallback.n_fallback

    def init(self, rho, ux, uy):
        super().init(rho, ux, uy)
        self.sync_mass()
        return self

    def load(self, g):
        super().load(g)
        self.sync_mass()
        return self

    def sync_mass(self):
        """Reference mass of the gate := FP64 mass of the current state."""
        _, _, _, sums = lbm_moments(self.a, ws=self.ws)
        self.fallback.mass.copy_(sums[0:1])

    def step_bgk(self, tau: float, n: int = 1):
        super().step_bgk(tau, n)
        if n:
            self.sync_mass()
        return self

    def step_gnn(self, tau: float, n: int = 1, gate: bool = True):
        for _ in range(n):
            lbm_step_gnn(self.a, self.b, tau, self.blob, self.rounds,
                         self.fallback if gate else None, self.ws)
            self.a, self.b = self.b, self.a
            self.steps += 1
        return self
