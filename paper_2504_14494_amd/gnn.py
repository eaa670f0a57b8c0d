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
           "lbm_step_gnn_noalloc",
           "Fallback", "GnnLattice", "gnn_backward", "gnn_mse", "gnn_adam", "GnnCollide",
           "GnnMse", "gnn_mse_weighted", "simple_forward", "lbm_step_simple", "lbm_step_simple_channel",
           "gnn_gelu_rate", "collide"]


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


def lbm_step_gnn_noalloc(src: torch.Tensor, dst: torch.Tensor, tau: float, blob: torch.Tensor,
                         rounds: int = 2, fallback: Fallback = None):
    """lbm_step_gnn on the library's static scratch: no workspace, nothing
    allocated (lattices of at most LBM_NOALLOC_MAX_NODES nodes; calls on one
    GPU must not overlap)."""
    _need(src, torch.float32, "src")
    _need(dst, torch.float32, "dst")
    if src.dim() != 3 or src.shape[1] != 9 or src.shape != dst.shape:
        raise ValueError("src and dst must both be [ny, 9, nx]")
    _check_blob(blob, rounds)
    ny, nx = int(src.shape[0]), int(src.shape[2])
    fb = ctypes.byref(fallback.struct()) if fallback is not None else None
    rc = _lib.load().lbm_step_gnn_noalloc(_ptr(src), _ptr(dst), nx, ny, float(tau), _ptr(blob),
                                          rounds, fb, _stream())
    check(rc, "lbm_step_gnn_noalloc")
    return dst


def simple_forward(g_pre: torch.Tensor, tau: torch.Tensor, blob: torch.Tensor,
                   want_z: bool = False, saved: torch.Tensor = None, ws: Workspace = None):
    """The per-node (Fig. 2) corrected collision of a batch of pre-collision
    states, no streaming.  blob: zero-round layout.  With `saved` (uint8,
    saved_bytes(B, nx, ny, 0)) the activations gnn_backward(rounds=0) needs
    are kept.  Returns (g_post, z)."""
    single = g_pre.dim() == 3
    if single:
        g_pre = g_pre.unsqueeze(0)
    _need(g_pre, torch.float32, "g_pre")
    B, nx, ny = _batch_dims(g_pre)
    _need(tau, torch.float32, "tau")
    if tau.numel() != B:
        raise ValueError("tau needs one value per lattice")
    _check_blob(blob, 0)
    out = torch.empty_like(g_pre)
    z = torch.empty((B, ny, nx, 10), dtype=torch.float32, device=g_pre.device) if want_z else None
    L = _lib.load()
    buf = (ws or _ws).get(L.lbm_workspace_bytes(_lib.LBM_WS_SIMPLE, B, nx, ny, 0))
    if saved is not None:
        _need(saved, torch.uint8, "saved")
    rc = L.simple_forward(_ptr(g_pre), _ptr(out), B, nx, ny, _ptr(tau), _ptr(blob), _ptr(z),
                          _ptr(saved), 0 if saved is None else saved.numel(), _ptr(buf),
                          buf.numel(), _stream())
    check(rc, "simple_forward")
    if single:
        out = out[0]
        z = z[0] if z is not None else None
    return out, z


def collide(g_pre: torch.Tensor, tau: torch.Tensor, blob: torch.Tensor, rounds: int,
            want_z: bool = False, saved: torch.Tensor = None):
    """Corrected collision of a batch of pre-collision states with either
    network: message passing (rounds >= 1, gnn_forward) or the per-node
    network of Fig. 2 (rounds = 0, simple_forward).  Returns (g_post, z)."""
    if rounds == 0:
        return simple_forward(g_pre, tau, blob, want_z=want_z, saved=saved)
    return gnn_forward(g_pre, tau, blob, rounds, want_z=want_z, saved=saved)


def _simple_step_args(src, dst, blob, fallback, ws):
    _need(src, torch.float32, "src")
    _need(dst, torch.float32, "dst")
    if src.dim() != 3 or src.shape[1] != 9 or src.shape != dst.shape:
        raise ValueError("src and dst must both be [ny, 9, nx]")
    _check_blob(blob, 0)
    ny, nx = int(src.shape[0]), int(src.shape[2])
    buf = (ws or _ws).get(_lib.load().lbm_workspace_bytes(_lib.LBM_WS_SIMPLE, 1, nx, ny, 0))
    fb = ctypes.byref(fallback.struct()) if fallback is not None else None
    return nx, ny, fb, buf


def lbm_step_simple(src: torch.Tensor, dst: torch.Tensor, tau: float, blob: torch.Tensor,
                    fallback: Fallback = None, ws: Workspace = None):
    """One step with the per-node (Fig. 2) corrected collision fused into the
    pull step; blob: zero-round layout."""
    nx, ny, fb, buf = _simple_step_args(src, dst, blob, fallback, ws)
    rc = _lib.load().lbm_step_simple(_ptr(src), _ptr(dst), nx, ny, float(tau), _ptr(blob), fb,
                                     _ptr(buf), buf.numel(), _stream())
    check(rc, "lbm_step_simple")
    return dst


def lbm_step_simple_channel(src: torch.Tensor, dst: torch.Tensor, tau: float, gx: float,
                            blob: torch.Tensor, fallback: Fallback = None,
                            ws: Workspace = None):
    """lbm_step_simple on the forced channel (bounce-back walls below row 0
    and above row ny - 1, body force rho * gx along x)."""
    nx, ny, fb, buf = _simple_step_args(src, dst, blob, fallback, ws)
    rc = _lib.load().lbm_step_simple_channel(_ptr(src), _ptr(dst), nx, ny, float(tau),
                                             float(gx), _ptr(blob), fb, _ptr(buf), buf.numel(),
                                             _stream())
    check(rc, "lbm_step_simple_channel")
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

    def init_ce(self, rho, ux, uy, tau: float):
        super().init_ce(rho, ux, uy, tau)
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

    def _graph_buffers(self):
        fb = self.fallback
        return super()._graph_buffers() + [self.blob, self.ws.buf, fb.flags, fb.n_fallback,
                                           fb.mass]

    def _graph_key(self, gate: bool):
        """What a captured corrected step freezes besides the step's own
        arguments: the parameter blob's address, the number of rounds and,
        with the gate, the drift threshold (copied into the kernel arguments
        at capture).  Changing any of them selects another graph."""
        return (self.blob.data_ptr(), int(self.rounds),
                float(self.fallback.threshold) if gate else None)

    def step_bgk(self, tau: float, n: int = 1, graph: bool = False):
        super().step_bgk(tau, n, graph)
        if n:
            self.sync_mass()
        return self

    def step_gnn(self, tau: float, n: int = 1, gate: bool = True, graph: bool = False):
        """Corrected steps: message passing for rounds >= 1, the fused
        per-node network of Fig. 2 for rounds == 0.  With the gate, the
        fallback state is updated on the device every step, also inside a
        captured graph."""
        def step(src, dst, fb):
            if self.rounds == 0:
                lbm_step_simple(src, dst, tau, self.blob, fb, self.ws)
            else:
                lbm_step_gnn(src, dst, tau, self.blob, self.rounds, fb, self.ws)

        fb = self.fallback if gate else None

        def warm():
            # same code path on copies: the gate state of the lattice is untouched
            tmp = None
            if gate:
                tmp = Fallback(0.0, self.fallback.threshold)
                tmp.mass.copy_(self.fallback.mass)
            step(self.a.clone(), torch.empty_like(self.a), tmp)
        return self._run(("gnn", float(tau), bool(gate)) + self._graph_key(gate),
                         lambda s, d: step(s, d, fb), warm, n, graph)

    def step_gnn_channel(self, tau: float, gx: float, n: int = 1, gate: bool = True,
                         graph: bool = False):
        """Corrected steps of the per-node network (rounds == 0) on the
        forced channel; the fallback is the forced BGK channel step."""
        if self.rounds != 0:
            raise ValueError("the channel step runs the per-node network (rounds = 0): "
                             "message passing has no wall treatment")

        def step(src, dst, fb):
            lbm_step_simple_channel(src, dst, tau, gx, self.blob, fb, self.ws)

        fb = self.fallback if gate else None

        def warm():
            tmp = None
            if gate:
                tmp = Fallback(0.0, self.fallback.threshold)
                tmp.mass.copy_(self.fallback.mass)
            step(self.a.clone(), torch.empty_like(self.a), tmp)
        return self._run(("gnn_channel", float(tau), float(gx), bool(gate)) + self._graph_key(gate),
                         lambda s, d: step(s, d, fb), warm, n, graph)


def backward_ws_bytes(batch: int, nx: int, ny: int, rounds: int = 2) -> int:
    return int(_lib.load().lbm_workspace_bytes(_lib.LBM_WS_GNN_BACKWARD, batch, nx, ny, rounds))


def gnn_backward(dL_dgpost: torch.Tensor, g_pre: torch.Tensor, saved: torch.Tensor,
                 tau: torch.Tensor, blob: torch.Tensor, rounds: int = 2,
                 grad: torch.Tensor = None, ws: Workspace = None) -> torch.Tensor:
    """dL/dparams (FP32, [gnn_param_count]) of the forward call that filled
    `saved` (same g_pre, tau, blob), given dL/dg_post: gnn_forward for
    rounds >= 1, simple_forward for rounds = 0."""
    if g_pre.dim() == 3:
        g_pre, dL_dgpost = g_pre.unsqueeze(0), dL_dgpost.unsqueeze(0)
    _need(g_pre, torch.float32, "g_pre")
    _need(dL_dgpost, torch.float32, "dL_dgpost")
    _need(saved, torch.uint8, "saved")
    B, nx, ny = _batch_dims(g_pre)
    if dL_dgpost.shape != g_pre.shape:
        raise ValueError("dL_dgpost must match g_pre")
    _check_blob(blob, rounds)
    if grad is None:
        grad = torch.empty(gnn_param_count(rounds), dtype=torch.float32, device=g_pre.device)
    _need(grad, torch.float32, "grad")
    buf = (ws or _ws_bwd).get(backward_ws_bytes(B, nx, ny, rounds))
    rc = _lib.load().gnn_backward(_ptr(dL_dgpost), _ptr(g_pre), _ptr(saved), B, nx, ny,
                                  _ptr(tau), _ptr(blob), rounds, _ptr(grad), _ptr(buf),
                                  buf.numel(), _stream())
    check(rc, "gnn_backward")
    return grad


_ws_bwd = Workspace()


def gnn_mse(a: torch.Tensor, b: torch.Tensor, scale: float = 1.0, want_grad: bool = True,
            ws: Workspace = None):
    """Eq. 4 over all nodes of a batch: scale / N * sum (a - b)^2, N = number
    of nodes.  Returns (loss as a device float64 [1], dloss/da or None)."""
    _need(a, torch.float32, "a")
    _need(b, torch.float32, "b")
    if a.shape != b.shape or a.numel() % 9:
        raise ValueError("a and b must be populations of the same shape")
    nodes = a.numel() // 9
    loss = torch.empty(1, dtype=torch.float64, device=a.device)
    grad = torch.empty_like(a) if want_grad else None
    L = _lib.load()
    buf = (ws or _ws).get(L.lbm_workspace_bytes(_lib.LBM_WS_MSE, 1, nodes, 1, 0))
    rc = L.gnn_mse(_ptr(a), _ptr(b), 1, nodes, 1, float(scale), _ptr(loss), _ptr(grad),
                   _ptr(buf), buf.numel(), _stream())
    check(rc, "gnn_mse")
    return loss, grad


def gnn_mse_weighted(a: torch.Tensor, b: torch.Tensor, q, scale: float = 1.0,
                     want_grad: bool = True, ws: Workspace = None):
    """Eq. 4 with each node's residual weighted by the symmetric 9 x 9 matrix
    q (host array-like): scale / N * sum over nodes of r^T q r.  a, b:
    populations [ny, 9, nx] or [batch, ny, 9, nx].  Returns (loss as a
    device float64 [1], dloss/da or None)."""
    _need(a, torch.float32, "a")
    _need(b, torch.float32, "b")
    if a.shape != b.shape:
        raise ValueError("a and b must be populations of the same shape")
    B, nx, ny = _batch_dims(a if a.dim() == 4 else a.unsqueeze(0))
    qd = (ctypes.c_double * 81)(*[float(v) for row in q for v in row])
    loss = torch.empty(1, dtype=torch.float64, device=a.device)
    grad = torch.empty_like(a) if want_grad else None
    L = _lib.load()
    buf = (ws or _ws).get(L.lbm_workspace_bytes(_lib.LBM_WS_MSE, B, nx, ny, 0))
    rc = L.gnn_mse_weighted(_ptr(a), _ptr(b), B, nx, ny, qd, float(scale), _ptr(loss),
                            _ptr(grad), _ptr(buf), buf.numel(), _stream())
    check(rc, "gnn_mse_weighted")
    return loss, grad


def gnn_adam(params: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor,
             step: int, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8):
    """One in-place Adam step on the first grad.numel() entries of params."""
    n = grad.numel()
    for t, nm in ((params, "params"), (grad, "grad"), (m, "m"), (v, "v")):
        _need(t, torch.float32, nm)
    if params.numel() < n or m.numel() < n or v.numel() < n:
        raise ValueError("params, m and v must hold at least grad.numel() values")
    rc = _lib.load().gnn_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), n, float(lr),
                              float(beta1), float(beta2), float(eps), int(step), _stream())
    check(rc, "gnn_adam")


class GnnCollide(torch.autograd.Function):
    """torch.autograd face of the corrected collision: forward = gnn_forward
    (rounds >= 1) or simple_forward (rounds = 0, the Fig. 2 network), with the
    activations saved; backward = gnn_backward (gradient with respect to the
    parameter blob only; populations and tau are data)."""

    @staticmethod
    def forward(ctx, blob, g_pre, tau, rounds):
        B, nx, ny = _batch_dims(g_pre)
        saved = torch.empty(saved_bytes(B, nx, ny, rounds), dtype=torch.uint8,
                            device=g_pre.device)
        if rounds == 0:
            out, _ = simple_forward(g_pre, tau, blob.detach(), saved=saved)
        else:
            out, _ = gnn_forward(g_pre, tau, blob.detach(), rounds, saved=saved)
        ctx.save_for_backward(blob, g_pre, tau)
        ctx.saved_acts = saved
        ctx.rounds = rounds
        return out

    @staticmethod
    def backward(ctx, grad_out):
        blob, g_pre, tau = ctx.saved_tensors
        gp = gnn_backward(grad_out.contiguous(), g_pre, ctx.saved_acts, tau, blob.detach(),
                          ctx.rounds)
        full = torch.zeros_like(blob)
        full[:gp.numel()] = gp
        ctx.saved_acts = None
        return full, None, None, None


class GnnMse(torch.autograd.Function):
    """Eq. 4 (scaled) with its gradient from the gnn_mse kernel."""

    @staticmethod
    def forward(ctx, a, b, scale):
        loss, grad = gnn_mse(a.detach(), b, scale, want_grad=True)
        ctx.save_for_backward(grad)
        return loss.to(torch.float32).reshape(())

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        return grad * gout, None, None


def gnn_gelu_rate(out: torch.Tensor, iters: int):
    """Runs the GELU throughput kernel: 8 * out.numel() * iters GELUs, with
    one value per thread written to `out` (a multiple of 256 floats)."""
    _need(out, torch.float32, "out")
    if out.numel() % 256 or out.numel() == 0:
        raise ValueError("out must hold a positive multiple of 256 floats")
    check(_lib.load().gnn_gelu_rate(_ptr(out), out.numel() // 256, int(iters), _stream()),
          "gnn_gelu_rate")
    return out
