"""Python face of the C ABI: torch tensors in, raw device pointers out.

Functions keep the C names (lbm_init, lbm_step_bgk, ...).  PyTorch supplies
device memory and the current HIP stream; all arithmetic runs in
liblbmgnn.so.  Populations are shifted (g = f - w) row-interleaved tensors
shaped [ny, 9, nx] (or [batch, ny, 9, nx]): for each lattice row, nine
contiguous runs of nx values, one per direction.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import LbmFallback, LbmTgv, check

__all__ = [
    "lbm_init", "lbm_init_ce", "lbm_step_bgk", "lbm_stream", "lbm_moments", "lbm_restrict", "lbm_copy",
    "lbm_step_channel", "lbm_channel_profile",
    "lbm_workspace_bytes", "Workspace", "Lattice",
]


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, what: str):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


def _pop_dims(g: torch.Tensor):
    if g.dim() != 3 or g.shape[1] != 9:
        raise ValueError(f"populations must be [ny, 9, nx], got {tuple(g.shape)}")
    return int(g.shape[2]), int(g.shape[0])


def lbm_workspace_bytes(op: int, batch: int, nx: int, ny: int, n_rounds: int = 0) -> int:
    return int(_lib.load().lbm_workspace_bytes(op, batch, nx, ny, n_rounds))


class Workspace:
    """Grows-only byte buffer on the current device, reused across calls."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int) -> torch.Tensor:
        nbytes = max(int(nbytes), 256)
        if self.buf is None or self.buf.numel() < nbytes or not self.buf.is_cuda:
            self.buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        return self.buf


_ws = Workspace()


def lbm_init(g: torch.Tensor, rho: torch.Tensor, ux: torch.Tensor, uy: torch.Tensor):
    dt = g.dtype
    for t, n in ((g, "g"), (rho, "rho"), (ux, "ux"), (uy, "uy")):
        _need(t, dt, n)
    nx, ny = _pop_dims(g)
    for t in (rho, ux, uy):
        if tuple(t.shape) != (ny, nx):
            raise ValueError("fields must be [ny, nx]")
    fn = _lib.load().lbm_init if dt == torch.float32 else _lib.load().lbm_init_f64
    check(fn(_ptr(g), nx, ny, _ptr(rho), _ptr(ux), _ptr(uy), _stream()), "lbm_init")
    return g


def lbm_init_ce(g: torch.Tensor, rho: torch.Tensor, ux: torch.Tensor, uy: torch.Tensor,
                tau: float):
    """Equilibrium plus first-order Chapman-Enskog non-equilibrium."""
    dt = g.dtype
    for t, n in ((g, "g"), (rho, "rho"), (ux, "ux"), (uy, "uy")):
        _need(t, dt, n)
    nx, ny = _pop_dims(g)
    for t in (rho, ux, uy):
        if tuple(t.shape) != (ny, nx):
            raise ValueError("fields must be [ny, nx]")
    fn = _lib.load().lbm_init_ce if dt == torch.float32 else _lib.load().lbm_init_ce_f64
    check(fn(_ptr(g), nx, ny, _ptr(rho), _ptr(ux), _ptr(uy), float(tau), _stream()),
          "lbm_init_ce")
    return g


def lbm_step_bgk(src: torch.Tensor, dst: torch.Tensor, tau: float):
    _need(src, src.dtype, "src")
    _need(dst, src.dtype, "dst")
    nx, ny = _pop_dims(src)
    if src.shape != dst.shape:
        raise ValueError("src and dst shapes differ")
    if src.dtype == torch.float32:
        rc = _lib.load().lbm_step_bgk(_ptr(src), _ptr(dst), nx, ny, float(tau), _stream())
    elif src.dtype == torch.float64:
        rc = _lib.load().lbm_step_bgk_f64(_ptr(src), _ptr(dst), nx, ny, float(tau), _stream())
    else:
        raise TypeError("populations must be float32 or float64")
    check(rc, "lbm_step_bgk")
    return dst


def lbm_step_channel(src: torch.Tensor, dst: torch.Tensor, tau: float, gx: float):
    """One step of the forced channel (walls at y = -1/2 and ny - 1/2,
    periodic in x, body force rho * gx along x)."""
    _need(src, src.dtype, "src")
    _need(dst, src.dtype, "dst")
    nx, ny = _pop_dims(src)
    if src.shape != dst.shape:
        raise ValueError("src and dst shapes differ")
    if src.dtype == torch.float32:
        rc = _lib.load().lbm_step_channel(_ptr(src), _ptr(dst), nx, ny, float(tau), float(gx),
                                          _stream())
    elif src.dtype == torch.float64:
        rc = _lib.load().lbm_step_channel_f64(_ptr(src), _ptr(dst), nx, ny, float(tau),
                                              float(gx), _stream())
    else:
        raise TypeError("populations must be float32 or float64")
    check(rc, "lbm_step_channel")
    return dst


def lbm_channel_profile(g: torch.Tensor, gx: float) -> torch.Tensor:
    """x-averaged fluid velocity u_x(y) of a channel state as
    lbm_step_channel leaves it (post-collision), FP64 [ny]."""
    _need(g, torch.float32, "g")
    nx, ny = _pop_dims(g)
    prof = torch.empty(ny, dtype=torch.float64, device=g.device)
    check(_lib.load().lbm_channel_profile(_ptr(g), nx, ny, float(gx), _ptr(prof), _stream()),
          "lbm_channel_profile")
    return prof


def lbm_stream(src: torch.Tensor, dst: torch.Tensor = None):
    """Streaming only: dst_i(x) = src_i(x - e_i) for [ny, 9, nx] or
    [batch, ny, 9, nx] FP32 populations."""
    _need(src, torch.float32, "src")
    if dst is None:
        dst = torch.empty_like(src)
    _need(dst, torch.float32, "dst")
    if src.shape != dst.shape:
        raise ValueError("src and dst shapes differ")
    if src.dim() == 4:
        batch, (nx, ny) = int(src.shape[0]), _pop_dims(src[0])
    else:
        batch, (nx, ny) = 1, _pop_dims(src)
    check(_lib.load().lbm_stream(_ptr(src), _ptr(dst), nx, ny, batch, _stream()), "lbm_stream")
    return dst


def lbm_moments(g: torch.Tensor, analytic=None, fields: bool = False, sums: bool = True,
                ws: Workspace = None):
    """Returns (rho, ux, uy, sums) — fields are None unless requested; sums is a
    device float64 tensor [8] (see lbmgnn.h) or None."""
    _need(g, torch.float32, "g")
    nx, ny = _pop_dims(g)
    rho = ux = uy = None
    if fields:
        rho, ux, uy = (torch.empty((ny, nx), dtype=torch.float32, device=g.device)
                       for _ in range(3))
    out = torch.empty(8, dtype=torch.float64, device=g.device) if sums else None
    wsb = lbm_workspace_bytes(_lib.LBM_WS_MOMENTS, 1, nx, ny)
    buf = (ws or _ws).get(wsb)
    tgv = None
    if analytic is not None:
        tgv = ctypes.byref(LbmTgv(*[float(v) for v in analytic]))
    rc = _lib.load().lbm_moments(_ptr(g), nx, ny, _ptr(rho), _ptr(ux), _ptr(uy), tgv,
                                 _ptr(out), _ptr(buf), buf.numel(), _stream())
    check(rc, "lbm_moments")
    return rho, ux, uy, out


def lbm_restrict(g_fine: torch.Tensor, factor: int, tau_f: float, tau_c: float,
                 pull: bool, unstream: bool, out: torch.Tensor = None):
    _need(g_fine, torch.float64, "g_fine")
    nxf, nyf = _pop_dims(g_fine)
    if out is None:
        out = torch.empty((nyf // factor, 9, nxf // factor), dtype=torch.float32,
                          device=g_fine.device)
    _need(out, torch.float32, "out")
    rc = _lib.load().lbm_restrict(_ptr(g_fine), nxf, nyf, factor, float(tau_f), float(tau_c),
                                  int(pull), int(unstream), _ptr(out), _stream())
    check(rc, "lbm_restrict")
    return out


def lbm_copy(src: torch.Tensor, dst: torch.Tensor):
    _need(src, torch.float32, "src")
    _need(dst, torch.float32, "dst")
    check(_lib.load().lbm_copy(_ptr(src), _ptr(dst), src.numel(), _stream()), "lbm_copy")
    return dst


class Lattice:
    """A/B population buffers of one periodic D2Q9 lattice on the GPU.

    Stepping methods take `graph=True` to run whole chunks of steps as one
    captured HIP graph (torch.cuda.CUDAGraph over the library's launches on
    the current stream), which removes the per-launch host cost that
    dominates small lattices.  The graph holds the buffer addresses, so one
    is captured per (step kind, parameters, buffer holding the state) and
    replayed; results are bitwise those of the eager steps."""

    GRAPH_CHUNK = 64   # steps per captured graph (even: the state returns to `a`)

    def __init__(self, nx: int, ny: int, dtype=torch.float32, device="cuda"):
        self.nx, self.ny = nx, ny
        self.a = torch.empty((ny, 9, nx), dtype=dtype, device=device)
        self.b = torch.empty_like(self.a)
        self.steps = 0
        self._graphs = {}

    def _capture(self, one_step, warmup):
        """HIP graph of GRAPH_CHUNK steps from self.a, ping-ponging with
        self.b.  `warmup()` runs one step on scratch copies first, on the
        side stream, so that library state and workspaces exist before the
        capture and the lattice itself does not advance."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            warmup()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            src, dst = self.a, self.b
            for _ in range(self.GRAPH_CHUNK):
                one_step(src, dst)
                src, dst = dst, src
        return g

    def _graph_buffers(self):
        """Device buffers a captured step reads or writes; the graph keeps
        them alive, so a later reallocation elsewhere (a grown workspace)
        cannot leave it pointing at freed memory."""
        return [self.a, self.b]

    def _run(self, key, one_step, warmup, n: int, graph: bool):
        """n steps: whole chunks from a captured graph when `graph`, the rest
        eagerly (one_step(src, dst) advances src into dst)."""
        if graph and n >= self.GRAPH_CHUNK:
            k = (key, self.a.data_ptr())
            if k not in self._graphs:
                g = self._capture(one_step, warmup)
                self._graphs[k] = (g, list(self._graph_buffers()))
            g = self._graphs[k][0]
            for _ in range(n // self.GRAPH_CHUNK):
                g.replay()
            self.steps += (n // self.GRAPH_CHUNK) * self.GRAPH_CHUNK
            n %= self.GRAPH_CHUNK
        for _ in range(n):
            one_step(self.a, self.b)
            self.a, self.b = self.b, self.a
            self.steps += 1
        return self

    @property
    def g(self) -> torch.Tensor:
        return self.a

    def init(self, rho, ux, uy):
        dt, dev = self.a.dtype, self.a.device
        lbm_init(self.a, *(torch.as_tensor(t, dtype=dt, device=dev).contiguous()
                           for t in (rho, ux, uy)))
        self.steps = 0
        return self

    def init_ce(self, rho, ux, uy, tau: float):
        """Start on the slow manifold (equilibrium + Chapman-Enskog term)."""
        dt, dev = self.a.dtype, self.a.device
        lbm_init_ce(self.a, *(torch.as_tensor(t, dtype=dt, device=dev).contiguous()
                              for t in (rho, ux, uy)), tau)
        self.steps = 0
        return self

    def load(self, g):
        self.a.copy_(torch.as_tensor(g, dtype=self.a.dtype))
        return self

    def step_bgk(self, tau: float, n: int = 1, graph: bool = False):
        def one(src, dst):
            lbm_step_bgk(src, dst, tau)

        def warm():
            one(self.a.clone(), torch.empty_like(self.a))
        return self._run(("bgk", float(tau)), one, warm, n, graph)

    def step_channel(self, tau: float, gx: float, n: int = 1, graph: bool = False):
        def one(src, dst):
            lbm_step_channel(src, dst, tau, gx)

        def warm():
            one(self.a.clone(), torch.empty_like(self.a))
        return self._run(("channel", float(tau), float(gx)), one, warm, n, graph)

    def moments(self, analytic=None, fields=False):
        return lbm_moments(self.a, analytic, fields)
