"""Plain FP64 CPU oracle for LBM-GNN (arXiv 2504.14494) — test infrastructure.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (built from
``lbm_oracle.c`` and ``gnn_oracle.c`` with plain gcc) through ctypes and
shares no code with the HIP library.

Population arrays are float64 numpy arrays laid out ``[9, ny, nx]`` (one
lattice) or ``[batch, 9, ny, nx]``; they hold the unshifted ``f_i``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "lbm_oracle.c"), os.path.join(_HERE, "gnn_oracle.c")]
LIB_PATH = os.path.join(_HERE, "liboracle.so")

HID = 64
NFEAT = 12
NOUT = 10


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, so IEEE FP64 holds)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
               "-D_GNU_SOURCE", "-shared", "-fPIC", *_SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        d, i, sz = ctypes.c_double, ctypes.c_int, ctypes.c_size_t
        pd, pi = P(ctypes.c_double), P(ctypes.c_int)
        L.orc_set_threads.argtypes = [i]
        L.orc_lattice.argtypes = [pi, pi, pd]
        L.orc_equilibrium.argtypes = [d, d, d, pd]
        L.orc_moments.argtypes = [pd, i, i, pd, pd, pd]
        L.orc_init_equilibrium.argtypes = [pd, i, i, pd, pd, pd]
        L.orc_init_ce.argtypes = [pd, i, i, pd, pd, pd, d]
        L.orc_collide_bgk.argtypes = [pd, pd, i, i, d]
        L.orc_stream.argtypes = [pd, pd, i, i]
        L.orc_unstream.argtypes = [pd, pd, i, i]
        L.orc_bgk_step.argtypes = [pd, pd, i, i, d]
        L.orc_bgk_run.argtypes = [pd, i, i, d, i]
        L.orc_collide_forced.argtypes = [pd, pd, i, i, d, d]
        L.orc_stream_channel.argtypes = [pd, pd, i, i]
        L.orc_channel_run.argtypes = [pd, i, i, d, d, i]
        L.orc_observables.argtypes = [pd, i, i, pd, pd]
        L.orc_restrict.argtypes = [pd, i, i, i, d, d, i, pd]
        L.orc_bf16_round.argtypes = [d]
        L.orc_bf16_round.restype = d
        L.orc_gelu.argtypes = [d]
        L.orc_gelu.restype = d
        L.orc_gelu_grad.argtypes = [d]
        L.orc_gelu_grad.restype = d
        L.orc_gnn_param_count.argtypes = [i]
        L.orc_gnn_param_count.restype = sz
        L.orc_gnn_blob_len.argtypes = [i]
        L.orc_gnn_blob_len.restype = sz
        L.orc_project.argtypes = [pd, pd]
        L.orc_gnn_collide.argtypes = [pd, pd, i, i, i, pd, pd, i, i, pd]
        L.orc_gnn_collide.restype = i
        L.orc_gnn_collide_act.argtypes = [pd, pd, i, i, i, pd, pd, i, i, i, pd]
        L.orc_gnn_collide_act.restype = i
        L.orc_gnn_collide_forced.argtypes = [pd, pd, i, i, i, pd, pd, i, i, i, d, pd]
        L.orc_gnn_collide_forced.restype = i
        L.orc_gnn_backward_act.argtypes = [pd, pd, i, i, i, pd, pd, i, i, i, pd]
        L.orc_gnn_backward_act.restype = i
        L.orc_gnn_collide_nodes.argtypes = [pd, i, i, d, pd, i, i,
                                            P(ctypes.c_long), i, pd, pd]
        L.orc_gnn_collide_nodes.restype = i
        L.orc_gnn_backward.argtypes = [pd, pd, i, i, i, pd, pd, i, i, pd]
        L.orc_gnn_backward.restype = i
        L.orc_gnn_collide_gated.argtypes = [pd, pd, i, i, d, pd, i, i, d, d,
                                            P(ctypes.c_uint), pd]
        L.orc_gnn_collide_gated.restype = i
        L.orc_mse.argtypes = [pd, pd, sz]
        L.orc_mse.restype = d
        L.orc_mse_weighted.argtypes = [pd, pd, sz, pd]
        L.orc_mse_weighted.restype = d
        L.orc_adam.argtypes = [pd, pd, pd, pd, sz, d, d, d, d, i]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- lattice ---

def set_threads(n: int) -> None:
    """Threads the BGK collision and streaming loops may share their nodes
    among (default 1); results do not depend on it."""
    lib().orc_set_threads(int(n))


def lattice():
    ex = (ctypes.c_int * 9)()
    ey = (ctypes.c_int * 9)()
    w = (ctypes.c_double * 9)()
    lib().orc_lattice(ex, ey, w)
    return np.array(ex[:]), np.array(ey[:]), np.array(w[:])


def equilibrium(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().orc_equilibrium(rho, ux, uy, _p(out))
    return out


def init_equilibrium(rho, ux, uy) -> np.ndarray:
    rho, ux, uy = _f64(rho), _f64(ux), _f64(uy)
    ny, nx = rho.shape
    f = np.zeros((9, ny, nx))
    lib().orc_init_equilibrium(_p(f), nx, ny, _p(rho), _p(ux), _p(uy))
    return f


def init_ce(rho, ux, uy, tau: float) -> np.ndarray:
    """Equilibrium plus first-order Chapman-Enskog non-equilibrium."""
    rho, ux, uy = _f64(rho), _f64(ux), _f64(uy)
    ny, nx = rho.shape
    f = np.zeros((9, ny, nx))
    lib().orc_init_ce(_p(f), nx, ny, _p(rho), _p(ux), _p(uy), float(tau))
    return f


def moments(f):
    f = _f64(f)
    _, ny, nx = f.shape
    rho, ux, uy = (np.zeros((ny, nx)) for _ in range(3))
    lib().orc_moments(_p(f), nx, ny, _p(rho), _p(ux), _p(uy))
    return rho, ux, uy


def collide_bgk(f, tau: float) -> np.ndarray:
    f = _f64(f)
    out = np.empty_like(f)
    lib().orc_collide_bgk(_p(f), _p(out), f.shape[2], f.shape[1], tau)
    return out


def stream(f) -> np.ndarray:
    f = _f64(f)
    out = np.empty_like(f)
    lib().orc_stream(_p(f), _p(out), f.shape[2], f.shape[1])
    return out


def unstream(f) -> np.ndarray:
    f = _f64(f)
    out = np.empty_like(f)
    lib().orc_unstream(_p(f), _p(out), f.shape[2], f.shape[1])
    return out


def bgk_step(f, tau: float) -> np.ndarray:
    f = _f64(f)
    out = np.empty_like(f)
    lib().orc_bgk_step(_p(f), _p(out), f.shape[2], f.shape[1], tau)
    return out


def bgk_run(f, tau: float, steps: int) -> np.ndarray:
    f = _f64(f).copy()
    lib().orc_bgk_run(_p(f), f.shape[2], f.shape[1], tau, steps)
    return f


def collide_forced(f, tau: float, gx: float) -> np.ndarray:
    """BGK collision with Guo's body-force term, force rho * gx along x."""
    f = _f64(f)
    out = np.empty_like(f)
    lib().orc_collide_forced(_p(f), _p(out), f.shape[2], f.shape[1], tau, gx)
    return out


def stream_channel(f) -> np.ndarray:
    """Streaming with halfway bounce-back walls at y = -1/2, ny - 1/2."""
    f = _f64(f)
    out = np.empty_like(f)
    lib().orc_stream_channel(_p(f), _p(out), f.shape[2], f.shape[1])
    return out


def channel_run(f, tau: float, gx: float, steps: int) -> np.ndarray:
    f = _f64(f).copy()
    lib().orc_channel_run(_p(f), f.shape[2], f.shape[1], tau, gx, steps)
    return f


def channel_velocity(f, gx: float):
    """Velocity of a forced state: u = (sum e f + rho g / 2) / rho."""
    rho, ux, uy = moments(f)
    return ux + 0.5 * gx, uy


def observables(f, tgv=None) -> np.ndarray:
    """[mass, mom_x, mom_y, KE, err_num, err_den, min_f, n_negative];
    tgv = (u0, kx, ky, x0, y0, nu, t) or None."""
    f = _f64(f)
    sums = np.zeros(8)
    t = None if tgv is None else _p(_f64(tgv))
    lib().orc_observables(_p(f), f.shape[2], f.shape[1], t, _p(sums))
    return sums


def restrict(ffine, factor: int, tau_f: float, tau_c: float,
             unstream_: bool = False) -> np.ndarray:
    ffine = _f64(ffine)
    _, nyf, nxf = ffine.shape
    out = np.zeros((9, nyf // factor, nxf // factor))
    lib().orc_restrict(_p(ffine), nxf, nyf, factor, tau_f, tau_c,
                       int(unstream_), _p(out))
    return out


# -------------------------------------------------------------------- GNN ---

def bf16_round(x: float) -> float:
    return lib().orc_bf16_round(float(x))


def gelu(x: float) -> float:
    return lib().orc_gelu(float(x))


def gelu_grad(x: float) -> float:
    return lib().orc_gelu_grad(float(x))


def param_count(rounds: int = 2) -> int:
    return int(lib().orc_gnn_param_count(rounds))


def blob_len(rounds: int = 2) -> int:
    return int(lib().orc_gnn_blob_len(rounds))


def project(v) -> np.ndarray:
    v = _f64(v)
    out = np.zeros(9)
    lib().orc_project(_p(v), _p(out))
    return out


def gnn_collide(f, tau, blob, rounds: int = 2, mode: int = 0,
                want_z: bool = False, act: int = 0, gx: float = 0.0):
    """GNN-corrected collision (Eq. 3) of pre-collision f ([9,ny,nx] or
    [B,9,ny,nx]).  mode 0 = FP64, 1 = BF16 storage emulation; act 0 = GELU,
    1 = ReLU (with rounds = 0: the per-node network of the paper's Fig. 2);
    gx != 0: under a body force rho * gx along x (Guo's velocity and source
    at the effective relaxation time tau * tau_adj)."""
    f = _f64(f)
    single = f.ndim == 3
    if single:
        f = f[None]
    B, _, ny, nx = f.shape
    tau = _f64(np.broadcast_to(np.asarray(tau, dtype=np.float64), (B,)))
    blob = _f64(blob)
    assert blob.size == blob_len(rounds)
    out = np.empty_like(f)
    z = np.zeros((B, ny, nx, NOUT)) if want_z else None
    if gx == 0.0:
        rc = lib().orc_gnn_collide_act(_p(f), _p(out), B, nx, ny, _p(tau), _p(blob),
                                       rounds, mode, act, _p(z) if want_z else None)
    else:
        rc = lib().orc_gnn_collide_forced(_p(f), _p(out), B, nx, ny, _p(tau),
                                          _p(blob), rounds, mode, act, gx,
                                          _p(z) if want_z else None)
    if rc:
        raise MemoryError("oracle forward could not allocate")
    if single:
        out = out[0]
        z = z[0] if want_z else None
    return (out, z) if want_z else out


def gnn_collide_nodes(f, tau: float, blob, nodes, rounds: int = 2,
                      mode: int = 0):
    """Forward at selected nodes (flat indices y*nx+x); returns
    (fstar [count,9], z [count,10])."""
    f = _f64(f)
    _, ny, nx = f.shape
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    blob = _f64(blob)
    fs = np.zeros((nodes.size, 9))
    z = np.zeros((nodes.size, NOUT))
    rc = lib().orc_gnn_collide_nodes(
        _p(f), nx, ny, tau, _p(blob), rounds, mode,
        nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), nodes.size,
        _p(fs), _p(z))
    if rc:
        raise ValueError("bad rounds")
    return fs, z


def gnn_backward(f, G, tau, blob, rounds: int = 2, mode: int = 0, act: int = 0):
    """dL/dparams given G = dL/df* at the forward output."""
    f = _f64(f)
    G = _f64(G)
    if f.ndim == 3:
        f, G = f[None], G[None]
    B, _, ny, nx = f.shape
    tau = _f64(np.broadcast_to(np.asarray(tau, dtype=np.float64), (B,)))
    blob = _f64(blob)
    grad = np.zeros(param_count(rounds))
    rc = lib().orc_gnn_backward_act(_p(f), _p(G), B, nx, ny, _p(tau), _p(blob),
                                    rounds, mode, act, _p(grad))
    if rc:
        raise MemoryError("oracle backward could not allocate")
    return grad


def gnn_collide_gated(f, tau: float, blob, thr: float, mass_prev: float,
                      rounds: int = 2, mode: int = 0):
    """Returns (out, flags, mass) following the per-step fallback rule."""
    f = _f64(f)
    _, ny, nx = f.shape
    out = np.empty_like(f)
    flags = ctypes.c_uint(0)
    mass = ctypes.c_double(0)
    rc = lib().orc_gnn_collide_gated(_p(f), _p(out), nx, ny, tau,
                                     _p(_f64(blob)), rounds, mode, thr,
                                     mass_prev, ctypes.byref(flags),
                                     ctypes.byref(mass))
    if rc:
        raise MemoryError
    return out, flags.value, mass.value


def mse(a, b) -> float:
    """Eq. 4 with N = number of nodes; a, b shaped [..., 9, ny, nx]."""
    a = _f64(np.moveaxis(np.asarray(a), -3, -1))
    b = _f64(np.moveaxis(np.asarray(b), -3, -1))
    return lib().orc_mse(_p(a), _p(b), a.size // 9)


def mse_weighted(a, b, q) -> float:
    """Eq. 4 with each node's residual weighted by the 9 x 9 matrix q;
    a, b shaped [..., 9, ny, nx]."""
    a = _f64(np.moveaxis(np.asarray(a), -3, -1))
    b = _f64(np.moveaxis(np.asarray(b), -3, -1))
    return lib().orc_mse_weighted(_p(a), _p(b), a.size // 9, _p(_f64(q)))


def adam(p, g, m, v, lr, beta1, beta2, eps, step):
    """In-place Adam step on float64 arrays p, m, v."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    g = _f64(g)
    lib().orc_adam(_p(p), _p(g), _p(m), _p(v), p.size, lr, beta1, beta2, eps,
                   step)
