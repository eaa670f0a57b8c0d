"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module holds only workload definitions and random draws — none of the
method's arithmetic.  Both sides receive exactly the arrays produced here
(rounded to FP32 where the GPU consumes FP32), so any difference between them
comes from their own computation.

Workloads are the Taylor-Green vortex of the paper's validation section on a
periodic lattice, with the sizes, Reynolds numbers and amplitudes of the
benchmark configurations: 64x64 at Re=100 for parity, 4096^2 / 8192^2 for
throughput, 2048^2 for the corrected collision, 128^2 coarse / 512^2 fine
lattices for training.
"""
from __future__ import annotations

import numpy as np

HID = 64
NFEAT = 12
NOUT = 10
EDGE_IN = 2 * HID + 2
NODE_IN = 2 * HID


def tgv_params(n: int, u0: float, re: float):
    """Viscosity and relaxation time of the Taylor-Green workload:
    nu = u0 * n / Re (lattice units), tau = 3 nu + 1/2."""
    nu = u0 * n / re
    return nu, 3.0 * nu + 0.5


def tgv_velocity(nx: int, ny: int, u0: float, x0: float = 0.0,
                 y0: float = 0.0, dtype=np.float64):
    """Uniform density and the Taylor-Green velocity field at t = 0 on integer
    nodes: u_x = -u0 cos(kx X) sin(ky Y), u_y = u0 (kx/ky) sin(kx X) cos(ky Y),
    kx = 2 pi / nx, ky = 2 pi / ny, X = x - x0, Y = y - y0."""
    kx, ky = 2 * np.pi / nx, 2 * np.pi / ny
    X = np.arange(nx, dtype=np.float64)[None, :] - x0
    Y = np.arange(ny, dtype=np.float64)[:, None] - y0
    ux = -u0 * np.cos(kx * X) * np.sin(ky * Y)
    uy = u0 * (kx / ky) * np.sin(kx * X) * np.cos(ky * Y)
    rho = np.ones((ny, nx))
    return rho.astype(dtype), ux.astype(dtype), uy.astype(dtype)


def tgv_pressure_density(nx: int, ny: int, u0: float, x0: float = 0.0, y0: float = 0.0,
                         dtype=np.float64):
    """Density that carries the Taylor-Green pressure field at t = 0,
    rho = 1 + p / c_s^2 with p = -(u0^2 / 4)(cos 2kx X + (kx/ky)^2 cos 2ky Y),
    the closed-form companion of tgv_velocity (uniform density instead
    launches an acoustic transient)."""
    kx, ky = 2 * np.pi / nx, 2 * np.pi / ny
    X = np.arange(nx, dtype=np.float64)[None, :] - x0
    Y = np.arange(ny, dtype=np.float64)[:, None] - y0
    rho = 1.0 - 0.75 * u0 * u0 * (np.cos(2 * kx * X) + (kx / ky) ** 2 * np.cos(2 * ky * Y))
    return rho.astype(dtype)


def tgv_spec(nx: int, ny: int, u0: float, nu: float, t: float,
             x0: float = 0.0, y0: float = 0.0):
    """(u0, kx, ky, x0, y0, nu, t) describing the decaying field."""
    return (u0, 2 * np.pi / nx, 2 * np.pi / ny, x0, y0, nu, t)


def planes_to_rows(a):
    """[..., 9, ny, nx] (one plane per direction, the oracle's order) ->
    [..., ny, 9, nx] (row-interleaved, the library's order).  Layout only."""
    a = np.asarray(a)
    return np.ascontiguousarray(np.swapaxes(a, -3, -2))


def rows_to_planes(a):
    """Inverse of planes_to_rows."""
    a = np.asarray(a)
    return np.ascontiguousarray(np.swapaxes(a, -3, -2))


def random_shifted_state(shape, amp: float, seed: int) -> np.ndarray:
    """Random shifted populations g = f - w with N(0, amp^2) entries, FP32.
    With amp <= 5e-3 every f = w + g stays positive (w >= 1/36)."""
    rng = np.random.default_rng(seed)
    return (amp * rng.standard_normal(shape)).astype(np.float32)


def gnn_tensor_shapes(rounds: int = 2):
    """(name, shape, fan_in) of every trainable tensor, in blob order."""
    out = [("W1", (HID, NFEAT), NFEAT), ("b1", (HID,), NFEAT),
           ("W2", (HID, HID), HID), ("b2", (HID,), HID)]
    for r in range(rounds):
        out += [(f"We{r}", (HID, EDGE_IN), EDGE_IN), (f"be{r}", (HID,), EDGE_IN),
                (f"Wn{r}", (HID, NODE_IN), NODE_IN), (f"bn{r}", (HID,), NODE_IN)]
    out += [("Wh", (NOUT, HID), HID), ("bh", (NOUT,), HID)]
    return out


def gnn_param_count(rounds: int = 2) -> int:
    return sum(int(np.prod(s)) for _, s, _ in gnn_tensor_shapes(rounds))


def gnn_blob_len(rounds: int = 2) -> int:
    return gnn_param_count(rounds) + 2 * NFEAT + 1


def feature_scales(u0: float):
    """Per-feature (mu, sigma) making the features O(1) for a flow of
    amplitude u0: mu = 0; sigma = 3 u0 w_i for g_i, 3 u0^2 for rho - 1 and u0
    for the velocity components."""
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    sigma = [3 * u0 * wi for wi in w] + [3 * u0 * u0, u0, u0]
    return np.zeros(NFEAT), np.array(sigma)


def gnn_blob(seed: int = 0, rounds: int = 2, s_delta: float = 1e-4,
             u0: float = 0.04, mu=None, sigma=None) -> np.ndarray:
    """FP32 parameter blob: every weight and bias ~ N(0, 1/fan_in) from
    numpy's default_rng(seed), followed by mu[12], sigma[12], s_delta."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, shape, fan_in in gnn_tensor_shapes(rounds):
        parts.append(rng.standard_normal(shape).ravel() / np.sqrt(fan_in))
    m0, s0 = feature_scales(u0)
    mu = m0 if mu is None else np.asarray(mu, dtype=np.float64)
    sigma = s0 if sigma is None else np.asarray(sigma, dtype=np.float64)
    parts += [mu, sigma, np.array([s_delta])]
    return np.concatenate(parts).astype(np.float32)


def blob_offsets(rounds: int = 2):
    """name -> (offset, shape) inside the blob."""
    off, out = 0, {}
    for name, shape, _ in gnn_tensor_shapes(rounds):
        out[name] = (off, shape)
        off += int(np.prod(shape))
    out["mu"] = (off, (NFEAT,))
    out["sigma"] = (off + NFEAT, (NFEAT,))
    out["s_delta"] = (off + 2 * NFEAT, (1,))
    return out


def training_draws(n_runs: int, seed: int):
    """Random flow conditions of the training set: u0 ~ U[0.02, 0.06],
    Re ~ U[1000, 5000], phase (x0, y0) ~ U[0, 1)^2 in units of the period."""
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(0.02, 0.06, n_runs)
    re = rng.uniform(1000.0, 5000.0, n_runs)
    phase = rng.uniform(0.0, 1.0, (n_runs, 2))
    return u0, re, phase
