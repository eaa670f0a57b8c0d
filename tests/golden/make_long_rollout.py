"""Writes tests/golden/tgv2048_re1e4_energy.txt: the FP64 oracle's reference for
the long high-Reynolds-number rollout.

Workload: Taylor-Green vortex on a 2048 x 2048 periodic lattice, u0 = 0.05,
Re = 1e4 (nu = u0 n / Re, tau = 3 nu + 1/2 rounded to FP32, the value the
GPU runs with), uniform density, f initialised to equilibrium, plain BGK
(Eq. 1 with the equilibrium of Eq. 2), 20000 steps.  Every 2000 steps the
script records, on the 256 x 256 restriction by injection (every 8th node in
x and y):
  - the kinetic energy 1/2 sum |u|^2 (the quantity behind the paper's
    energy-decay comparison, validation section and "Reynolds Number Study"),
  - the velocity (u_x, u_y) at eight fixed sampled nodes of that restriction,
and, over the whole lattice, the total mass.

Everything is computed by oracle/ (FP64); numpy only slices and sums its
outputs.  The oracle's loops share their nodes among OMP threads, which does
not change any value.  Takes about 35 minutes on 8 cores.

    python tests/golden/make_long_rollout.py [--threads 8]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2504_14494_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "tgv2048_re1e4_energy.txt")
N, U0, RE, STEPS, EVERY, STRIDE = 2048, 0.05, 1.0e4, 20000, 2000, 8
# sampled nodes of the 256^2 restriction (indices on the 2048^2 lattice)
NODES = [(0, 0), (0, 2040), (2040, 8), (1024, 1024), (512, 1536), (1536, 512), (8, 1000),
         (2000, 2000)]


def tau32():
    _, tau = inputs.tgv_params(N, U0, RE)
    return float(np.float32(tau))


def injection_row(f, step):
    sub = np.ascontiguousarray(f[:, ::STRIDE, ::STRIDE])
    _, ux, uy = oracle.moments(sub)
    energy = 0.5 * float((ux * ux + uy * uy).sum())
    mass = float(oracle.observables(f)[0])
    row = [step, energy, mass]
    for y, x in NODES:
        row += [float(ux[y // STRIDE, x // STRIDE]), float(uy[y // STRIDE, x // STRIDE])]
    return row


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=8)
    args = ap.parse_args(argv)
    oracle.build(force=False)
    oracle.set_threads(args.threads)
    tau = tau32()
    rho, ux, uy = inputs.tgv_velocity(N, N, U0, dtype=np.float32)
    f = oracle.init_equilibrium(rho.astype(np.float64), ux.astype(np.float64),
                                uy.astype(np.float64))
    rows = [injection_row(f, 0)]
    t0 = time.perf_counter()
    for step in range(EVERY, STEPS + 1, EVERY):
        f = oracle.bgk_run(f, tau, EVERY)
        rows.append(injection_row(f, step))
        print(f"step {step}: energy {rows[-1][1]:.12e} ({time.perf_counter() - t0:.0f} s)",
              flush=True)
    head = [
        "FP64 oracle reference of the long high-Re Taylor-Green rollout (plain BGK, Eq. 1-2).",
        f"lattice {N}x{N} periodic, u0 = {U0}, Re = {RE:g}, tau = {tau!r} (FP32 value), "
        f"uniform density, f = f^eq at t = 0, {STEPS} steps",
        f"energy_256: 1/2 sum |u|^2 over the injection of every {STRIDE}th node (256 x 256); "
        "mass: sum f over the whole lattice",
        "ux/uy: velocity at the sampled nodes (y, x) " + " ".join(f"{y},{x}" for y, x in NODES),
        "written by tests/golden/make_long_rollout.py (calls oracle/ only)",
        "columns: step energy_256 mass " + " ".join(f"ux{k} uy{k}" for k in range(len(NODES))),
    ]
    tmp = OUT + ".tmp"
    np.savetxt(tmp, np.array(rows), fmt="%.17g", header="\n".join(head))
    os.replace(tmp, OUT)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
