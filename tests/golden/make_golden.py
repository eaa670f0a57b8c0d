"""Writes the stored expected values under tests/golden/ from the FP64 CPU
oracle alone (no GPU, no library code of the package's HIP path).

tgv64_re100.txt -- the validation section's Taylor-Green case ("Taylor-Green
Vortex Validation": 64 x 64 periodic lattice, Re = 100, errors at 1000, 3000
and 5000 steps).  u0 = 0.04, nu = u0 * 64 / Re, tau = 3 nu + 1/2 rounded to
FP32 (the value the FP32 lattice steps with), uniform density and f = f^eq
(Eq. 2) at t = 0, plain BGK (Eq. 1).  Errors against the analytic decay
u_a = u(0) exp(-2 nu k^2 t), nu = (tau - 1/2) / 3, k = 2 pi / 64:
  velocity error  ||u - u_a||_2 / ||u_a||_2 over all nodes and both components,
  energy error    |E - E_a| / E_a with E = 1/2 sum |u|^2.

Run from the repository root:  python tests/golden/make_golden.py
"""
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2504_14494_amd import inputs  # noqa: E402  (seeded/closed-form inputs only)

N, RE, U0 = 64, 100.0, 0.04
CHECKPOINTS = (1000, 3000, 5000)


def tgv_errors():
    _, tau = inputs.tgv_params(N, U0, RE)
    tau = float(np.float32(tau))
    rho, ux0, uy0 = inputs.tgv_velocity(N, N, U0)
    f = oracle.init_equilibrium(np.ones_like(rho), ux0, uy0)
    nu, k = (tau - 0.5) / 3.0, 2 * math.pi / N
    rows, done = [], 0
    for t in CHECKPOINTS:
        f = oracle.bgk_run(f, tau, t - done)
        done = t
        _, vx, vy = oracle.moments(f)
        decay = math.exp(-2 * nu * k * k * t)
        ax, ay = ux0 * decay, uy0 * decay
        num = ((vx - ax) ** 2 + (vy - ay) ** 2).sum()
        den = (ax ** 2 + ay ** 2).sum()
        e_h = 0.5 * (vx ** 2 + vy ** 2).sum()
        e_a = 0.5 * den
        rows.append((t, float(math.sqrt(num / den)), float(abs(e_h - e_a) / e_a)))
    return tau, rows


def main():
    oracle.build(force=False)
    tau, rows = tgv_errors()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tgv64_re100.txt")
    with open(path, "w") as fh:
        fh.write("# Taylor-Green vortex, 64x64 periodic D2Q9, Re = 100, u0 = 0.04, plain BGK, FP64 oracle\n")
        fh.write("# (validation section 'Taylor-Green Vortex Validation', table of velocity errors at\n")
        fh.write("#  1000/3000/5000 steps; the paper prints 1.83e-2 2.41e-2 2.72e-2 for its own, unstated\n")
        fh.write("#  start and u0 -- context only, not reproduced by this start)\n")
        fh.write("# start: uniform density, f = f^eq(1, u_TGV); tau rounded to FP32\n")
        fh.write("# written by tests/golden/make_golden.py (calls only the oracle)\n")
        fh.write(f"tau {tau!r}\n")
        fh.write("# steps vel_err energy_err\n")
        for t, ve, ee in rows:
            fh.write(f"{t} {ve!r} {ee!r}\n")
    print(open(path).read())


if __name__ == "__main__":
    main()
