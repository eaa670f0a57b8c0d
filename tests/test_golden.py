"""Stored expected values under tests/golden/ (written by
tests/golden/make_golden.py from the FP64 oracle alone).

The validation section's Taylor-Green case ("Taylor-Green Vortex
Validation": 64 x 64, Re = 100, errors at 1000, 3000 and 5000 steps).  The
CPU test guards the stored values against later oracle changes; the GPU test
runs the same case through the FP32 library and compares its errors with the
stored ones.  The paper's own printed errors (1.83e-2, 2.41e-2, 2.72e-2) are
for a start and amplitude it does not state and are kept in the fixture as
context only.
"""
import math
import os

import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tgv64_re100.txt")


def _load():
    tau, rows = None, []
    with open(GOLDEN) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "tau":
                tau = float(parts[1])
            else:
                rows.append((int(parts[0]), float(parts[1]), float(parts[2])))
    return tau, rows


def test_golden_tgv_matches_the_oracle(orc):
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_golden", os.path.join(os.path.dirname(GOLDEN), "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    tau, rows = _load()
    tau_now, rows_now = mg.tgv_errors()
    assert tau_now == tau
    assert [r[0] for r in rows_now] == [r[0] for r in rows]
    for (t, ve, ee), (_, ve2, ee2) in zip(rows, rows_now):
        assert abs(ve2 - ve) <= 1e-12 * ve, (t, ve, ve2)
        assert abs(ee2 - ee) <= 1e-12 * ee, (t, ee, ee2)
    # the uniform-density start carries an acoustic transient of relative
    # size ~ 0.43 u0 = 1.7e-2 in the pressure, but its velocity imprint on a
    # viscous 64^2 lattice at Re = 100 is a few 1e-3 and does not grow
    assert all(1e-3 < ve < 5e-3 for _, ve, _ in rows)


@pytest.mark.gpu
def test_golden_tgv_fp32_library():
    """FP32 library run of the same case against the stored FP64 errors.  The
    errors of the two runs differ by at most ||u_32 - u_64|| / ||u_a||.  The
    FP32 deviation is bounded by 1e-5 of ||u_a|| after 1000 steps (the FP32
    BGK parity bar) and grows at most in proportion to the step count, while
    ||u_a|| decays as exp(-2 nu k^2 t) (by 0.37 and 0.14 from step 1000 to
    steps 3000 and 5000), so the bar is 1e-5 (t / 1000) scaled by that decay;
    the energy error, quadratic in u, gets twice that."""
    from paper_2504_14494_amd import experiments
    tau, rows = _load()
    rep = experiments.tgv_validation(None, checkpoints=tuple(r[0] for r in rows))
    assert rep["tau"] == tau
    nu, k = (tau - 0.5) / 3.0, 2 * math.pi / 64
    for (t, ve, ee), got in zip(rows, rep["rows"]):
        decay = math.exp(-2 * nu * k * k * t) / math.exp(-2 * nu * k * k * 1000)
        tol = 1e-5 * (t / 1000) / decay
        print(f"{t} steps: velocity error GPU {got['vel_err']:.6e} oracle {ve:.6e}; "
              f"energy error GPU {got['energy_err']:.6e} oracle {ee:.6e}")
        assert abs(got["vel_err"] - ve) <= tol
        assert abs(got["energy_err"] - ee) <= 2 * tol
