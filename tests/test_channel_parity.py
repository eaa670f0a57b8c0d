"""GPU parity of the forced channel step (validation section, "Poiseuille
Flow", Eq. 5: halfway bounce-back walls, Guo body force) against the FP64
oracle, one step on random states and the steady profile against its closed
form."""
import math

import numpy as np
import pytest
import torch

from paper_2504_14494_amd import experiments, inputs, lbm

pytestmark = pytest.mark.gpu


def _w(orc):
    return orc.lattice()[2][:, None, None]


@pytest.mark.parametrize("ny,nx", [(1, 1), (1, 5), (2, 3), (3, 70), (17, 257)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_one_step_matches_oracle(orc, ny, nx, dtype):
    post = inputs.random_shifted_state((9, ny, nx), 4e-3, seed=ny * 1000 + nx)
    tau, g = 0.7, 3e-4
    src = torch.as_tensor(inputs.planes_to_rows(post), dtype=dtype, device="cuda")
    dst = torch.full_like(src, float("nan"))
    lbm.lbm_step_channel(src, dst, tau, g)
    got = inputs.rows_to_planes(dst.double().cpu().numpy()) + _w(orc)
    f = inputs.rows_to_planes(src.double().cpu().numpy()) + _w(orc)
    ref = orc.collide_forced(orc.stream_channel(f), tau, g)
    err = np.abs(got - ref).max()
    print(f"{dtype} {ny}x{nx}: max abs {err:.2e}")
    assert err <= (2e-7 if dtype == torch.float32 else 5e-15)


@pytest.mark.parametrize("g", [0.0, float(np.float32(2e-4))])
def test_profile_kernel_matches_oracle(orc, g):
    """A post-collision state carries the step's whole force in its momentum
    (the forced collision adds rho g): its fluid velocity is
    sum e f* / rho - g / 2, the oracle's (sum e f + rho g / 2) / rho of the
    pre-collision state it came from."""
    pre = inputs.random_shifted_state((9, 11, 300), 4e-3, seed=3) + _w(orc)
    tau = 0.8
    post = orc.collide_forced(pre, tau, g)
    src = torch.as_tensor(inputs.planes_to_rows(post - _w(orc)), dtype=torch.float32,
                          device="cuda")
    prof = lbm.lbm_channel_profile(src, g).cpu().numpy()
    ux_pre, _ = orc.channel_velocity(pre, g)
    # post rounded to FP32 (|g| <= 0.02, so <= 1e-9 absolute per population)
    err = np.abs(prof - ux_pre.mean(1)).max()
    print(f"profile vs oracle velocity of the pre-collision state: {err:.2e}")
    assert err <= 1e-8
    # and the exact FP64 identity on the rounded state itself
    f32 = inputs.rows_to_planes(src.double().cpu().numpy()) + _w(orc)
    rho, ux, _ = orc.moments(f32)
    assert np.abs(prof - (ux - 0.5 * g).mean(1)).max() <= 1e-15


def _steady_profile(tau, ny, g, dtype):
    nu = (tau - 0.5) / 3.0
    lat = lbm.Lattice(4, ny, dtype=dtype)
    lat.a.zero_()
    lat.step_channel(tau, g, int(25 * ny * ny / nu))
    g32 = lat.a if dtype == torch.float32 else lbm.lbm_restrict(lat.a, 1, tau, tau, False, False)
    return lbm.lbm_channel_profile(g32, g).cpu().numpy(), nu


def test_steady_fp64_profile_is_parabola_plus_slip():
    tau, ny, g = 1.2, 24, 1e-6
    prof, nu = _steady_profile(tau, ny, g, torch.float64)
    y = np.arange(ny)
    ref = g / (2 * nu) * (y + 0.5) * (ny - y - 0.5) + g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu)
    err = np.abs(prof - ref).max() / ref.max()
    print(f"FP64 steady profile vs closed form: {err:.2e}")
    # the profile is read through FP32 moments of the FP64 state
    assert err <= 1e-6


def test_steady_fp32_profile_at_the_magic_tau_is_the_parabola():
    tau = float(np.float32(0.5 + math.sqrt(3.0 / 16.0)))
    ny, g = 24, 1e-6
    prof, nu = _steady_profile(tau, ny, g, torch.float32)
    y = np.arange(ny)
    ref = g / (2 * nu) * (y + 0.5) * (ny - y - 0.5) + g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu)
    err = np.abs(prof - ref).max() / ref.max()
    print(f"FP32 steady profile vs Eq. 5: {err:.2e}")
    assert err <= 1e-4


def test_poiseuille_study_reports_the_closed_form_error():
    rep = experiments.poiseuille_study(re_list=(10, 100), ny=16, u_max=0.05)
    for row in rep["rows"]:
        print(row)
        assert abs(row["max_rel_err"] - abs(row["slip_rel_closed_form"])) <= 1e-4
