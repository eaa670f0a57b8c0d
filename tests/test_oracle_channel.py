"""Pins of the oracle's channel flow (validation section, "Poiseuille Flow",
Eq. 5) against closed forms: the steady profile of BGK with halfway
bounce-back and Guo forcing is the parabola of Eq. 5 plus a uniform slip
g (16 (tau - 1/2)^2 - 3) / (24 nu) (He, Zou, Luo and Dembo's analysis of
bounce-back; it vanishes at tau = 1/2 + sqrt(3/16)), and the forced
collision adds exactly the force to each node's momentum."""
import math

import numpy as np
import pytest


def _rest(orc, ny, nx):
    w = orc.lattice()[2]
    return np.broadcast_to(w[:, None, None], (9, ny, nx)).copy()


def _steady(orc, tau, ny=16, nx=2, g=1e-6, diffusion_times=20):
    nu = (tau - 0.5) / 3.0
    f = orc.channel_run(_rest(orc, ny, nx), tau, g, int(diffusion_times * ny * ny / nu))
    ux, uy = orc.channel_velocity(f, g)
    return ux, uy, nu


@pytest.mark.parametrize("tau", [0.8, 0.5 + math.sqrt(3.0 / 16.0), 1.2])
def test_steady_profile_is_parabola_plus_bounce_back_slip(orc, tau):
    ny, g = 16, 1e-6
    ux, uy, nu = _steady(orc, tau, ny=ny, g=g)
    y = np.arange(ny)
    parabola = g / (2 * nu) * (y + 0.5) * (ny - y - 0.5)
    slip = g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu)
    for col in range(ux.shape[1]):
        err = np.abs(ux[:, col] - parabola - slip).max() / parabola.max()
        assert err < 1e-9, (tau, err)
    assert np.abs(uy).max() < 1e-12
    # the bulk solves the steady momentum balance exactly: nu u'' = -g
    d2 = ux[2:, 0] - 2 * ux[1:-1, 0] + ux[:-2, 0]
    assert np.abs(d2 + g / nu).max() < 1e-9 * g / nu


def test_forced_collision_adds_the_force_and_keeps_mass(orc):
    rng = np.random.default_rng(5)
    w = orc.lattice()[2]
    f = w[:, None, None] * (1.0 + 0.05 * rng.standard_normal((9, 4, 5)))
    g = 3e-4
    out = orc.collide_forced(f, 0.7, g)
    ex, ey, _ = orc.lattice()
    rho = f.sum(0)
    assert np.allclose(out.sum(0), rho, rtol=0, atol=1e-15)
    jx0 = np.tensordot(ex.astype(float), f, 1)
    jx1 = np.tensordot(ex.astype(float), out, 1)
    assert np.allclose(jx1 - jx0, rho * g, rtol=1e-12, atol=1e-17)
    jy0 = np.tensordot(ey.astype(float), f, 1)
    jy1 = np.tensordot(ey.astype(float), out, 1)
    assert np.allclose(jy1, jy0, rtol=0, atol=1e-15)
    # zero force: the plain BGK collision
    assert np.array_equal(orc.collide_forced(f, 0.7, 0.0), orc.collide_bgk(f, 0.7))


@pytest.mark.parametrize("ny,nx", [(1, 3), (2, 2), (5, 7)])
def test_bounce_back_streaming_is_a_mass_conserving_permutation(orc, ny, nx):
    vals = np.arange(9 * ny * nx, dtype=np.float64).reshape(9, ny, nx) + 1.0
    out = orc.stream_channel(vals)
    assert np.array_equal(np.sort(out.ravel()), np.sort(vals.ravel()))
    # a population that meets a wall comes back reversed at its own node
    opp = [0, 3, 4, 1, 2, 7, 8, 5, 6]
    assert out[opp[4], 0, 0] == vals[4, 0, 0]          # down through the bottom wall
    assert out[opp[2], ny - 1, 0] == vals[2, ny - 1, 0]  # up through the top wall


def test_channel_at_rest_without_force_stays_at_rest(orc):
    f = orc.channel_run(_rest(orc, 6, 3), 0.9, 0.0, 50)
    # equal up to the FP64 rounding of sum(w) = 1 inside the equilibrium
    assert np.abs(f - _rest(orc, 6, 3)).max() < 1e-15
