"""GPU parity of the per-node corrected step of the paper's Fig. 2 on the
forced channel (validation section, "Poiseuille Flow": halfway bounce-back
walls, Guo body force rho * gx) against the FP64 oracle: the oracle's
bounce-back streaming, then its corrected collision under the force (Guo's
velocity among the features and in f^eq, Guo's source at the effective
relaxation time tau * tau_adj).

Bars as for the periodic fused step: corrected populations within 1e-3
relative of the FP64 oracle, the correction itself within 5e-2 as a relative
L2 norm and at every node (relative to the largest correction).
"""
import numpy as np
import pytest
import torch

from paper_2504_14494_amd import experiments, gnn, inputs, lbm

pytestmark = pytest.mark.gpu

GX = float(np.float32(2e-4))


def _w(orc):
    return orc.lattice()[2][:, None, None]


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _node_max(a, b):
    """Largest deviation at any node and component, relative to the largest
    reference value: one wrong node is enough to fail it."""
    return float(np.abs(a - b).max() / np.abs(b).max())


def _blob(seed, s_delta):
    return inputs.gnn_blob(seed, 0, s_delta=s_delta)


@pytest.mark.parametrize("ny,nx", [(1, 1), (1, 70), (2, 3), (3, 64), (24, 100), (17, 129)])
def test_channel_step_matches_oracle(orc, ny, nx):
    post = inputs.random_shifted_state((9, ny, nx), 4e-3, seed=700 + 13 * ny + nx)
    blob = _blob(6, 1e-4)
    src = _dev(inputs.planes_to_rows(post))
    dst = torch.full_like(src, float("nan"))
    gnn.lbm_step_simple_channel(src, dst, 0.7, GX, _dev(blob))
    got = inputs.rows_to_planes(dst.double().cpu().numpy()) + _w(orc)
    fpre = orc.stream_channel(post.astype(np.float64) + _w(orc))
    ref = orc.gnn_collide(fpre, 0.7, blob.astype(np.float64), 0, mode=0, act=1, gx=GX)
    forced_bgk = orc.collide_forced(fpre, 0.7, GX)
    rel, rel_c = _rel(got, ref), _rel(got - forced_bgk, ref - forced_bgk)
    node_c = _node_max(got - forced_bgk, ref - forced_bgk)
    print(f"{ny}x{nx}: f* rel-L2 {rel:.2e}, correction rel-L2 {rel_c:.2e}, per node {node_c:.2e}")
    assert np.isfinite(got).all()
    assert rel <= 1e-3 and rel_c <= 5e-2 and node_c <= 5e-2


def _velocity_head_blob(gx_shift=0.0):
    """A network whose tau head reads only the normalised x-velocity feature:
    z0 = (u_x - mu) / sigma with sigma = 1e-2 (the ReLUs held open by a bias
    of 4), all other head outputs zero, s_delta = 1."""
    blob = _blob(7, 1.0)
    off = inputs.blob_offsets(0)

    def put(k, v):
        o, shape = off[k]
        blob[o:o + int(np.prod(shape))] = np.broadcast_to(np.float32(v), shape).ravel()
    W1 = np.zeros((64, 12)); W1[0, 10] = 1.0
    W2 = np.zeros((64, 64)); W2[0, 0] = 1.0
    b1 = np.zeros(64); b1[0] = 4.0
    Wh = np.zeros((10, 64)); Wh[0, 0] = 1.0
    bh = np.zeros(10); bh[0] = -4.0
    for k, v in (("W1", W1), ("b1", b1), ("W2", W2), ("b2", 0.0), ("Wh", Wh), ("bh", bh)):
        put(k, v)
    o = off["mu"][0]
    blob[o + 10] = np.float32(gx_shift)
    blob[o + 12 + 10] = np.float32(1e-2)
    return blob


def test_network_reads_guo_velocity(orc):
    """The relaxation-time head follows the velocity feature, so the
    correction against the forced BGK collision shows which velocity the
    kernel fed the network: against the BF16-emulating oracle within 3e-2,
    where features at the unforced velocity would miss by about 15%."""
    ny, nx = 12, 70
    g = float(np.float32(3e-3))
    post = inputs.random_shifted_state((9, ny, nx), 4e-3, seed=710)
    blob = _velocity_head_blob()
    src = _dev(inputs.planes_to_rows(post))
    dst = torch.empty_like(src)
    gnn.lbm_step_simple_channel(src, dst, 0.8, g, _dev(blob))
    got = inputs.rows_to_planes(dst.double().cpu().numpy()) + _w(orc)
    fpre = orc.stream_channel(post.astype(np.float64) + _w(orc))
    bgk = orc.collide_forced(fpre, 0.8, g)
    ref = orc.gnn_collide(fpre, 0.8, blob.astype(np.float64), 0, mode=1, act=1, gx=g)
    # the same network fed the unforced velocity (mu moved by the half force)
    unforced = orc.gnn_collide(fpre, 0.8, _velocity_head_blob(g / 2).astype(np.float64), 0,
                               mode=1, act=1, gx=g)
    err, miss = _rel(got - bgk, ref - bgk), _rel(unforced - bgk, ref - bgk)
    print(f"correction rel-L2 {err:.2e}; unforced features would give {miss:.2e}")
    assert err <= 3e-2 and miss > 0.1


def test_zero_head_is_the_forced_bgk_channel_step():
    ny, nx = 9, 77
    post = _dev(inputs.planes_to_rows(inputs.random_shifted_state((9, ny, nx), 4e-3, seed=711)))
    blob = _blob(8, 1.0)
    o, _ = inputs.blob_offsets(0)["Wh"]
    blob[o:o + 650] = 0
    a, b = torch.empty_like(post), torch.empty_like(post)
    gnn.lbm_step_simple_channel(post, a, 0.63, GX, _dev(blob))
    lbm.lbm_step_channel(post, b, 0.63, GX)
    d = float((a - b).abs().max().item())
    scale = float(b.abs().max().item())
    print(f"max |simple channel - channel| = {d:.2e} (max |g| {scale:.2e})")
    assert d <= 1e-6 * scale


def test_fallback_is_the_forced_bgk_channel_step(orc):
    ny, nx = 20, 40
    post = inputs.random_shifted_state((9, ny, nx), 3e-3, seed=712)
    blob = _blob(9, 1.0)
    o, _ = inputs.blob_offsets(0)["bh"]
    blob[o + 1:o + 3] = np.float32([50, -50])
    src = _dev(inputs.planes_to_rows(post))
    fb = gnn.Fallback(float((post.astype(np.float64) + _w(orc)).sum()), 1e-6)
    dst, ref = torch.empty_like(src), torch.empty_like(src)
    gnn.lbm_step_simple_channel(src, dst, 0.7, GX, _dev(blob), fb)
    lbm.lbm_step_channel(src, ref, 0.7, GX)
    periodic = torch.empty_like(src)
    lbm.lbm_step_bgk(src, periodic, 0.7)
    assert int(fb.flags.item()) & 1 and int(fb.n_fallback.item()) == 1
    # the same arithmetic in two kernels: equal up to where the compiler
    # fuses multiplies and adds (a few ulps)
    d = float((dst - ref).abs().max().item())
    scale = float(ref.abs().max().item())
    d_periodic = float((dst - periodic).abs().max().item())
    print(f"max |fallback - channel step| = {d:.2e}; vs periodic BGK {d_periodic:.2e}")
    assert d <= 1e-6 * scale and d_periodic > 1e-4 * scale


def test_channel_gate_keeps_mass_with_walls(orc):
    """Bounce-back and the forcing keep mass: a sane network never trips the
    drift branch on the channel over many steps."""
    blob = torch.as_tensor(_blob(10, 1e-4), device="cuda")
    lat = gnn.GnnLattice(6, 16, blob, 0)
    lat.a.zero_()
    lat.sync_mass()
    lat.step_gnn_channel(0.8, GX, 300)
    torch.cuda.synchronize()
    assert int(lat.n_fallback.item()) == 0
    _, _, _, sums = lbm.lbm_moments(lat.a)   # sums[0]: total mass
    assert abs(float(sums[0].item()) - 6 * 16) < 1e-7 * 6 * 16


def test_message_passing_lattice_refuses_the_channel():
    blob = torch.as_tensor(inputs.gnn_blob(1, 2, s_delta=1e-4), device="cuda")
    lat = gnn.GnnLattice(8, 8, blob, 2)
    with pytest.raises(ValueError):
        lat.step_gnn_channel(0.7, GX, 1)


def test_poiseuille_study_with_the_per_node_network():
    """A network whose head is zero reproduces the BGK channel study, and a
    random small-correction network stays close to it without falling back."""
    blob = _blob(11, 1e-4)
    o, _ = inputs.blob_offsets(0)["Wh"]
    zero = blob.copy()
    zero[o:o + 650] = 0
    kw = dict(re_list=(10,), ny=16, diffusion_times=2.0)
    bgk = experiments.poiseuille_study(**kw)["rows"][0]
    z = experiments.poiseuille_study(blob=torch.as_tensor(zero, device="cuda"), **kw)["rows"][0]
    r = experiments.poiseuille_study(blob=torch.as_tensor(blob, device="cuda"), **kw)["rows"][0]
    print(bgk, z, r, sep="\n")
    assert abs(z["max_rel_err"] - bgk["max_rel_err"]) < 1e-4
    assert z["fallback_steps"] == 0 and r["fallback_steps"] == 0
    assert r["max_rel_err"] < 0.1
