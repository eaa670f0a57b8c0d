"""GPU parity of the GNN-corrected collision (paper: Methodology, GNN
enhancement and its integration with the LBM, Eq. 3) against the CPU oracle.

The library computes the network in BF16 with FP32 accumulation.  It is
compared with the oracle in two modes:
  mode 0  FP64 throughout: corrected populations within 1e-3 relative at
          the inference workload's correction scale s_delta = 1e-4, and a
          bound on the correction itself;
  mode 1  FP64 arithmetic with BF16 rounding at the points where the kernel
          stores BF16 (weights, features, activations, summed messages):
          head outputs agree to summation-order effects only.
Every comparison is made twice: as a relative L2 norm over the field and
node by node (largest deviation at any node relative to the largest
reference value), so that a single wrong node fails.
Layouts: the library stores [.., ny, 9, nx]; the oracle [.., 9, ny, nx]
(inputs.planes_to_rows / rows_to_planes, a transpose).
"""
import numpy as np
import pytest
import torch

from paper_2504_14494_amd import gnn, inputs, lbm

pytestmark = pytest.mark.gpu

R = 2


def _w(orc):
    return orc.lattice()[2][:, None, None]


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _node_max(a, b):
    """Largest deviation at any node and component, relative to the largest
    reference value: one wrong node is enough to fail it."""
    return float(np.abs(a - b).max() / np.abs(b).max())


def _head_nodes_ok(z, zref):
    """Head outputs node by node against the BF16-emulating oracle.  The two
    sides sum in different orders (FP32 MFMA against FP64), so now and then
    a value that sits within ~1e-7 of a BF16 rounding boundary rounds the
    other way; about 5000 rounded values feed each node's head, so some nodes
    carry one such flip, worth up to ~2e-3 of max|z|.  Bar: within 1e-3 of
    max|z| at 95 % of the nodes or more, within 5e-3 at every node (a
    wrong node, e.g. one message missing, is off by several percent)."""
    dz = np.abs(z - zref).max(axis=-1) / np.abs(zref).max()
    frac = float(np.mean(dz > 1e-3))
    print(f"head outputs: worst node {dz.max():.2e} of max|z|, nodes above 1e-3: {frac:.1%}")
    return dz.max() <= 5e-3 and frac <= 0.05


def _forward(g_planes, taus, blob, want_z=True):
    """Library forward of shifted pre-collision populations [B, 9, ny, nx];
    returns the shifted post-collision populations in the same order (float64)
    and the head outputs z [B, ny, nx, 10]."""
    out, z = gnn.gnn_forward(_dev(inputs.planes_to_rows(g_planes)), _dev(taus), _dev(blob), R,
                             want_z=want_z)
    torch.cuda.synchronize()
    g_post = inputs.rows_to_planes(out.double().cpu().numpy())
    return g_post, (z.double().cpu().numpy() if want_z else None)


def _bgk_planes(orc, f, taus):
    return np.stack([orc.collide_bgk(f[b], float(taus[b])) for b in range(f.shape[0])])


@pytest.mark.parametrize("B,ny,nx", [(1, 1, 1), (1, 3, 5), (2, 8, 12), (1, 16, 16),
                                     (1, 17, 33), (1, 40, 24), (3, 20, 37)])
def test_forward_matches_oracle_at_inference_scale(orc, B, ny, nx):
    g = inputs.random_shifted_state((B, 9, ny, nx), 4e-3, seed=1000 * B + 10 * ny + nx)
    taus = np.float32(0.6 + 0.07 * np.arange(B))
    blob = inputs.gnn_blob(0, R, s_delta=1e-4)
    got, z = _forward(g, taus, blob)
    f = g.astype(np.float64) + _w(orc)
    ref, zref = orc.gnn_collide(f, taus.astype(np.float64), blob.astype(np.float64), R, mode=0,
                                want_z=True)
    got_f = got + _w(orc)
    rel = _rel(got_f, ref)
    bgk = _bgk_planes(orc, f, taus.astype(np.float64))
    rel_corr = _rel(got_f - bgk, ref - bgk)
    node_corr = _node_max(got_f - bgk, ref - bgk)
    print(f"f* rel-L2 {rel:.2e}; correction rel-L2 {rel_corr:.2e}, per node {node_corr:.2e}; "
          f"z rel {_rel(z, zref):.2e}")
    assert rel <= 1e-3
    assert rel_corr <= 5e-2
    assert node_corr <= 5e-2
    assert np.isfinite(got).all()


@pytest.mark.parametrize("B,ny,nx", [(1, 5, 7), (2, 16, 16), (1, 19, 35)])
def test_head_matches_bf16_emulating_oracle(orc, B, ny, nx):
    """s_delta = 1 so that the correction is as large as the populations."""
    g = inputs.random_shifted_state((B, 9, ny, nx), 4e-3, seed=7 * nx + ny)
    taus = np.float32(np.full(B, 0.8))
    blob = inputs.gnn_blob(3, R, s_delta=1.0)
    got, z = _forward(g, taus, blob)
    f = g.astype(np.float64) + _w(orc)
    ref1, z1 = orc.gnn_collide(f, taus.astype(np.float64), blob.astype(np.float64), R, mode=1,
                               want_z=True)
    rz, rf = _rel(z, z1), _rel(got + _w(orc), ref1)
    print(f"vs BF16-emulating oracle: z rel-L2 {rz:.2e}; f* rel-L2 {rf:.2e}")
    assert rz <= 1e-3
    assert _head_nodes_ok(z, z1)
    assert rf <= 1e-3


def test_step_gnn_pulls_then_collides(orc):
    ny, nx = 24, 40
    post = inputs.random_shifted_state((9, ny, nx), 4e-3, seed=5)
    blob = inputs.gnn_blob(1, R, s_delta=1e-4)
    tau = np.float32(0.7)
    dst = torch.full((ny, 9, nx), float("nan"), device="cuda")
    gnn.lbm_step_gnn(_dev(inputs.planes_to_rows(post)), dst, float(tau), _dev(blob), R)
    torch.cuda.synchronize()
    got = inputs.rows_to_planes(dst.double().cpu().numpy()) + _w(orc)
    fpre = orc.stream(post.astype(np.float64) + _w(orc))
    ref = orc.gnn_collide(fpre, float(tau), blob.astype(np.float64), R, mode=0)
    assert np.isfinite(got).all()
    assert _rel(got, ref) <= 1e-3
    bgk = orc.collide_bgk(fpre, float(tau))
    assert _rel(got - bgk, ref - bgk) <= 5e-2
    assert _node_max(got - bgk, ref - bgk) <= 5e-2


def _zero_head(blob):
    off = inputs.blob_offsets(R)
    b = blob.copy()
    o, shp = off["Wh"]
    b[o:o + int(np.prod(shp))] = 0
    o, shp = off["bh"]
    b[o:o + int(np.prod(shp))] = 0
    return b


@pytest.mark.parametrize("ny,nx", [(7, 9), (33, 48)])
def test_zero_head_step_equals_bgk_step(ny, nx):
    """W_h = 0, b_h = 0 gives tau_adj = 1 and delta f = 0: the corrected
    step must reproduce the plain BGK step value for value."""
    post = _dev(inputs.planes_to_rows(inputs.random_shifted_state((9, ny, nx), 4e-3, seed=9)))
    blob = _dev(_zero_head(inputs.gnn_blob(2, R, s_delta=1.0)))
    a = torch.empty_like(post)
    b = torch.empty_like(post)
    gnn.lbm_step_gnn(post, a, 0.63, blob, R)
    lbm.lbm_step_bgk(post, b, 0.63)
    assert torch.equal(a, b)


def test_batch_lattices_are_independent(orc):
    """Each lattice of a batch is its own periodic domain with its own tau."""
    B, ny, nx = 3, 12, 20
    g = inputs.random_shifted_state((B, 9, ny, nx), 4e-3, seed=77)
    taus = np.float32([0.55, 0.8, 1.3])
    blob = inputs.gnn_blob(4, R, s_delta=1e-2)
    got, _ = _forward(g, taus, blob, want_z=False)
    for b in range(B):
        one, _ = _forward(g[b:b + 1], taus[b:b + 1], blob, want_z=False)
        assert np.array_equal(one[0], got[b])


def test_translation_equivariance_and_determinism():
    ny, nx = 40, 56
    post = inputs.random_shifted_state((9, ny, nx), 4e-3, seed=12)
    blob = _dev(inputs.gnn_blob(5, R, s_delta=1.0))
    dst = torch.empty((ny, 9, nx), device="cuda")
    gnn.lbm_step_gnn(_dev(inputs.planes_to_rows(post)), dst, 0.7, blob, R)
    again = torch.empty_like(dst)
    gnn.lbm_step_gnn(_dev(inputs.planes_to_rows(post)), again, 0.7, blob, R)
    assert torch.equal(dst, again)
    sy, sx = 5, 11                                     # not multiples of the 16-node tile
    shifted = np.roll(post, (sy, sx), axis=(1, 2))
    dst2 = torch.empty_like(dst)
    gnn.lbm_step_gnn(_dev(inputs.planes_to_rows(shifted)), dst2, 0.7, blob, R)
    assert torch.equal(torch.roll(dst, (sy, sx), dims=(0, 2)), dst2)


def test_receptive_field_is_three_nodes():
    """One streaming step plus two rounds: a change at one source node can
    only reach destination nodes within Chebyshev distance 3."""
    ny, nx = 32, 32
    post = inputs.random_shifted_state((9, ny, nx), 4e-3, seed=13)
    blob = _dev(inputs.gnn_blob(6, R, s_delta=1.0))
    a = torch.empty((ny, 9, nx), device="cuda")
    gnn.lbm_step_gnn(_dev(inputs.planes_to_rows(post)), a, 0.7, blob, R)
    pert = post.copy()
    pert[:, 16, 16] += 1e-3
    b = torch.empty_like(a)
    gnn.lbm_step_gnn(_dev(inputs.planes_to_rows(pert)), b, 0.7, blob, R)
    diff = (a != b).any(dim=1).cpu().numpy()          # [ny, nx]
    ys, xs = np.nonzero(diff)
    assert diff[16, 16]
    assert np.abs(ys - 16).max() <= 3 and np.abs(xs - 16).max() <= 3
    assert diff[13:20, 13:20].sum() > 30              # the ball is actually reached


# --------------------------------------------------------------- fallback ---

def _gate_case(orc, blob, thr, poison=False):
    ny, nx = 20, 28
    post = inputs.random_shifted_state((9, ny, nx), 3e-3, seed=31)
    if poison:
        post[4, 3, 5] = np.nan
    src = _dev(inputs.planes_to_rows(post))
    w = _w(orc)
    mass0 = float((post.astype(np.float64) + w).sum()) if not poison else float(ny * nx)
    fb = gnn.Fallback(mass0, thr)
    dst = torch.empty_like(src)
    gnn.lbm_step_gnn(src, dst, 0.7, _dev(blob), R, fallback=fb)
    ref = torch.empty_like(src)
    lbm.lbm_step_bgk(src, ref, 0.7)
    torch.cuda.synchronize()
    return post, dst, ref, fb, mass0


def test_fallback_on_negative_populations(orc):
    blob = inputs.gnn_blob(7, R, s_delta=1.0)
    off = inputs.blob_offsets(R)
    o, _ = off["bh"]
    blob[o + 1:o + 10] = np.float32([50, -50, 0, 0, 0, 0, 0, 0, 0])  # delta f far beyond w
    post, dst, ref, fb, _ = _gate_case(orc, blob, 1e-6)
    assert int(fb.flags.item()) & 1
    assert int(fb.n_fallback.item()) == 1
    assert torch.equal(dst, ref)
    fpre = orc.stream(post.astype(np.float64) + _w(orc))
    _, oflags, omass = orc.gnn_collide_gated(fpre, 0.7, blob.astype(np.float64), 1e-6,
                                             float(fpre.sum()), R)
    assert oflags & 1
    assert abs(fb.mass.item() - omass) / omass < 1e-9


def test_fallback_on_drift_threshold(orc):
    blob = inputs.gnn_blob(8, R, s_delta=1e-4)
    _, dst, ref, fb, _ = _gate_case(orc, blob, -1.0)
    assert int(fb.flags.item()) == 2
    assert int(fb.n_fallback.item()) == 1
    assert torch.equal(dst, ref)


def test_no_fallback_keeps_corrected_step_and_updates_mass(orc):
    blob = inputs.gnn_blob(9, R, s_delta=1e-4)
    post, dst, ref, fb, mass0 = _gate_case(orc, blob, 1e-6)
    assert int(fb.flags.item()) == 0 and int(fb.n_fallback.item()) == 0
    assert not torch.equal(dst, ref)
    got = inputs.rows_to_planes(dst.double().cpu().numpy()) + _w(orc)
    assert abs(fb.mass.item() - got.sum()) / got.sum() < 1e-12
    # projection: the corrected collision conserves mass to FP32 roundoff
    assert abs(fb.mass.item() - mass0) / mass0 < 1e-6


def test_fallback_on_non_finite_source(orc):
    blob = inputs.gnn_blob(10, R, s_delta=1e-4)
    _, dst, ref, fb, _ = _gate_case(orc, blob, 1e-6, poison=True)
    assert int(fb.flags.item()) & 1
    assert torch.equal(torch.nan_to_num(dst, nan=7.0), torch.nan_to_num(ref, nan=7.0))


@pytest.mark.parametrize("net", ["message_passing", "fig2"])
def test_gate_over_many_workgroups_step_after_step(orc, net):
    """The gate on a 384 x 512 lattice, where the corrected step runs 512
    workgroups and the fallback 768, for three steps in a row: kept, forced
    to fall back (negative threshold), kept.  Each step's decision is taken
    by whichever workgroup finishes last, found by counting arrivals, so the
    counts must start from zero at every step.  After each step the recorded
    mass equals the sum of what was stored (in the kernel's order of
    summation), the flags and the fallback count are those of the steps so
    far, and the fallback step's output is the plain BGK step's value for
    value."""
    ny, nx = 384, 512
    post = inputs.random_shifted_state((9, ny, nx), 3e-3, seed=41)
    a = _dev(inputs.planes_to_rows(post))
    b = torch.empty_like(a)
    w = _w(orc)
    if net == "fig2":
        blob = _dev(inputs.gnn_blob(12, 0, s_delta=1e-4))
        step = lambda s, d, fb: gnn.lbm_step_simple(s, d, 0.7, blob, fallback=fb)
    else:
        blob = _dev(inputs.gnn_blob(11, R, s_delta=1e-4))
        step = lambda s, d, fb: gnn.lbm_step_gnn(s, d, 0.7, blob, R, fallback=fb)
    fb = gnn.Fallback(float((post.astype(np.float64) + w).sum()), 1e-6)
    ref = torch.empty_like(a)
    for k, thr in enumerate((1e-6, -1.0, 1e-6)):
        fb.threshold = thr
        step(a, b, fb)
        lbm.lbm_step_bgk(a, ref, 0.7)
        torch.cuda.synchronize()
        g = inputs.rows_to_planes(b.cpu().numpy())
        if net == "fig2" and thr > 0:
            # the fused step adds each node's nine stored values in FP32
            # (in direction order) before its FP64 partial sum
            node = np.zeros(g.shape[1:], np.float32)
            for i in range(9):
                node = (node + g[i]).astype(np.float32)
            expect = ny * nx + node.astype(np.float64).sum()
        else:
            expect = ny * nx + g.astype(np.float64).sum()
        assert abs(fb.mass.item() - expect) / expect < 1e-12, k
        assert int(fb.n_fallback.item()) == (0 if k == 0 else 1), k
        assert int(fb.flags.item()) == (0 if k == 0 else 2), k
        if thr < 0:
            assert torch.equal(b, ref)
        else:
            assert not torch.equal(b, ref)
        a, b = b, a


@pytest.mark.parametrize("net", ["message_passing", "fig2"])
def test_gate_mass_does_not_depend_on_the_work_order(net):
    """The corrected steps hand out tiles and chunks to whichever workgroup or
    wave is free, so which partial sum a node's mass lands in changes from run
    to run; the gate's total is accumulated in exact fixed point, so the same
    state gives the same recorded mass, bit for bit, and the same output.
    Eight repetitions of one gated step on a 384 x 512 lattice."""
    ny, nx = 384, 512
    post = inputs.random_shifted_state((9, ny, nx), 3e-3, seed=43)
    a = _dev(inputs.planes_to_rows(post))
    if net == "fig2":
        blob = _dev(inputs.gnn_blob(12, 0, s_delta=1e-4))
        step = lambda d, fb: gnn.lbm_step_simple(a, d, 0.7, blob, fallback=fb)
    else:
        blob = _dev(inputs.gnn_blob(11, R, s_delta=1e-4))
        step = lambda d, fb: gnn.lbm_step_gnn(a, d, 0.7, blob, R, fallback=fb)
    mass0 = float(inputs.rows_to_planes(a.double().cpu().numpy()).sum()) + ny * nx
    masses, outs = [], []
    for _ in range(8):
        fb = gnn.Fallback(mass0, 1e-6)
        d = torch.empty_like(a)
        step(d, fb)
        torch.cuda.synchronize()
        assert int(fb.n_fallback.item()) == 0
        masses.append(fb.mass.item())
        outs.append(d)
    assert all(m == masses[0] for m in masses), masses
    assert all(torch.equal(o, outs[0]) for o in outs)


# ------------------------------------------------------ full-size sample ---

@pytest.mark.parametrize("ny,nx", [(1004, 2008), (1001, 1950)])
def test_ragged_lattice_with_counter_drawn_tiles_sampled_nodes(orc, ny, nx):
    """Ragged lattices whose work is mostly drawn from the counters.
    1004 x 2008: the last tile column is half wide (2008 = 125 x 16 + 8), the
    last tile row half high (1004 = 125 x 8 + 4), 15,876 tiles per round.
    1001 x 1950: the last tile row is one node high and the last column 14
    wide; the encoder's 31 chunks per row make 31,031 chunks, whose eight
    parts (3,879 and 3,878 chunks) each end in a batch of fewer than four.
    300 random nodes, every node of the corner tile and the four corners,
    against the oracle evaluated on their own neighbourhoods."""
    post = inputs.random_shifted_state((9, ny, nx), 3e-3, seed=47)
    a = _dev(inputs.planes_to_rows(post))
    b = torch.full_like(a, float("nan"))
    blob = inputs.gnn_blob(13, R, s_delta=1e-4)
    gnn.lbm_step_gnn(a, b, 0.7, _dev(blob), R)
    torch.cuda.synchronize()
    assert not torch.isnan(b).any().item()
    fpre = orc.stream(post.astype(np.float64) + _w(orc))
    rng = np.random.default_rng(ny)
    ty0, tx0 = ny - (ny % 8 or 8), nx - (nx % 16 or 16)
    corner = [(y, x) for y in range(ty0, ny) for x in range(tx0, nx)]
    nodes = np.concatenate([rng.integers(0, nx * ny, 300),
                            np.array([y * nx + x for y, x in corner]),
                            np.array([0, nx - 1, nx * ny - 1, nx * (ny - 1)])])
    ref, _ = orc.gnn_collide_nodes(fpre, 0.7, blob.astype(np.float64), nodes, R, mode=0)
    ys, xs = nodes // nx, nodes % nx
    got = b.double()[torch.as_tensor(ys), :, torch.as_tensor(xs)].cpu().numpy() + _w(orc)[:, 0, 0]
    bgk = np.stack([orc.collide_bgk(fpre[:, y:y + 1, x:x + 1], 0.7)[:, 0, 0]
                    for y, x in zip(ys, xs)])
    rel = _rel(got, ref)
    node_c = _node_max(got - bgk, ref - bgk)
    print(f"{ny} x {nx} sampled: f* rel-L2 {rel:.2e}, correction per node {node_c:.2e}")
    assert rel <= 1e-3
    assert node_c <= 5e-2


def test_inference_workload_2048_sampled_nodes(orc):
    """The 2048^2 inference workload in the benchmark's launch configuration:
    100 BGK steps of Taylor-Green (Re = 1000, u0 = 0.04), then one corrected
    step; 256 random nodes checked against the oracle evaluated on their own
    neighbourhoods."""
    n, u0 = 2048, 0.04
    _, tau = inputs.tgv_params(n, u0, 1000.0)
    tau = float(np.float32(tau))
    rho, ux, uy = inputs.tgv_velocity(n, n, u0, dtype=np.float32)
    blob = inputs.gnn_blob(0, R, s_delta=1e-4, u0=u0)
    lat = gnn.GnnLattice(n, n, _dev(blob), R).init(rho, ux, uy)
    lat.step_bgk(tau, 100)
    src = lat.a.clone()
    lat.step_gnn(tau, 1)
    torch.cuda.synchronize()
    assert int(lat.n_fallback.item()) == 0
    post = inputs.rows_to_planes(src.double().cpu().numpy()) + _w(orc)
    fpre = orc.stream(post)
    rng = np.random.default_rng(2048)
    nodes = rng.integers(0, n * n, 256)
    nodes[:4] = [0, n - 1, n * n - 1, n * (n - 1)]    # corners: wrap in x and y
    ref, zref = orc.gnn_collide_nodes(fpre, tau, blob.astype(np.float64), nodes, R, mode=0)
    out = lat.a.double()
    ys, xs = nodes // n, nodes % n
    got = out[torch.as_tensor(ys), :, torch.as_tensor(xs)].cpu().numpy() + _w(orc)[:, 0, 0]
    rel = _rel(got, ref)
    bgk = np.stack([orc.collide_bgk(fpre[:, y:y + 1, x:x + 1], tau)[:, 0, 0]
                    for y, x in zip(ys, xs)])
    rel_c = _rel(got - bgk, ref - bgk)
    node_c = _node_max(got - bgk, ref - bgk)
    print(f"2048^2 sampled: f* rel-L2 {rel:.2e}, correction rel-L2 {rel_c:.2e}, "
          f"per node {node_c:.2e}")
    assert rel <= 1e-3
    assert rel_c <= 5e-2
    assert node_c <= 5e-2
