"""Training on data the plain method generates (paper: Training
Methodology): the pair generator against the oracle, bitwise checkpoint
resume, and the gain of the trained collision over plain BGK on held-out
Taylor-Green flows.  Training itself has no unique answer; its acceptance is
the gain (parity unpinned beyond the pieces: forward, backward, loss, Adam
and the data pairs, each checked against the oracle)."""
import dataclasses

import numpy as np
import pytest
import torch

from paper_2504_14494_amd import inputs, train

pytestmark = pytest.mark.gpu


def test_pairs_match_oracle_generated_pairs(orc):
    """Pairs from the library's FP64 runs and restriction against pairs built
    from the oracle's runs: input R(f(4m)), target S_c^-1 R(f(4m + 4)), both
    lattices started on the slow manifold."""
    cfg = train.DataConfig(n_fine=32, factor=4, runs=1, snaps=2, coarse_steps=6, seed=3,
                           coarse_pairs=False)
    u0, re, ph = 0.05, 1500.0, (0.3, 0.7)
    X, Y, tau_c = train.run_pairs(u0, re, ph, cfg)
    tau_f, tc = train.taus(u0, re, 32, 4)
    assert tc == tau_c
    rho, ux, uy = train.tgv_fields(32, u0, ph)
    f0 = orc.init_ce(rho, ux, uy, tau_f)          # pre-collision state at t = 0
    w = orc.lattice()[2][:, None, None]
    for k, m in enumerate(cfg.snapshot_steps()):
        f = orc.bgk_run(f0, tau_f, 4 * m)
        xin = orc.restrict(f, 4, tau_f, tau_c)
        yt = orc.restrict(orc.bgk_run(f, tau_f, 4), 4, tau_f, tau_c, unstream_=True)
        gx = inputs.rows_to_planes(X[k].double().cpu().numpy()) + w
        gy = inputs.rows_to_planes(Y[k].double().cpu().numpy()) + w
        assert np.abs(gx - xin).max() < 1e-7
        assert np.abs(gy - yt).max() < 1e-7


def _small_cfg():
    return train.DataConfig(n_fine=128, factor=4, runs=8, snaps=8, coarse_steps=400, seed=11)


def test_checkpoint_resume_is_bitwise(tmp_path):
    cfg = dataclasses.replace(_small_cfg(), runs=2, snaps=4)
    X, Y, T = train.make_dataset(cfg)
    blob0 = torch.as_tensor(inputs.gnn_blob(0, 2, s_delta=1e-4), device="cuda")
    a = train.Trainer(blob0.clone(), 2, shuffle_seed=5)
    for _ in range(6):
        a.step(X, Y, T, 1e9, batch=3)
    b = train.Trainer(blob0.clone(), 2, shuffle_seed=5)
    for _ in range(3):
        b.step(X, Y, T, 1e9, batch=3)
    path = str(tmp_path / "ck.npz")
    b.save(path)
    c = train.Trainer(torch.zeros_like(blob0), 2, shuffle_seed=99)
    c.load(path)
    for _ in range(3):
        c.step(X, Y, T, 1e9, batch=3)
    assert torch.equal(a.blob, c.blob)
    assert torch.equal(a.m, c.m) and torch.equal(a.v, c.v)


def test_trained_collision_beats_bgk_on_held_out_flows():
    tr, rep = train.train(_small_cfg(), steps=300, batch=16, held_out_runs=4, log_every=50)
    print({k: v for k, v in rep.items() if k != "history"}, rep["history"])
    assert rep["heldout_rel_loss_before"] > 0.5
    assert rep["heldout_rel_loss_after"] < 1.0
    assert rep["train_rel_loss_after"] < 1.0


def test_trained_fig2_network_beats_bgk_on_held_out_flows():
    """The same training (Eq. 4 relative to BGK, Adam) of the paper's Fig. 2
    network: per-node ReLU MLP, zero rounds, fused forward with saved
    activations and the zero-round backward."""
    tr, rep = train.train(_small_cfg(), steps=300, batch=16, rounds=0, held_out_runs=4,
                          log_every=50)
    print({k: v for k, v in rep.items() if k != "history"}, rep["history"])
    assert rep["heldout_rel_loss_before"] > 0.5
    assert rep["heldout_rel_loss_after"] < 1.0
    assert rep["train_rel_loss_after"] < 1.0


def test_rollout_criterion_on_held_out_flows(trained):
    """The training acceptance's rollout half: on held-out Taylor-Green flows
    (drawn like the training runs but from the held-out seed), the trained
    message-passing network's 128^2 rollout error against the restricted
    FP64 512^2 run, next to plain BGK on a ladder of lattices.

    Measured outcome, asserted as such: the network's one-step held-out loss
    is below plain BGK's (other tests), but its rollout is less accurate than
    plain BGK on the same 128^2 lattice, and BGK reaches the network's error
    on a coarser lattice.  The paper's claim that the network buys accuracy at
    coarse resolution is therefore not reproduced here; a change to the method
    or the training that reverses this makes this test fail on purpose."""
    from paper_2504_14494_amd import experiments
    u0s, res, phases = inputs.training_draws(8, train.DataConfig().seed + 1)
    for k in range(2):
        u0, re, ph = float(u0s[k]), float(res[k]), tuple(float(p) for p in phases[k])
        rep = experiments.fixed_error_report(trained[2], u0=u0, re=re, phase=ph)
        e_gnn = rep["errors"]["gnn_128"][-1]
        e_bgk = rep["errors"]["bgk_128"][-1]
        print(f"held-out flow u0={u0:.4f} Re={re:.0f}: network {e_gnn:.3e}, BGK 128^2 {e_bgk:.3e}, "
              f"BGK lattice at the network's error {rep['bgk_lattice_at_gnn_error']}, "
              f"fallbacks {rep['fallback_steps']}")
        assert np.isfinite(e_gnn)
        assert e_gnn > e_bgk
        assert rep["bgk_lattice_at_gnn_error"] is not None
        assert rep["bgk_lattice_at_gnn_error"] < 128


def test_trained_rollout_tracks_the_fp64_oracle_and_its_loss_is_the_networks(orc):
    """A network trained in an under-resolved regime (32^2 coarse from 128^2
    fine, Re in [100, 500]) rolled out for 256 gated steps at Re = 200 by the
    library (BF16 network) and by the oracle (FP64 network, same gate) from
    the identical start state, both against the restricted FP64 128^2 run.

    Rollout-level parity: the two trajectories stay within a tenth of their
    common error (measured 6 %: 9.4e-4 against 1.6e-2 after 256 steps).
    Measured outcome, asserted as such: the FP64 network's rollout error equals
    the BF16 library's within 10 % (measured 3 %) and is over ten times plain
    BGK's on the same lattice (1.3e-4), so the rollout loss of the trained
    network is the function it learned, not its BF16 storage."""
    from paper_2504_14494_amd import experiments, gnn
    cfg = train.DataConfig(n_fine=128, factor=4, re_range=(100.0, 500.0), coarse_steps=256)
    tr, _ = train.train(cfg, steps=2000, batch=32, rounds=2)
    n, u0, re, phase, steps = 32, 0.04, 200.0, (0.25, 0.4), 256
    ref = experiments.fine_reference(u0, re, phase, 128, [n], [4 * steps])
    rx, ry = (t.cpu().numpy() for t in ref[n][4 * steps])
    tau = float(np.float32(experiments._tau(u0, re, n)))
    lat = gnn.GnnLattice(n, n, tr.blob, 2).init_ce(*train.tgv_fields(n, u0, phase, np.float32), tau)
    w = orc.lattice()[2][:, None, None]
    post = inputs.rows_to_planes(lat.a.double().cpu().numpy()) + w
    blob64 = tr.blob.double().cpu().numpy()
    mass, fell = float(post.sum()), 0
    lat.step_gnn(tau, steps)
    for _ in range(steps):
        post, flags, mass = orc.gnn_collide_gated(orc.stream(post), tau, blob64, 1e-6, mass, 2)
        fell += 1 if flags else 0
    _, gx, gy, _ = lat.moments(fields=True)
    gx, gy = gx.double().cpu().numpy(), gy.double().cpu().numpy()
    _, ox, oy = orc.moments(post)
    den = np.sqrt((rx ** 2 + ry ** 2).sum())
    e_lib = np.sqrt(((gx - rx) ** 2 + (gy - ry) ** 2).sum()) / den
    e_o64 = np.sqrt(((ox - rx) ** 2 + (oy - ry) ** 2).sum()) / den
    apart = np.sqrt(((gx - ox) ** 2 + (gy - oy) ** 2).sum()) / den
    bgk, _, _ = experiments.coarse_run(n, u0, re, phase, [steps])
    e_bgk = np.sqrt(((bgk[steps][0].double().cpu().numpy() - rx) ** 2
                     + (bgk[steps][1].double().cpu().numpy() - ry) ** 2).sum()) / den
    print(f"256 steps: library {e_lib:.3e}, FP64 oracle {e_o64:.3e}, apart {apart:.3e}, "
          f"BGK {e_bgk:.3e}; fallbacks library {int(lat.n_fallback.item())}, oracle {fell}")
    assert int(lat.n_fallback.item()) == fell == 0
    assert apart <= 0.1 * e_o64
    assert abs(e_lib - e_o64) <= 0.1 * e_o64
    assert e_o64 > 10 * e_bgk
