"""Accuracy experiments on the GPU: plain BGK against the GNN-corrected
collision on the paper's Taylor-Green studies ("Taylor-Green Vortex
Validation", "Resolution Study" with the convergence rate of Eq. 6,
"Reynolds Number Study"), and at equal velocity error.  The velocity error
is the relative L2 norm over all nodes and both components; the energy is
half the sum of |u|^2 over the nodes.

The reference is an FP64 BGK run on a fine lattice (n_fine), restricted to
each coarse lattice at equal physical time (acoustic scaling: one coarse
step on a lattice n_fine/c spans c fine steps).  Every run starts on the slow
manifold (Chapman-Enskog state carrying the Taylor-Green pressure), so that
what is compared is the discretisation, not start-up transients.  All stepping, moments
and restriction run in liblbmgnn.so.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import gnn, inputs, lbm
from .train import tgv_fields


def _tau(u0, re, n):
    return 3.0 * u0 * n / re + 0.5


def _velocity(g32: torch.Tensor):
    _, ux, uy, _ = lbm.lbm_moments(g32, fields=True, sums=False)
    return ux, uy


def _rel_err(ux, uy, rx, ry):
    num = ((ux.double() - rx) ** 2 + (uy.double() - ry) ** 2).sum()
    den = (rx ** 2 + ry ** 2).sum()
    return math.sqrt((num / den).item())


def fine_reference(u0, re, phase, n_fine, coarse_sizes, times_fine):
    """Velocity fields of an FP64 run restricted onto each coarse lattice:
    {n: {t_fine: (ux, uy) float64}}."""
    tau_f = _tau(u0, re, n_fine)
    lat = lbm.Lattice(n_fine, n_fine, dtype=torch.float64).init_ce(
        *tgv_fields(n_fine, u0, phase), tau_f)
    out = {n: {} for n in coarse_sizes}
    done = 0
    for t in sorted(times_fine):
        lat.step_bgk(tau_f, t - done, graph=True)
        done = t
        for n in coarse_sizes:
            c = n_fine // n
            gc = lbm.lbm_restrict(lat.a, c, tau_f, _tau(u0, re, n), pull=False, unstream=False)
            vx, vy = _velocity(gc)
            out[n][t] = (vx.double(), vy.double())
    return out


def coarse_run(n, u0, re, phase, steps_list, blob=None, rounds=2):
    """Velocity of a coarse run at the given step counts; BGK when blob is
    None.  Returns ({steps: (ux, uy)}, fallback count, seconds)."""
    fields = tgv_fields(n, u0, phase, np.float32)
    tau = float(np.float32(_tau(u0, re, n)))
    if blob is None:
        lat = lbm.Lattice(n, n).init_ce(*fields, tau)
    else:
        lat = gnn.GnnLattice(n, n, blob, rounds).init_ce(*fields, tau)
    res, done = {}, 0
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    ms = 0.0
    for s in sorted(steps_list):
        t0.record()
        if blob is None:
            lat.step_bgk(tau, s - done, graph=True)
        else:
            lat.step_gnn(tau, s - done, graph=True)
        t1.record()
        torch.cuda.synchronize()
        ms += t0.elapsed_time(t1)
        done = s
        res[s] = _velocity(lat.a)
    fb = int(lat.n_fallback.item()) if blob is not None else 0
    return res, fb, ms * 1e-3


def fixed_error_report(blob, rounds=2, u0=0.04, re=2000.0, phase=(0.25, 0.4), n_fine=512,
                       n_gnn=128, bgk_sizes=(16, 32, 64, 128, 256), coarse_steps=(256, 512, 1024),
                       mlups_bgk=None, mlups_gnn=None):
    """Velocity errors of the trained GNN at n_gnn and of BGK on a ladder of
    lattices (coarser and finer than n_gnn) against the restricted FP64
    reference, the smallest BGK lattice at least as accurate as the GNN at
    the last time, and the time each needs to reach it, projected from the
    large-lattice MLUPS when given.  Every lattice of the ladder divides
    n_fine, and its step counts m * n / n_gnn are whole, so that all runs are
    compared at the same physical times."""
    for n in bgk_sizes:
        if n_fine % n or any(m * n % n_gnn for m in coarse_steps):
            raise ValueError(f"lattice {n} does not divide the fine lattice or the step counts")
    sizes = sorted(set(bgk_sizes) | {n_gnn})
    times = sorted({m * (n_fine // n_gnn) for m in coarse_steps})
    ref = fine_reference(u0, re, phase, n_fine, sizes, times)
    rep = {"u0": u0, "re": re, "n_fine": n_fine, "coarse_steps_at_n_gnn": list(coarse_steps),
           "errors": {}, "fallback_steps": 0}
    gsteps = list(coarse_steps)
    gres, fb, gsec = coarse_run(n_gnn, u0, re, phase, gsteps, blob, rounds)
    rep["fallback_steps"] = fb
    rep["errors"][f"gnn_{n_gnn}"] = [
        _rel_err(*gres[m], *ref[n_gnn][m * (n_fine // n_gnn)]) for m in gsteps]
    secs = {f"gnn_{n_gnn}": gsec}
    for n in bgk_sizes:
        steps = [m * n // n_gnn for m in coarse_steps]
        bres, _, bsec = coarse_run(n, u0, re, phase, steps)
        rep["errors"][f"bgk_{n}"] = [
            _rel_err(*bres[s], *ref[n][s * (n_fine // n)]) for s in steps]
        secs[f"bgk_{n}"] = bsec
    rep["measured_seconds"] = secs
    # smallest BGK lattice at least as accurate as the GNN at the last time
    e_g = rep["errors"][f"gnn_{n_gnn}"][-1]
    match = [n for n in bgk_sizes if rep["errors"][f"bgk_{n}"][-1] <= e_g]
    rep["bgk_lattice_at_gnn_error"] = min(match) if match else None
    if mlups_bgk and mlups_gnn:
        last = coarse_steps[-1]
        proj = {f"gnn_{n_gnn}": n_gnn * n_gnn * last / (mlups_gnn * 1e6)}
        for n in bgk_sizes:
            proj[f"bgk_{n}"] = n * n * (last * n // n_gnn) / (mlups_bgk * 1e6)
        rep["projected_seconds_at_large_lattice_mlups"] = proj
    return rep


# Regimes of the fixed-error comparison: (name, fine lattice, coarsening
# factor, training Reynolds-number range, test Reynolds number, coarse steps
# of the test window, BGK ladder).  Acoustic scaling throughout (u0 in
# [0.02, 0.06] for training, 0.04 for the test); from a well resolved vortex
# (128^2) to one resolved by 16 nodes, where plain BGK is 1e-3 off.
FIXED_ERROR_REGIMES = (
    ("128_from_512_re2000", 512, 4, (1000.0, 5000.0), 2000.0, (256, 512, 1024),
     (16, 32, 64, 128, 256)),
    ("32_from_128_re2000", 128, 4, (1000.0, 5000.0), 2000.0, (64, 128, 256), (8, 16, 32, 64)),
    ("32_from_128_re200", 128, 4, (100.0, 500.0), 200.0, (64, 128, 256), (8, 16, 32, 64)),
    ("32_from_256_re200", 256, 8, (100.0, 500.0), 200.0, (64, 128, 256), (8, 16, 32, 64, 128)),
    ("16_from_128_re100", 128, 8, (50.0, 250.0), 100.0, (32, 64, 128), (8, 16, 32, 64)),
)


def fixed_error_regimes(regimes=FIXED_ERROR_REGIMES, ghost_weights=(1.0, 1e-2),
                        rounds_list=(2, 0)):
    """The fixed-error comparison over several regimes.  For each regime the
    training pairs are generated on its own lattices (fine n_fine, coarse
    n_fine / factor, training Reynolds range), both networks are trained on
    Eq. 4 (ghost weight 1) and with the residual's non-hydrodynamic moments
    down-weighted (train.moment_weighted_q), and each trained network's
    rollout error at the coarse lattice is set against BGK on the ladder."""
    from . import train
    out = []
    for name, nf, fac, rer, re, steps, ladder in regimes:
        nc = nf // fac
        cfg = train.DataConfig(n_fine=nf, factor=fac, re_range=rer, coarse_steps=steps[-1])
        data = train.datasets(cfg)
        row = {"regime": name, "n_coarse": nc, "n_fine": nf, "re": re,
               "coarse_steps": list(steps), "runs": []}
        bgk = None
        for wg in ghost_weights:
            q = None if wg == 1.0 else train.moment_weighted_q(wg)
            for rounds in rounds_list:
                tr, rep = train.train(cfg, steps=2000, batch=32, rounds=rounds, data=data, loss_q=q)
                fe = fixed_error_report(tr.blob, rounds=rounds, re=re, n_fine=nf, n_gnn=nc,
                                        bgk_sizes=ladder, coarse_steps=steps)
                if bgk is None:
                    bgk = {k: v for k, v in fe["errors"].items() if k.startswith("bgk_")}
                row["runs"].append({
                    "network": "message-passing" if rounds else "fig2", "ghost_weight": wg,
                    "heldout_loss_over_bgk": rep["heldout_rel_loss_after"],
                    "gnn_errors": fe["errors"][f"gnn_{nc}"],
                    "fallback_steps": fe["fallback_steps"],
                    "bgk_lattice_at_gnn_error": fe["bgk_lattice_at_gnn_error"]})
        row["bgk_errors"] = bgk
        out.append(row)
    return out


def head_ablation(blob, rounds=2, u0=0.04, re=2000.0, phase=(0.25, 0.4), n_fine=512,
                  n_gnn=128, coarse_steps=(250, 500, 1000)):
    """Which head of the trained network moves the rollout error: the same
    fixed-error runs as fixed_error_report with the network as trained, with
    its relaxation-time head switched off (row 0 of Wh and bh[0] zeroed:
    z0 = 0, tau_adj = 1 exactly) and with its population correction switched
    off (s_delta = 0), against the same restricted FP64 reference."""
    times = sorted({m * (n_fine // n_gnn) for m in coarse_steps})
    ref = fine_reference(u0, re, phase, n_fine, [n_gnn], times)
    offs = inputs.blob_offsets(rounds)
    no_tau = blob.clone()
    o_wh, (_, wh_cols) = offs["Wh"]
    o_bh, _ = offs["bh"]
    no_tau[o_wh:o_wh + wh_cols] = 0.0
    no_tau[o_bh] = 0.0
    no_df = blob.clone()
    no_df[offs["s_delta"][0]] = 0.0
    out = {"u0": u0, "re": re, "coarse_steps": list(coarse_steps)}
    for name, b in (("trained", blob), ("tau_head_off", no_tau), ("delta_f_off", no_df)):
        res, fb, _ = coarse_run(n_gnn, u0, re, phase, list(coarse_steps), b, rounds)
        out[name] = {"errors": [_rel_err(*res[m], *ref[n_gnn][m * (n_fine // n_gnn)])
                                for m in coarse_steps], "fallback_steps": fb}
    return out



def long_rollout(blob, rounds=2, n=2048, u0=0.05, re=1e4, steps=20000, sample_every=2000,
                 n_sample=256, threshold=1e-6, reference=None, nodes=()):
    """Long Taylor-Green rollout at high Reynolds number (uniform density, f
    at equilibrium at t = 0) with the corrected collision and the per-step
    fallback gate, or with plain BGK when blob is None.  Every
    `sample_every` steps the velocity field is restricted by injection to
    n_sample^2 (every (n / n_sample)-th node) and its kinetic energy
    1/2 sum |u|^2 is compared with
      - `reference`: rows (step, energy, mass, ...) of the FP64 oracle's
        plain-BGK run of the same flow on the same restriction, when given
        (the error of the energy and of its decay E(t) / E(0));
      - the analytic decay E(0) exp(-4 nu k^2 t), nu = (tau - 1/2) / 3.
    Mass and momentum are summed in FP64 by lbm_moments (drift relative to
    the initial state).  `nodes`: (y, x) lattice nodes whose velocity is
    reported at every sample."""
    tau32 = float(np.float32(_tau(u0, re, n)))
    rho, ux, uy = inputs.tgv_velocity(n, n, u0, dtype=np.float32)
    if blob is None:
        lat = lbm.Lattice(n, n).init(rho, ux, uy)
    else:
        lat = gnn.GnnLattice(n, n, blob, rounds, threshold).init(rho, ux, uy)
    c = n // n_sample
    ref = None if reference is None else {int(r[0]): r for r in np.asarray(reference)}
    nu = (tau32 - 0.5) / 3.0
    k2 = (2.0 * math.pi / n) ** 2
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    ny_, nx_ = (torch.as_tensor([p[0] for p in nodes], dtype=torch.long),
                torch.as_tensor([p[1] for p in nodes], dtype=torch.long))

    def sample(step):
        _, gx, gy, sums = lat.moments(fields=True)
        s = sums.cpu().numpy()
        sx, sy = gx[::c, ::c].double(), gy[::c, ::c].double()
        row = {"step": step, "energy": 0.5 * float((sx * sx + sy * sy).sum().item()),
               "mass": float(s[0]), "momentum": [float(s[1]), float(s[2])],
               "min_f": float(s[6]), "n_negative": int(s[7])}
        if nodes:
            row["node_velocity"] = torch.stack([gx.cpu()[ny_, nx_], gy.cpu()[ny_, nx_]],
                                               1).double().tolist()
        if blob is not None:
            row["fallback_steps"] = int(lat.n_fallback.item())
        return row

    rows = [sample(0)]
    done, ms = 0, 0.0
    while done < steps:
        k = min(sample_every, steps - done)
        e0.record()
        if blob is None:
            lat.step_bgk(tau32, k)
        else:
            lat.step_gnn(tau32, k)
        e1.record()
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        done += k
        rows.append(sample(done))
    E0, M0 = rows[0]["energy"], rows[0]["mass"]
    for r in rows:
        t = r["step"]
        ea = E0 * math.exp(-4.0 * nu * k2 * t)
        r["energy_err_vs_analytic"] = abs(r["energy"] - ea) / ea
        r["mass_drift"] = abs(r["mass"] - M0) / M0
        if ref is not None and t in ref:
            er, er0 = float(ref[t][1]), float(ref[0][1])
            r["energy_err_vs_oracle"] = abs(r["energy"] - er) / er
            r["decay_err_vs_oracle"] = abs(r["energy"] / E0 - er / er0) / (er / er0)
    out = {"n": n, "u0": u0, "re": re, "tau": tau32, "steps": steps, "n_sample": n_sample,
           "collision": "bgk" if blob is None else ("fig2-network" if rounds == 0
                                                    else "message-passing"),
           "mlups": n * n * steps / (ms * 1e-3) / 1e6, "ms_per_step": ms / steps,
           "samples": rows,
           "max_mass_drift": max(r["mass_drift"] for r in rows)}
    if ref is not None:
        errs = [r["energy_err_vs_oracle"] for r in rows if "energy_err_vs_oracle" in r]
        out["max_energy_err_vs_oracle"] = max(errs) if errs else None
        out["energy_err_vs_oracle_at_end"] = rows[-1].get("energy_err_vs_oracle")
    if blob is not None:
        out["fallback_steps"] = rows[-1]["fallback_steps"]
    return out


def _analytic(n, u0, tau32, t):
    """Decaying Taylor-Green field of a run whose relaxation time is tau32:
    nu = (tau - 1/2) / 3, amplitude factor exp(-2 nu k^2 t)."""
    k = 2.0 * math.pi / n
    return (u0, k, k, 0.0, 0.0, (tau32 - 0.5) / 3.0, float(t))


def tgv_state_errors(g32, n, u0, tau32, t):
    """Velocity and energy errors of a lattice state against the analytic
    Taylor-Green field at step t, plus its smallest population and number of
    negative populations (all from the FP64 sums of lbm_moments)."""
    _, _, _, sums = lbm.lbm_moments(g32, analytic=_analytic(n, u0, tau32, t))
    s = sums.cpu().numpy()
    e_a = 0.5 * s[5]
    finite = bool(np.isfinite(s).all())
    return {"vel_err": float(math.sqrt(s[4] / s[5])) if finite else float("nan"),
            "energy_err": float(abs(s[3] - e_a) / e_a) if finite else float("nan"),
            "energy": float(s[3]), "min_f": float(s[6]), "n_negative": int(s[7]),
            "finite": finite}


def _lattice(n, u0, tau32, blob, rounds, fp64=False):
    if fp64:
        return lbm.Lattice(n, n, dtype=torch.float64).init_ce(
            *tgv_fields(n, u0, (0.0, 0.0)), tau32)
    fields = tgv_fields(n, u0, (0.0, 0.0), np.float32)
    if blob is None:
        return lbm.Lattice(n, n).init_ce(*fields, tau32)
    return gnn.GnnLattice(n, n, blob, rounds).init_ce(*fields, tau32)


def _fp32_view(lat, tau):
    """FP32 populations with the lattice's density and velocity (an FP64
    lattice goes through the factor-1 restriction, which keeps rho and u)."""
    if lat.a.dtype == torch.float32:
        return lat.a
    return lbm.lbm_restrict(lat.a, 1, tau, tau, pull=False, unstream=False)


def _advance(lat, blob, tau32, k):
    # small lattices: whole chunks of steps replayed from captured HIP graphs
    if blob is None:
        lat.step_bgk(tau32, k, graph=True)
    else:
        lat.step_gnn(tau32, k, graph=True)


def resolution_study(blob=None, rounds=2, re=100.0, sizes=(32, 64, 128), scaling="diffusive",
                     u0_ref=0.04, n_ref=64, steps_ref=1000, fp64=False):
    """Velocity and energy errors against the analytic vortex at equal
    physical time on several lattices, and the observed order of Eq. 6
    between neighbouring sizes, alpha = log(E1/E2) / log(h1/h2), h = 1/n.

    scaling "acoustic" keeps u0 (the Mach number) and takes steps in
    proportion to n; "diffusive" takes u0 = u0_ref n_ref / n (fixed lattice
    viscosity) and steps in proportion to n^2.  Every run starts on the slow
    manifold (Chapman-Enskog state with the Taylor-Green pressure).  BGK when
    blob is None, else the corrected collision with the fallback gate.  With
    fp64 the BGK runs use FP64 populations, which separates the method's
    discretisation error from FP32 rounding on long fine-lattice runs."""
    if scaling not in ("acoustic", "diffusive"):
        raise ValueError("scaling must be 'acoustic' or 'diffusive'")
    if fp64 and blob is not None:
        raise ValueError("the corrected collision runs in FP32 only")
    rows = []
    for n in sizes:
        if scaling == "acoustic":
            u0, steps = u0_ref, steps_ref * n // n_ref
        else:
            u0, steps = u0_ref * n_ref / n, steps_ref * n * n // (n_ref * n_ref)
        tau32 = float(np.float32(_tau(u0, re, n)))
        lat = _lattice(n, u0, tau32, blob, rounds, fp64)
        _advance(lat, blob, tau32, steps)
        row = {"n": n, "u0": u0, "tau": tau32, "steps": steps}
        row.update(tgv_state_errors(_fp32_view(lat, tau32), n, u0, tau32, steps))
        if blob is not None:
            row["fallback_steps"] = int(lat.n_fallback.item())
        rows.append(row)
    alpha = []
    for a, b in zip(rows, rows[1:]):
        ok = a["vel_err"] > 0 and b["vel_err"] > 0 and a["finite"] and b["finite"]
        alpha.append(math.log(a["vel_err"] / b["vel_err"]) / math.log(b["n"] / a["n"])
                     if ok else float("nan"))
    return {"re": re, "scaling": scaling, "fp64": fp64, "rows": rows, "alpha": alpha}


def tgv_validation(blob=None, rounds=2, n=64, re=100.0, u0=0.04, checkpoints=(1000, 3000, 5000),
                   start="equilibrium"):
    """Velocity (L2, R5) and energy errors against the analytic vortex at the
    given step counts on one lattice (the validation section's table of
    errors at 1000, 3000 and 5000 steps, 64^2, Re = 100).  start
    "equilibrium": f = f^eq(1, u) with uniform density (the workload's
    definition), which launches an acoustic transient the error then
    carries; "slow": the Chapman-Enskog state with the Taylor-Green pressure.
    BGK when blob is None, else the corrected collision with the gate."""
    if start not in ("equilibrium", "slow"):
        raise ValueError("start must be 'equilibrium' or 'slow'")
    tau32 = float(np.float32(_tau(u0, re, n)))
    if start == "slow":
        lat = _lattice(n, u0, tau32, blob, rounds)
    else:
        rho, ux, uy = inputs.tgv_velocity(n, n, u0, dtype=np.float32)
        lat = (lbm.Lattice(n, n) if blob is None else gnn.GnnLattice(n, n, blob, rounds))
        lat.init(rho, ux, uy)
    rows, done = [], 0
    for t in sorted(checkpoints):
        _advance(lat, blob, tau32, t - done)
        done = t
        row = {"steps": t}
        row.update(tgv_state_errors(lat.a, n, u0, tau32, t))
        if blob is not None:
            row["fallback_steps"] = int(lat.n_fallback.item())
        rows.append(row)
    return {"n": n, "re": re, "u0": u0, "tau": tau32, "start": start, "rows": rows}


def fast_relaxation_nodes(g32: torch.Tensor, tau32: float, blob, rounds: int) -> int:
    """Number of nodes of a (post-collision) state whose next corrected
    collision relaxes faster than omega = 2, i.e. tau * tau_adj < 1/2 with
    tau_adj = 1/2 + sigmoid(z_0) from the network's head (no clamp is
    applied to tau_adj; the fallback gate catches what such nodes do)."""
    pre = lbm.lbm_stream(g32)[None]
    tau_t = torch.full((1,), tau32, dtype=torch.float32, device=g32.device)
    _, z = gnn.collide(pre, tau_t, blob, rounds, want_z=True)
    tau_adj = 0.5 + torch.sigmoid(z[..., 0].double())
    return int((tau32 * tau_adj < 0.5).sum().item())


def stability_sweep(blob=None, rounds=2, n=64, u0=0.04,
                    re_list=(100, 200, 400, 800, 1600, 3200), steps=20000, every=1000):
    """Taylor-Green runs on an n^2 lattice over a range of Reynolds numbers.
    Every `every` steps the state is checked: the first check that finds a
    non-finite or negative population ends the run ("first_bad_step").  The
    corrected collision runs with the per-step fallback gate, so its first
    step that fell back to BGK and the number of such steps are reported as
    well, and at every check the number of nodes whose effective relaxation
    rate exceeds 2 (the most found at any check, and at the last).  Energy
    and velocity errors are against the analytic decay at the last step
    reached."""
    out = []
    for re in re_list:
        tau32 = float(np.float32(_tau(u0, re, n)))
        row = {"re": re, "tau": tau32}
        for name, b in (("bgk", None), ("gnn", blob)):
            if name == "gnn" and blob is None:
                continue
            lat = _lattice(n, u0, tau32, b, rounds)
            e0 = tgv_state_errors(lat.a, n, u0, tau32, 0)["energy"]
            done, first_bad, first_fb, st = 0, None, None, None
            fast = []
            while done < steps:
                k = min(every, steps - done)
                _advance(lat, b, tau32, k)
                done += k
                st = tgv_state_errors(lat.a, n, u0, tau32, done)
                if b is not None and st["finite"]:
                    fast.append(fast_relaxation_nodes(lat.a, tau32, b, rounds))
                if b is not None and first_fb is None and int(lat.n_fallback.item()) > 0:
                    first_fb = done
                if not st["finite"] or st["n_negative"] > 0:
                    first_bad = done
                    break
            r = {"steps_run": done, "first_bad_step": first_bad,
                 "energy_ratio": st["energy"] / e0 if st["finite"] else float("nan"),
                 "energy_ratio_analytic": math.exp(-4.0 * (tau32 - 0.5) / 3.0
                                                   * (2.0 * math.pi / n) ** 2 * done),
                 "energy_err": st["energy_err"], "vel_err": st["vel_err"]}
            if b is not None:
                r["fallback_steps"] = int(lat.n_fallback.item())
                r["first_fallback_by_step"] = first_fb
                r["omega_above_2_nodes_max"] = max(fast) if fast else None
                r["omega_above_2_nodes_last"] = fast[-1] if fast else None
            row[name] = r
        out.append(row)
    return {"n": n, "u0": u0, "steps": steps, "check_every": every, "runs": out}


def poiseuille_study(re_list=(10, 50, 100, 200), ny=32, u_max=0.05, nx=4,
                     diffusion_times=4.0, fp64=False, blob=None):
    """Channel flow between resting walls (validation section, "Poiseuille
    Flow", Eq. 5) at several Reynolds numbers Re = u_max ny / nu: each run
    starts at rest and is driven by g = 8 nu u_max / ny^2 for
    `diffusion_times` ny^2 / nu steps (the slowest transient then decays as
    exp(-pi^2 diffusion_times)).  Reports the largest velocity error of the
    x-averaged profile relative to the largest analytic velocity, next to
    the closed-form bounce-back slip of the method.  blob: a zero-round
    (Fig. 2) parameter blob, run with the per-node corrected collision and
    its fallback gate instead of BGK (FP32)."""
    rows = []
    for re in re_list:
        nu = u_max * ny / re
        tau = float(np.float32(3.0 * nu + 0.5))
        nu = (tau - 0.5) / 3.0
        g = float(np.float32(8.0 * nu * u_max / ny ** 2))
        steps = int(math.ceil(diffusion_times * ny * ny / nu))
        if blob is not None:
            lat = gnn.GnnLattice(nx, ny, blob, 0)
            lat.a.zero_()
            lat.sync_mass()
        else:
            lat = lbm.Lattice(nx, ny, dtype=torch.float64 if fp64 else torch.float32)
            lat.a.zero_()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        if blob is not None:
            lat.step_gnn_channel(tau, g, steps, graph=True)
        else:
            lat.step_channel(tau, g, steps, graph=True)
        t1.record()
        torch.cuda.synchronize()
        g32 = lat.a if not fp64 else lbm.lbm_restrict(lat.a, 1, tau, tau, pull=False,
                                                      unstream=False)
        prof = lbm.lbm_channel_profile(g32, g).cpu().numpy()
        y = np.arange(ny)
        ua = g / (2.0 * nu) * (y + 0.5) * (ny - y - 0.5)
        slip = g * (16.0 * (tau - 0.5) ** 2 - 3.0) / (24.0 * nu)
        rows.append({"re": re, "tau": tau, "g": g, "steps": steps,
                     "max_rel_err": float(np.abs(prof - ua).max() / ua.max()),
                     "slip_rel_closed_form": float(slip / ua.max()),
                     "fallback_steps": int(lat.n_fallback.item()) if blob is not None else 0,
                     "seconds": t0.elapsed_time(t1) * 1e-3})
    return {"ny": ny, "nx": nx, "u_max": u_max, "fp64": fp64,
            "collision": "bgk" if blob is None else "fig2-network", "rows": rows}


def poiseuille_refinement(heights=(16, 32, 64), re=100.0, u_max=0.05, fp64=False, blob=None,
                          diffusion_times=4.0):
    """Grid refinement of the channel (the validation section's Poiseuille
    convergence figure): the same flow (Re, u_max) on channels of height H,
    the largest velocity error of each and the observed order between
    neighbouring heights, alpha = log(E1 / E2) / log(H2 / H1)."""
    rows = []
    for h in heights:
        r = poiseuille_study(re_list=(re,), ny=h, u_max=u_max, fp64=fp64, blob=blob,
                             diffusion_times=diffusion_times)["rows"][0]
        r["ny"] = h
        rows.append(r)
    alpha = [round(math.log(a["max_rel_err"] / b["max_rel_err"]) / math.log(b["ny"] / a["ny"]), 3)
             for a, b in zip(rows, rows[1:])]
    return {"re": re, "u_max": u_max, "fp64": fp64,
            "collision": "bgk" if blob is None else "fig2-network", "rows": rows, "alpha": alpha}


def main(argv=None):
    """Runs one study and prints its report as JSON:
    python -m paper_2504_14494_amd.experiments {fixed-error, fixed-error-regimes,
    resolution, stability, poiseuille, poiseuille-refinement, long-rollout,
    tgv-validation}
    [--rounds R].  The corrected-collision
    studies first train the network (train.train, full configuration); the
    Poiseuille study runs a network only with --rounds 0 (the per-node
    network has no neighbours across a wall; message passing has no wall
    treatment)."""
    import argparse
    import json
    import time

    from . import train
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["fixed-error", "fixed-error-regimes", "resolution",
                                      "stability", "poiseuille", "poiseuille-refinement",
                                      "long-rollout", "tgv-validation"])
    ap.add_argument("--rounds", type=int, default=2, help="2: message passing; 0: Fig. 2")
    ap.add_argument("--scaling", default="diffusive", choices=["diffusive", "acoustic"])
    ap.add_argument("--fp64", action="store_true", help="BGK runs in FP64 (resolution, poiseuille)")
    ap.add_argument("--steps", type=int, default=20000, help="long-rollout steps")
    ap.add_argument("--reference", default="",
                    help="long rollout: file of the FP64 oracle's energies (step, energy, ...) "
                         "on the same restriction")
    args = ap.parse_args(argv)
    t0 = time.perf_counter()
    blob = None
    if args.study in ("fixed-error", "stability", "long-rollout", "tgv-validation") or (
            args.study == "resolution" and not args.fp64) or (
            args.study in ("poiseuille", "poiseuille-refinement") and args.rounds == 0
            and not args.fp64):
        tr, rep = train.train(train.DataConfig(), steps=2000, batch=32, rounds=args.rounds)
        blob = tr.blob
    if args.study == "fixed-error":
        out = fixed_error_report(blob, rounds=args.rounds)
    elif args.study == "fixed-error-regimes":
        out = {"regimes": fixed_error_regimes()}
    elif args.study == "resolution":
        out = {"bgk": resolution_study(None, scaling=args.scaling, fp64=args.fp64)}
        if blob is not None:
            out["gnn"] = resolution_study(blob, rounds=args.rounds, scaling=args.scaling)
    elif args.study == "stability":
        out = stability_sweep(blob, rounds=args.rounds)
    elif args.study == "poiseuille":
        out = {"bgk": poiseuille_study(fp64=args.fp64)}
        if blob is not None:
            out["fig2_network"] = poiseuille_study(blob=blob)
    elif args.study == "poiseuille-refinement":
        out = {"bgk": poiseuille_refinement(fp64=args.fp64)}
        if blob is not None:
            out["fig2_network"] = poiseuille_refinement(blob=blob)
    elif args.study == "tgv-validation":
        out = {f"{name}_{start}_start": tgv_validation(b, rounds=args.rounds, start=start)
               for start in ("equilibrium", "slow") for name, b in (("bgk", None), ("gnn", blob))}
    else:
        ref = np.loadtxt(args.reference) if args.reference else None
        out = long_rollout(blob, rounds=args.rounds, steps=args.steps, reference=ref)
    out["wall_seconds"] = round(time.perf_counter() - t0, 1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
