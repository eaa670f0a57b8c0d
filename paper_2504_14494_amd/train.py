"""Training of the GNN collision on data the plain method generates
(paper: Training Methodology, supervised pairs from high-resolution LBM
runs, loss of Eq. 4).

Data.  Fine FP64 Taylor-Green runs (lattice nf, random amplitude u0, Reynolds
number and phase) are stepped with the library's FP64 BGK kernel.  A coarse
lattice node X sits on fine node factor * X; one coarse step spans `factor`
fine steps at equal Reynolds and Mach numbers (acoustic scaling), so
tau_c = 3 u0 nc / Re + 1/2 while tau_f = 3 u0 nf / Re + 1/2.  For coarse step
m the pair is
    input  = R(pre-collision fine state at fine step factor*m)
    target = S_c^-1 R(pre-collision fine state at fine step factor*(m+1))
where R is the library's restriction (equilibrium of the fine node's density
and velocity plus its non-equilibrium momentum flux rescaled by
factor * tau_c / tau_f) and S_c^-1 undoes one coarse streaming step, so the
target is the coarse post-collision state that streams into the next
restricted state.

Loss.  Eq. 4 with N the number of nodes of the batch, divided by the same
loss of the plain BGK collision over the training set (a constant), so that
the loss is O(1) for Adam and 1 - loss is the gain over BGK.

Every array operation of the method (stepping, restriction, forward,
backward, loss, Adam) runs in liblbmgnn.so; torch provides memory, random
batch indices and host copies only.
"""
from __future__ import annotations

import dataclasses
import json
import os

import numpy as np
import torch

from . import gnn, inputs, lbm


@dataclasses.dataclass
class DataConfig:
    n_fine: int = 512
    factor: int = 4
    runs: int = 32
    snaps: int = 8
    coarse_steps: int = 1000
    u0_range: tuple = (0.02, 0.06)
    re_range: tuple = (1000.0, 5000.0)
    seed: int = 1234
    # also pair states of a coarse plain-BGK run of the same flow with the
    # restricted fine targets (the coarse lattice regressed toward the fine run)
    coarse_pairs: bool = True

    @property
    def n_coarse(self):
        return self.n_fine // self.factor

    def snapshot_steps(self):
        """Coarse steps m >= 1 of the snapshots, spread over the first
        coarse_steps."""
        stride = max(1, self.coarse_steps // self.snaps)
        return [1 + k * stride for k in range(self.snaps)]


def taus(u0: float, re: float, nf: int, factor: int):
    nu_f = u0 * nf / re
    nu_c = u0 * (nf // factor) / re
    return 3.0 * nu_f + 0.5, 3.0 * nu_c + 0.5


def tgv_fields(n: int, u0: float, phase, dtype=np.float64):
    """Taylor-Green density (with its pressure field) and velocity on an n^2
    lattice with the given phase (fractions of the period)."""
    x0, y0 = phase[0] * n, phase[1] * n
    _, ux, uy = inputs.tgv_velocity(n, n, u0, x0=x0, y0=y0, dtype=dtype)
    rho = inputs.tgv_pressure_density(n, n, u0, x0=x0, y0=y0, dtype=dtype)
    return rho, ux, uy


def run_pairs(u0: float, re: float, phase, cfg: DataConfig, device="cuda"):
    """Training pairs of one fine run: (inputs [S, nc, 9, nc], targets, tau_c).

    Both lattices start on the slow manifold (Chapman-Enskog state with the
    Taylor-Green pressure).  After k steps the buffers hold the
    post-collision state P_k, and streaming it gives the pre-collision state
    f_{k+1} at time k + 1; coarse step m spans fine steps 4m..4m+4.  For every
    snapshot m >= 1:
        input  = R(f_fine(4m))                 restricted fine pre-collision state
        target = S_c^-1 R(f_fine(4m + 4))      post-collision state streaming into it
    and, when cfg.coarse_pairs is set, also input = f_coarse(m) of a coarse
    plain-BGK run of the same flow with the same target.  The coarse states
    carry the coarse lattice's own non-hydrodynamic content, which a corrected
    coarse run meets and restricted fine states never show."""
    nf, fac, nc = cfg.n_fine, cfg.factor, cfg.n_coarse
    tau_f, tau_c = taus(u0, re, nf, fac)
    lat = lbm.Lattice(nf, nf, dtype=torch.float64, device=device).init_ce(
        *tgv_fields(nf, u0, phase), tau_f)
    clat = None
    tc32 = float(np.float32(tau_c))
    if cfg.coarse_pairs:
        clat = lbm.Lattice(nc, nc, device=device).init_ce(
            *tgv_fields(nc, u0, phase, np.float32), tc32)
    ins, outs, cins = [], [], []
    done = cdone = 0
    for m in cfg.snapshot_steps():
        lat.step_bgk(tau_f, fac * m - 1 - done, graph=True)  # P_f(4m - 1)
        done = fac * m - 1
        ins.append(lbm.lbm_restrict(lat.a, fac, tau_f, tau_c, pull=True, unstream=False))
        if clat is not None:
            clat.step_bgk(tc32, m - 1 - cdone, graph=True)   # P_c(m - 1)
            cdone = m - 1
            cins.append(lbm.lbm_stream(clat.a))
        lat.step_bgk(tau_f, fac)                            # P_f(4m + 3)
        done += fac
        outs.append(lbm.lbm_restrict(lat.a, fac, tau_f, tau_c, pull=True, unstream=True))
    if clat is not None:
        ins += cins
        outs += outs
    return torch.stack(ins), torch.stack(outs), tau_c


def make_dataset(cfg: DataConfig, device="cuda"):
    """Pairs from cfg.runs fine runs; draws from inputs.training_draws."""
    u0s, res, phases = inputs.training_draws(cfg.runs, cfg.seed)
    X, Y, T = [], [], []
    for u0, re, ph in zip(u0s, res, phases):
        x, y, tc = run_pairs(float(u0), float(re), ph, cfg, device)
        X.append(x)
        Y.append(y)
        T += [tc] * x.shape[0]
    return (torch.cat(X).contiguous(), torch.cat(Y).contiguous(),
            torch.tensor(T, dtype=torch.float32, device=device))


# An orthogonal moment basis of D2Q9 (rows over the directions 0:(0,0)
# 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)):
# density, energy, energy square, x- and y-momentum, the two energy fluxes,
# and the two shear stresses.  The density and momentum rows are conserved by
# the corrected collision; energy and the stresses are hydrodynamic; the
# energy square and the fluxes are non-hydrodynamic ("ghost") moments.
MOMENT_BASIS = np.array([
    [1, 1, 1, 1, 1, 1, 1, 1, 1],
    [-4, -1, -1, -1, -1, 2, 2, 2, 2],
    [4, -2, -2, -2, -2, 1, 1, 1, 1],
    [0, 1, 0, -1, 0, 1, -1, -1, 1],
    [0, -2, 0, 2, 0, 1, -1, -1, 1],
    [0, 0, 1, 0, -1, 1, 1, -1, -1],
    [0, 0, -2, 0, 2, 1, 1, -1, -1],
    [0, 1, -1, 1, -1, 0, 0, 0, 0],
    [0, 0, 0, 0, 0, 1, -1, 1, -1]], dtype=np.float64)
GHOST_MOMENTS = (2, 4, 6)


def moment_weighted_q(w_ghost: float) -> np.ndarray:
    """9 x 9 weight matrix of the residual for gnn_mse_weighted: the residual
    is taken to the orthonormal moment basis, its ghost moments are scaled
    by w_ghost, the others by 1.  w_ghost = 1 gives the identity (Eq. 4)."""
    mh = MOMENT_BASIS / np.linalg.norm(MOMENT_BASIS, axis=1, keepdims=True)
    w = np.ones(9)
    w[list(GHOST_MOMENTS)] = w_ghost
    q = mh.T @ np.diag(w) @ mh
    return 0.5 * (q + q.T)              # exactly symmetric, as gnn_mse_weighted requires


def _loss(out, y, scale, loss_q, want_grad):
    if loss_q is None:
        return gnn.gnn_mse(out, y, scale, want_grad=want_grad)
    return gnn.gnn_mse_weighted(out, y, loss_q, scale, want_grad=want_grad)


def zero_head(blob: torch.Tensor, rounds: int) -> torch.Tensor:
    """The same network with W_h = 0, b_h = 0: the plain BGK collision."""
    off = inputs.blob_offsets(rounds)
    b = blob.clone()
    o, shp = off["Wh"]
    b[o:o + int(np.prod(shp)) + 10] = 0.0           # W_h and b_h are contiguous
    return b


def bgk_loss(X, Y, T, rounds: int, chunk: int = 32, loss_q=None) -> float:
    """Eq. 4 (or its moment-weighted form) of the plain BGK collision over a
    whole set (scale 1)."""
    blob = zero_head(torch.as_tensor(inputs.gnn_blob(0, rounds), device=X.device), rounds)
    total, nodes = 0.0, 0
    for s in range(0, X.shape[0], chunk):
        out, _ = gnn.collide(X[s:s + chunk], T[s:s + chunk], blob, rounds)
        loss, _ = _loss(out, Y[s:s + chunk], 1.0, loss_q, False)
        n = out.numel() // 9
        total += loss.item() * n
        nodes += n
    return total / nodes


def eval_loss(blob, X, Y, T, rounds: int, scale: float, chunk: int = 32, loss_q=None) -> float:
    total, nodes = 0.0, 0
    for s in range(0, X.shape[0], chunk):
        out, _ = gnn.collide(X[s:s + chunk], T[s:s + chunk], blob, rounds)
        loss, _ = _loss(out, Y[s:s + chunk], scale, loss_q, False)
        n = out.numel() // 9
        total += loss.item() * n
        nodes += n
    return total / nodes


class Trainer:
    """Adam on the FP32 parameter blob with the library's forward, backward,
    loss and update kernels."""

    def __init__(self, blob: torch.Tensor, rounds: int = 2, lr: float = 1e-3,
                 betas=(0.9, 0.999), eps: float = 1e-8, shuffle_seed: int = 0, loss_q=None):
        self.blob = blob.contiguous()
        self.rounds = rounds
        self.loss_q = loss_q      # None: Eq. 4; else the 9 x 9 residual weight matrix
        self.lr, self.betas, self.eps = lr, betas, eps
        n = gnn.gnn_param_count(rounds)
        self.m = torch.zeros(n, dtype=torch.float32, device=blob.device)
        self.v = torch.zeros_like(self.m)
        self.step_count = 0
        self.rng = np.random.default_rng(shuffle_seed)
        self.order = None
        self.pos = 0

    def next_batch(self, nsamples: int, batch: int):
        if self.order is None or self.pos + batch > nsamples:
            self.order = self.rng.permutation(nsamples)
            self.pos = 0
        idx = self.order[self.pos:self.pos + batch]
        self.pos += batch
        return torch.as_tensor(idx, device=self.blob.device)

    def step(self, X, Y, T, scale: float, batch: int = 32) -> float:
        idx = self.next_batch(X.shape[0], batch)
        xb, yb, tb = X[idx].contiguous(), Y[idx].contiguous(), T[idx].contiguous()
        B, ny, _, nx = xb.shape
        saved = torch.empty(gnn.saved_bytes(B, nx, ny, self.rounds), dtype=torch.uint8,
                            device=xb.device)
        out, _ = gnn.collide(xb, tb, self.blob, self.rounds, saved=saved)
        loss, dl = _loss(out, yb, scale, self.loss_q, True)
        grad = gnn.gnn_backward(dl, xb, saved, tb, self.blob, self.rounds)
        self.step_count += 1
        gnn.gnn_adam(self.blob, grad, self.m, self.v, self.step_count, self.lr, self.betas[0],
                     self.betas[1], self.eps)
        return loss

    # ---- checkpoint / resume (bitwise: every kernel is deterministic) ----
    def state(self):
        return {"blob": self.blob.cpu().numpy(), "m": self.m.cpu().numpy(),
                "v": self.v.cpu().numpy(), "step": np.int64(self.step_count),
                "pos": np.int64(self.pos),
                "order": (self.order if self.order is not None else np.zeros(0, np.int64)),
                "rng": np.frombuffer(json.dumps(self.rng.bit_generator.state).encode(),
                                     dtype=np.uint8)}

    def save(self, path: str):
        tmp = path + ".tmp.npz"
        np.savez(tmp, **self.state())
        os.replace(tmp, path)

    def load(self, path: str):
        with np.load(path, allow_pickle=False) as z:
            self.blob.copy_(torch.as_tensor(z["blob"]))
            self.m.copy_(torch.as_tensor(z["m"]))
            self.v.copy_(torch.as_tensor(z["v"]))
            self.step_count = int(z["step"])
            self.pos = int(z["pos"])
            self.order = z["order"] if z["order"].size else None
            self.rng.bit_generator.state = json.loads(bytes(z["rng"]).decode())


def datasets(cfg: DataConfig = None, held_out_runs: int = 8, device="cuda"):
    """Training and held-out pairs: ((X, Y, T), (Xh, Yh, Th))."""
    cfg = cfg or DataConfig()
    hcfg = dataclasses.replace(cfg, runs=held_out_runs, seed=cfg.seed + 1)
    return make_dataset(cfg, device), make_dataset(hcfg, device)


def train(cfg: DataConfig = None, steps: int = 2000, batch: int = 32, rounds: int = 2,
          lr: float = 1e-3, init_seed: int = 0, s_delta: float = 1e-4, held_out_runs: int = 8,
          log_every: int = 0, device="cuda", data=None, loss_q=None):
    """Full training run; returns (trainer, report dict).  `data` reuses the
    pairs of datasets() (same cfg and held_out_runs) instead of generating
    them.  loss_q: None trains on Eq. 4; a 9 x 9 matrix (moment_weighted_q)
    weights each node's residual, the loss then relative to the same
    weighted loss of plain BGK."""
    import time
    t0 = time.perf_counter()
    if data is None:
        data = datasets(cfg, held_out_runs, device)
    (X, Y, T), (Xh, Yh, Th) = data
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    l_bgk = bgk_loss(X, Y, T, rounds, loss_q=loss_q)
    l_bgk_h = bgk_loss(Xh, Yh, Th, rounds, loss_q=loss_q)
    blob = torch.as_tensor(inputs.gnn_blob(init_seed, rounds, s_delta=s_delta), device=device)
    tr = Trainer(blob, rounds, lr, loss_q=loss_q)
    before = eval_loss(tr.blob, Xh, Yh, Th, rounds, 1.0 / l_bgk_h, loss_q=loss_q)
    hist = []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(steps):
        loss = tr.step(X, Y, T, 1.0 / l_bgk, batch)
        if log_every and (k % log_every == 0 or k == steps - 1):
            hist.append((k, loss.item()))
    torch.cuda.synchronize()
    t_opt = time.perf_counter() - t1
    after = eval_loss(tr.blob, Xh, Yh, Th, rounds, 1.0 / l_bgk_h, loss_q=loss_q)
    train_after = eval_loss(tr.blob, X, Y, T, rounds, 1.0 / l_bgk, loss_q=loss_q)
    return tr, {"bgk_loss_train": l_bgk, "bgk_loss_heldout": l_bgk_h,
                "heldout_rel_loss_before": before, "heldout_rel_loss_after": after,
                "train_rel_loss_after": train_after, "history": hist,
                "samples": int(X.shape[0]), "heldout_samples": int(Xh.shape[0]),
                "data_seconds": t_data, "optimizer_seconds": t_opt,
                # one sample = one 128^2 lattice through forward, Eq. 4, backward
                "samples_per_s": steps * batch / t_opt if t_opt > 0 else None}


def main(argv=None):
    import argparse
    import time
    ap = argparse.ArgumentParser(description="Train the GNN collision on self-generated data")
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--runs", type=int, default=32)
    ap.add_argument("--n-fine", type=int, default=512)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--s-delta", type=float, default=1e-4)
    ap.add_argument("--rounds", type=int, default=2, help="2: message passing; 0: Fig. 2")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    cfg = DataConfig(n_fine=args.n_fine, runs=args.runs)
    t0 = time.perf_counter()
    tr, rep = train(cfg, steps=args.steps, batch=args.batch, rounds=args.rounds, lr=args.lr,
                    s_delta=args.s_delta, log_every=max(1, args.steps // 20))
    torch.cuda.synchronize()
    rep["wall_s"] = time.perf_counter() - t0
    rep["config"] = dataclasses.asdict(cfg)
    rep["steps"], rep["batch"], rep["lr"], rep["rounds"] = args.steps, args.batch, args.lr, args.rounds
    print(json.dumps(rep), flush=True)
    if args.out:
        tr.save(args.out)


if __name__ == "__main__":
    main()
