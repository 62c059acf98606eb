"""Data generation, training and evaluation of the learned multipath surrogate.

Orchestration only: the pings, residual targets, network forward and
backward passes, Adam updates, predicted profiles and their dB errors all run
in the library's HIP kernels; this module assembles batches and schedules.

Data: multi-bounce pings (3 bounces, c(z) gradient) of the harbor multipath
scene from random survey poses. Each ping yields the single-bounce G-buffer
(network input) and the two incoherent channels, whose range-smoothed dB
residual, aligned to each beam's first-hit bin, compressed to 64 DCT
coefficients and standardised, is the target.

    python -m paper_2606_06130_amd.surrogate --train-pings 2000 --epochs 3 \\
        --eval-pings 200 --out surrogate_run
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import scenes as S
from . import sonar


class PingSource:
    """Runs multi-bounce pings into preallocated buffers."""

    def __init__(self, scene, cfg):
        import torch
        self.scene, self.cfg = scene, cfg
        bv, bh = sonar.beams_of(cfg)
        self.H, self.W = bv, bh
        self.rows = bv * bh
        self.out = sonar.alloc_outputs(cfg, gbuffer=True, incoh=True)
        self.params = sonar.params_of(cfg)
        self.torch = torch

    def run(self, pose, gbuf_slot=None):
        """One ping; the G-buffer goes to `gbuf_slot` ([H, W, 8] view) if given.
        Returns (gbuffer [H, W, 8], i1 [rows, bins], im [rows, bins]) views."""
        o = self.out
        if gbuf_slot is not None:
            o = dict(o)
            o["gbuffer"] = gbuf_slot
        sonar.ping(self.scene, self.cfg, pose, out=o, params=self.params)
        inc = self.out["incoh"].view(2, self.rows, self.cfg.n_range)
        return o["gbuffer"], inc[0], inc[1]


def coefficient_stats(sur, src, poses):
    """Mean and standard deviation of the raw residual coefficients over pings."""
    torch = src.torch
    coef = torch.empty((src.rows, 64), dtype=torch.float32, device="cuda")
    s1 = np.zeros(64)
    s2 = np.zeros(64)
    n = 0
    for p in poses:
        gb, i1, im = src.run(p)
        sur.residual(i1, im, gb, standardize=False, out=coef)
        a, b = sur.moments(coef)
        s1 += a
        s2 += b
        n += src.rows
    mean = s1 / n
    std = np.sqrt(np.maximum(s2 / n - mean * mean, 1e-12))
    return mean.astype(np.float32), np.maximum(std, 1e-3).astype(np.float32)


def train(sur, src, poses, epochs, batch_pings, lr0, log=print, start_step=0):
    """Adam with cosine learning-rate decay over mini-batches of `batch_pings`
    pings. Returns the per-step losses."""
    torch = src.torch
    B = batch_pings
    gb = torch.empty((B, src.H, src.W, 8), dtype=torch.float32, device="cuda")
    tgt = torch.empty((B * src.rows, 64), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    steps_per_epoch = len(poses) // B
    total = steps_per_epoch * epochs
    losses = []
    rng = np.random.Generator(np.random.PCG64(77))
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        order = rng.permutation(len(poses))
        for s in range(steps_per_epoch):
            if step < start_step:
                step += 1
                continue
            for b in range(B):
                _, i1, im = src.run(poses[order[s * B + b]], gbuf_slot=gb[b])
                sur.residual(i1, im, gb[b], standardize=True, out=tgt[b * src.rows:(b + 1) * src.rows])
            lr = 0.5 * lr0 * (1.0 + math.cos(math.pi * step / max(total, 1)))
            sur.train_step(gb, tgt, lr, loss)
            if step % 50 == 0 or step == total - 1:
                lv = float(loss.item())
                losses.append((step, lv))
                log(f"step {step}/{total} epoch {ep} loss {lv:.4f} lr {lr:.2e} {time.time() - t0:.0f}s")
            step += 1
    torch.cuda.synchronize()
    return losses


def evaluate(sur, src, poses):
    """Mean and p95 per-beam dB errors over beams with occupied bins:
    surrogate, single bounce only, single bounce + mean residual, and the
    best any 64-coefficient prediction can do (the truncated truth), all
    against the smoothed truth; and the surrogate against the truncated truth
    (the network's own error, the DCT truncation taken out)."""
    torch = src.torch
    errs, errt, errn = [], [], []
    coef = torch.empty((src.rows, 64), dtype=torch.float32, device="cuda")
    exact = torch.empty((src.rows, 64), dtype=torch.float32, device="cuda")
    gbv = torch.empty((1, src.H, src.W, 8), dtype=torch.float32, device="cuda")
    # standardised coefficients of a zero residual: the profile is then the smoothed input channel
    zero = torch.from_numpy(-sur.mean / sur.std).cuda().expand(src.rows, 64).contiguous()
    occupied_db = 10.0 * math.log10(1e-11) + 3.0
    for p in poses:
        _, i1, im = src.run(p, gbuf_slot=gbv[0])
        sur.forward(gbv, out=coef)
        pred, e = sur.profile(coef, i1, gbv, im)
        sur.residual(i1, im, gbv, standardize=True, out=exact)
        trunc, et = sur.profile(exact, i1, gbv, im)
        truth, _ = sur.profile(zero, i1 + im, gbv)
        occ = truth > occupied_db
        cnt = occ.sum(dim=1)
        en = torch.where(occ, (pred - trunc).abs(), torch.zeros_like(pred)).sum(dim=1) / cnt.clamp(min=1)
        errs.append(e.cpu().numpy())
        errt.append(et.cpu().numpy())
        errn.append(en.cpu().numpy())
    e = np.concatenate(errs)
    et = np.concatenate(errt)
    en = np.concatenate(errn)
    ok = e[:, 3] > 0
    e, et, en = e[ok], et[ok], en[ok]
    out = {"beams": int(ok.sum()), "pings": len(poses)}
    for i, nm in enumerate(("surrogate", "single_bounce", "mean_residual")):
        out[nm] = {"mean_db": float(np.mean(e[:, i])), "p95_db": float(np.percentile(e[:, i], 95))}
    out["truncated_truth"] = {"mean_db": float(np.mean(et[:, 0])), "p95_db": float(np.percentile(et[:, 0], 95))}
    out["surrogate_vs_truncated_truth"] = {"mean_db": float(np.mean(en)), "p95_db": float(np.percentile(en, 95))}
    return out


def save_checkpoint(path, sur, mean, std, extra=None):
    p, m, v, step = sur.get_state()
    np.savez(path, params=p, adam_m=m, adam_v=v, step=np.int64(step), mean=mean, std=std,
             extra=json.dumps(extra or {}))


def load_checkpoint(path, sur):
    d = np.load(path, allow_pickle=False)
    sur.set_state(d["params"], d["adam_m"], d["adam_v"], int(d["step"]))
    sur.set_norm(d["mean"], d["std"])
    return d["mean"], d["std"], int(d["step"])


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-pings", type=int, default=2000)
    ap.add_argument("--eval-pings", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=3)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--stats-pings", type=int, default=64)
    ap.add_argument("--out", default="surrogate_run")
    ap.add_argument("--resume", default=None)
    args = ap.parse_args(argv)
    import torch
    os.makedirs(args.out, exist_ok=True)
    logf = open(os.path.join(args.out, "train.log"), "a")

    def log(msg):
        print(msg, flush=True)
        logf.write(msg + "\n")
        logf.flush()

    mesh = S.scene_harbor_multipath()
    scene = sonar.Scene(mesh)
    cfg = S.sensor_harbor_multipath()
    train_poses = S.random_poses(5, args.train_pings)
    eval_poses = S.random_poses(6, args.eval_pings)
    src = PingSource(scene, cfg)
    sur = sonar.Surrogate(args.batch * src.rows, cfg.n_range, cfg.r_min, cfg.r_max)
    t0 = time.time()
    start = 0
    if args.resume:
        mean, std, start = load_checkpoint(args.resume, sur)
    else:
        mean, std = coefficient_stats(sur, src, train_poses[:args.stats_pings])
        sur.set_norm(mean, std)
        sur.set_state(S.surrogate_init_params(11))
    log(f"setup {time.time() - t0:.1f}s; rows/ping {src.rows}; params {sur.n_params}")
    losses = train(sur, src, train_poses, args.epochs, args.batch, args.lr, log, start_step=start)
    t_train = time.time() - t0
    save_checkpoint(os.path.join(args.out, "checkpoint.npz"), sur, mean, std)
    res = evaluate(sur, src, eval_poses)
    res.update({"train_pings": args.train_pings, "epochs": args.epochs, "batch_pings": args.batch,
                "train_seconds": t_train, "final_loss": losses[-1][1] if losses else None,
                "losses": losses[::max(1, len(losses) // 20)]})
    with open(os.path.join(args.out, "summary.json"), "w") as f:
        json.dump(res, f, indent=1)
    log(json.dumps(res))
    torch.cuda.synchronize()
    return 0


if __name__ == "__main__":
    sys.exit(main())
