"""Data generation, training and evaluation of the learned multipath surrogate.

Orchestration only: the pings, level targets, network forward and backward
passes, Adam updates, predicted profiles and their dB errors all run in the
library's HIP kernels; this module assembles batches and schedules.

Data: multi-bounce pings (3 bounces, c(z) gradient) of the harbor multipath
scene from random survey poses. Each ping yields the single-bounce G-buffer
(network input) and the later-bounce incoherent channel, whose range-smoothed
dB level above the intensity floor, aligned to each beam's first-hit bin,
compressed to 64 DCT coefficients and standardised, is the target. The loss
weights coefficient j by its variance over the mean variance, which makes it
the squared error of the level profile (Parseval).

    python -m paper_2606_06130_amd.surrogate --train-pings 20000 --epochs 5 \\
        --eval-pings 1000 --out surrogate_run
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
    """Mean and standard deviation of the raw level coefficients over pings."""
    torch = src.torch
    coef = torch.empty((src.rows, 64), dtype=torch.float32, device="cuda")
    s1 = np.zeros(64)
    s2 = np.zeros(64)
    n = 0
    for p in poses:
        gb, _, im = src.run(p)
        sur.target(im, gb, standardize=False, out=coef)
        a, b = sur.moments(coef)
        s1 += a
        s2 += b
        n += src.rows
    mean = s1 / n
    std = np.sqrt(np.maximum(s2 / n - mean * mean, 1e-12))
    return mean.astype(np.float32), np.maximum(std, 1e-3).astype(np.float32)


def loss_weights(std):
    """w_j = std_j^2 / mean(std^2): the loss on standardised coefficients is
    then the squared error of the de-standardised ones (up to one scale)."""
    v = np.asarray(std, np.float64) ** 2
    return (v / v.mean()).astype(np.float32)


def geometry(src, poses):
    """Device [len(poses), 16]: the geometry blocks of the poses."""
    return src.torch.from_numpy(sonar.surrogate_geometry(src.cfg, poses)).cuda()


def train(sur, src, poses, epochs, batch_pings, lr0, log=print, start_step=0, stop_step=None):
    """Adam with cosine learning-rate decay over mini-batches of `batch_pings`
    pings, from step `start_step` up to (not including) `stop_step` (default:
    the end of the schedule). Returns the per-step losses."""
    torch = src.torch
    B = batch_pings
    geo_all = geometry(src, poses)
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
            if stop_step is not None and step >= stop_step:
                break
            pick = order[s * B:(s + 1) * B]
            for b in range(B):
                _, _, im = src.run(poses[pick[b]], gbuf_slot=gb[b])
                sur.target(im, gb[b], standardize=True, out=tgt[b * src.rows:(b + 1) * src.rows])
            geo = geo_all[torch.from_numpy(pick).cuda()].contiguous()
            lr = 0.5 * lr0 * (1.0 + math.cos(math.pi * step / max(total, 1)))
            sur.train_step(gb, geo, tgt, lr, loss)
            if step % 50 == 0 or step == total - 1:
                lv = float(loss.item())
                losses.append((step, lv))
                log(f"step {step}/{total} epoch {ep} loss {lv:.4f} lr {lr:.2e} {time.time() - t0:.0f}s")
            step += 1
    torch.cuda.synchronize()
    return losses


ERROR_COLUMNS = ("surrogate", "single_bounce", "mean_level", "occupied_bins",
                 "surrogate_raw", "mean_level_raw", "single_bounce_raw", "occupied_bins_raw")


def evaluate(sur, src, poses):
    """Per-beam dB errors over held-out pings, mean and p95 over beams.

    Against the range-smoothed truth (beams with occupied smoothed bins), of
    range-smoothed profiles: the surrogate, the single bounce, the single
    bounce plus the mean level and the truncated truth (the best any
    64-coefficient prediction can do: the truncation floor). Against the raw
    truth (beams with occupied raw bins), of full-resolution profiles (the
    raw single-bounce channel plus a level): the same four, and the surrogate
    against the truncated truth (the network's own error)."""
    torch = src.torch
    errs, errt, errn = [], [], []
    coef = torch.empty((src.rows, 64), dtype=torch.float32, device="cuda")
    exact = torch.empty((src.rows, 64), dtype=torch.float32, device="cuda")
    gbv = torch.empty((1, src.H, src.W, 8), dtype=torch.float32, device="cuda")
    # standardised coefficients of a zero level: the profile is then the smoothed input channel
    zero = torch.from_numpy(-sur.mean / sur.std).cuda().expand(src.rows, 64).contiguous()
    occupied_db = 10.0 * math.log10(1e-11) + 3.0
    geo_all = geometry(src, poses)
    for i, p in enumerate(poses):
        _, i1, im = src.run(p, gbuf_slot=gbv[0])
        sur.forward(gbv, geo_all[i:i + 1], out=coef)
        pred, e = sur.profile(coef, i1, gbv, im)
        sur.target(im, gbv, standardize=True, out=exact)
        trunc, et = sur.profile(exact, i1, gbv, im)
        truth, _ = sur.profile(zero, i1 + im, gbv)     # 10 log10(I1 + Im + floor): the raw truth
        occ = truth > occupied_db
        cnt = occ.sum(dim=1)
        en = torch.where(occ, (pred - trunc).abs(), torch.zeros_like(pred)).sum(dim=1) / cnt.clamp(min=1)
        errs.append(e.cpu().numpy())
        errt.append(et.cpu().numpy())
        errn.append(en.cpu().numpy())
    e = np.concatenate(errs)
    et = np.concatenate(errt)
    en = np.concatenate(errn)

    def stat(v):
        return {"mean_db": float(np.mean(v)), "p95_db": float(np.percentile(v, 95))}

    ok = e[:, 3] > 0
    okr = e[:, 7] > 0
    out = {"pings": len(poses), "beams": int(ok.sum()), "beams_raw": int(okr.sum())}
    out["surrogate"] = stat(e[ok, 0])
    out["single_bounce"] = stat(e[ok, 1])
    out["mean_level"] = stat(e[ok, 2])
    out["truncated_truth"] = stat(et[ok, 0])
    out["raw"] = {"surrogate": stat(e[okr, 4]), "single_bounce": stat(e[okr, 6]), "mean_level": stat(e[okr, 5]),
                  "truncated_truth": stat(et[okr, 4]), "surrogate_vs_truncated_truth": stat(en[okr])}
    out["meets_1db"] = bool(out["surrogate"]["mean_db"] <= 1.0)
    return out


def save_checkpoint(path, sur, mean, std, extra=None, weights_only=False):
    """Weights, standardisation and (unless weights_only) the Adam state, as
    plain arrays in an .npz (loadable without pickle)."""
    p, m, v, step = sur.get_state()
    arrays = dict(params=p, step=np.int64(step), mean=np.asarray(mean, np.float32),
                  std=np.asarray(std, np.float32), extra=np.str_(json.dumps(extra or {})))
    if not weights_only:
        arrays.update(adam_m=m, adam_v=v)
    np.savez_compressed(path, **arrays)


def load_checkpoint(path, sur):
    """Loads a checkpoint into `sur`; returns (mean, std, step, extra dict)."""
    with np.load(path, allow_pickle=False) as d:
        if d["params"].shape != (sur.n_params,):
            raise ValueError(f"{path}: {d['params'].shape[0]} parameters, the network has {sur.n_params}")
        m = d["adam_m"] if "adam_m" in d.files else None
        v = d["adam_v"] if "adam_v" in d.files else None
        sur.set_state(d["params"], m, v, int(d["step"]))
        mean, std = d["mean"], d["std"]
        sur.set_norm(mean, std)
        extra = json.loads(str(d["extra"])) if "extra" in d.files else {}
        return mean, std, int(d["step"]), extra


WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "surrogate_harbor_multipath.npz")


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
    ap.add_argument("--stop-step", type=int, default=None,
                    help="stop before this step of the schedule: write the checkpoint, skip the evaluation")
    ap.add_argument("--weights-out", default=None, help="also write the weights-only checkpoint here")
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
        mean, std, start, _ = load_checkpoint(args.resume, sur)
    else:
        mean, std = coefficient_stats(sur, src, train_poses[:args.stats_pings])
        sur.set_norm(mean, std)
        sur.set_state(S.surrogate_init_params(11))
    sur.set_loss_weights(loss_weights(std))
    log(f"setup {time.time() - t0:.1f}s; rows/ping {src.rows}; params {sur.n_params}")
    losses = train(sur, src, train_poses, args.epochs, args.batch, args.lr, log, start_step=start,
                   stop_step=args.stop_step)
    t_train = time.time() - t0
    save_checkpoint(os.path.join(args.out, "checkpoint.npz"), sur, mean, std)
    if args.stop_step is not None and args.stop_step < (args.train_pings // args.batch) * args.epochs:
        log(f"stopped before step {args.stop_step}; resume from {os.path.join(args.out, 'checkpoint.npz')}")
        return
    meta = {"target": "level", "inputs": "gbuffer+geometry+mirror", "smooth": 32, "train_pings": args.train_pings,
            "train_pose_seed": 5,
            "epochs": args.epochs, "batch_pings": args.batch, "lr": args.lr, "stats_pings": args.stats_pings}
    if args.weights_out:
        save_checkpoint(args.weights_out, sur, mean, std, extra=meta, weights_only=True)
    res = evaluate(sur, src, eval_poses)
    res.update(meta)
    res.update({"train_seconds": t_train, "final_loss": losses[-1][1] if losses else None,
                "losses": losses[::max(1, len(losses) // 20)], "eval_pose_seed": 6})
    with open(os.path.join(args.out, "summary.json"), "w") as f:
        json.dump(res, f, indent=1)
    log(json.dumps(res))
    torch.cuda.synchronize()
    return 0


if __name__ == "__main__":
    sys.exit(main())
