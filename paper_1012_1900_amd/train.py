"""Train the learned-radius CNN on the GPU with the library's own kernels.

Data: seeded synthetic 3D pairs of the 128x128x96 / 2.5 mm IMRT-like generator
(``dosegen``), training seeds ``--train-seed0 ..``, held-out seeds ``--heldout-seed0 ..``.
Labels are the library's exact gamma (3%/3mm global, 10 % cutoff); features come from the
library too.  Training takes crops of ``--crop`` output nodes around random evaluated
nodes (with their 4-node neighbourhood of features), and minimises the mean squared error
of log(gamma + 0.01) over the evaluated nodes of a batch with Adam.

The held-out report compares the prediction with the exact gamma (RMSE of the log,
rank correlation), and the learned search with the plain one (identical gamma, fallback
rate, time).

  python -m paper_1012_1900_amd.train --out paper_1012_1900_amd/weights/cnn_3d_2.5mm_3pct3mm.npy
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "3d_128x128x96_2.5mm"


def _make(seed):
    from dosegen import make_config_pair
    p = make_config_pair(WORKLOAD, seed)
    return seed, p.ref, p.eval, p.spacing


def log(msg):
    print(msg, flush=True)


def init_params(seed):
    """He-uniform weights, zero biases (FP32), in the flat layout of the C ABI."""
    rng = np.random.default_rng(seed)
    parts = []
    for ci, co in ((2, 16), (16, 16), (16, 16), (16, 1)):
        lim = np.sqrt(6.0 / (ci * 27))
        parts.append(rng.uniform(-lim, lim, size=co * ci * 27).astype(np.float32))
        parts.append(np.zeros(co, dtype=np.float32))
    return np.concatenate(parts)


def spearman(a, b):
    ra = np.argsort(np.argsort(a)).astype(np.float64)
    rb = np.argsort(np.argsort(b)).astype(np.float64)
    ra -= ra.mean()
    rb -= rb.mean()
    return float((ra * rb).sum() / np.sqrt((ra * ra).sum() * (rb * rb).sum()))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--train-pairs", type=int, default=2000)
    ap.add_argument("--heldout-pairs", type=int, default=200)
    ap.add_argument("--train-seed0", type=int, default=10000)
    ap.add_argument("--heldout-seed0", type=int, default=20000)
    ap.add_argument("--crops-per-pair", type=int, default=8)
    ap.add_argument("--crop", type=int, nargs=3, default=[24, 24, 32])
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--high-gamma", type=float, default=0.5,
                    help="half of the crops centre on nodes with gamma at least this")
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--dd", type=float, default=0.03)
    ap.add_argument("--dta", type=float, default=3.0)
    ap.add_argument("--out", required=True)
    ap.add_argument("--checkpoint", default=None,
                    help="write a checkpoint (parameters and Adam state) here every --checkpoint-every "
                         "steps and at the end")
    ap.add_argument("--checkpoint-every", type=int, default=1000)
    ap.add_argument("--resume", default=None,
                    help="continue the training from this checkpoint: its parameters, Adam state and step")
    args = ap.parse_args()

    # worker processes first, before anything touches the GPU
    pool = mp.get_context("fork").Pool(args.workers)

    import torch
    import paper_1012_1900_amd as gx

    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(args.seed)
    c0, c1, c2 = args.crop
    n_crops = args.train_pairs * args.crops_per_pair
    feats_all = torch.empty((n_crops, c0 + 8, c1 + 8, c2 + 8, 2), dtype=torch.int16, device=dev)
    labels_all = torch.empty((n_crops, c0, c1, c2), dtype=torch.float32, device=dev)
    ctx = gx.context(0)

    t0 = time.time()
    k = 0
    seeds = range(args.train_seed0, args.train_seed0 + args.train_pairs)
    for j, (seed, ref_h, ev_h, spacing) in enumerate(pool.imap(_make, seeds, chunksize=4)):
        ref = torch.from_numpy(ref_h).to(dev)
        ev = torch.from_numpy(ev_h).to(dev)
        gam, _ = gx.gammax_map(ref, ev, spacing, args.dd, args.dta, 0.1, ctx=ctx)
        feat = gx.model_features(ref, ev, spacing, args.dd, args.dta, ctx=ctx)
        masked = torch.nonzero(gam >= 0).cpu().numpy()
        # half of the crops centre on nodes of large gamma: the ones that walk past the
        # key-0 cells are rare, and they are where the prediction is used
        high = torch.nonzero(gam >= args.high_gamma).cpu().numpy()
        nz, ny, nx = gam.shape
        for c in range(args.crops_per_pair):
            pool_c = high if (c % 2 == 1 and len(high)) else masked
            z, y, x = pool_c[rng.integers(len(pool_c))]
            oz = int(np.clip(z - c0 // 2, 0, nz - c0))
            oy = int(np.clip(y - c1 // 2, 0, ny - c1))
            ox = int(np.clip(x - c2 // 2, 0, nx - c2))
            feats_all[k] = feat[oz:oz + c0 + 8, oy:oy + c1 + 8, ox:ox + c2 + 8]
            labels_all[k] = gam[oz:oz + c0, oy:oy + c1, ox:ox + c2]
            k += 1
        if (j + 1) % 100 == 0:
            log(f"data: {j + 1}/{args.train_pairs} pairs, {time.time() - t0:.1f} s")
    torch.cuda.synchronize()
    t_data = time.time() - t0

    start = 0
    if args.resume:
        model = gx.Model.load(args.resume)
        with open(args.resume, "rb") as f:
            start = int(json.loads(f.readline())["adam_step"])
        log(f"resumed from {args.resume} at step {start}")
        # the batches after a resume come from their own stream of the same seed
        rng = np.random.default_rng([args.seed, start])
    else:
        model = gx.Model(init_params(args.seed + 1))
    t0 = time.time()
    losses = []
    for step in range(start, args.steps):
        lr = args.lr * 0.5 * (1.0 + np.cos(np.pi * step / args.steps))   # cosine decay
        idx = torch.from_numpy(rng.integers(0, n_crops, size=args.batch)).to(dev)
        loss = model.train_step(feats_all[idx].contiguous(), labels_all[idx].contiguous(), lr=lr)
        losses.append(loss)
        if (step + 1) % 1000 == 0:
            log(f"step {step + 1}: loss {np.mean(losses[-1000:]):.4f} lr {lr:.2e} ({time.time() - t0:.1f} s)")
        if args.checkpoint and (step + 1) % args.checkpoint_every == 0:
            model.save(args.checkpoint)
    t_train = time.time() - t0
    if args.checkpoint:
        model.save(args.checkpoint)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    model.save_params(args.out)

    # held-out report
    del feats_all, labels_all
    rmse, rho_hat, rho_dd, certified, fb_rate, ms_plain, ms_learned = [], [], [], [], [], [], []
    hseeds = range(args.heldout_seed0, args.heldout_seed0 + args.heldout_pairs)
    for seed, ref_h, ev_h, spacing in pool.imap(_make, hseeds, chunksize=4):
        ref = torch.from_numpy(ref_h).to(dev)
        ev = torch.from_numpy(ev_h).to(dev)
        gam, rp = gx.gammax_map(ref, ev, spacing, args.dd, args.dta, 0.1, ctx=ctx, timing=True)
        y = model.predict(ref, ev, spacing, args.dd, args.dta, ctx=ctx)
        gl, rl = gx.gammax_map(ref, ev, spacing, args.dd, args.dta, 0.1, ctx=ctx, timing=True,
                               radius="learned", sort="predicted", model=model)
        if not torch.equal(gam, gl):
            raise RuntimeError(f"learned search differs from the plain search on seed {seed}")
        g = gam.cpu().numpy()
        yh = y.cpu().numpy()
        m = g >= 0
        t = np.log(g[m].astype(np.float64) + 0.01)
        rmse.append(float(np.sqrt(np.mean((yh[m] - t) ** 2))))
        ghat = np.maximum(np.exp(yh[m]) - 0.01, 0.0)
        g0 = np.abs(ev_h - ref_h)[m] / (args.dd * float(ref_h.max()))
        sub = rng.choice(m.sum(), size=min(20000, int(m.sum())), replace=False)
        rho_hat.append(spearman(ghat[sub], g[m][sub]))
        rho_dd.append(spearman(g0[sub], g[m][sub]))
        certified.append(float(np.mean(g[m] <= 1.1 * ghat)))
        fb_rate.append(rl.n_fallback / max(rl.n_tail, 1))
        ms_plain.append(rp.ms_prep + rp.ms_search + rp.ms_sort + rp.ms_tail + rp.ms_guard)
        ms_learned.append(rl.ms_prep + rl.ms_cnn + rl.ms_search + rl.ms_sort + rl.ms_tail + rl.ms_guard)
    pool.close()
    report = {
        "workload": WORKLOAD, "criteria": f"{args.dd * 100:g}%/{args.dta:g}mm global, 10% cutoff",
        "train_seeds": [args.train_seed0, args.train_seed0 + args.train_pairs - 1],
        "heldout_seeds": [args.heldout_seed0, args.heldout_seed0 + args.heldout_pairs - 1],
        "crops_per_pair": args.crops_per_pair, "crop": args.crop, "batch": args.batch,
        "high_gamma": args.high_gamma,
        "steps": args.steps, "lr": args.lr, "seed": args.seed,
        "final_train_loss": float(np.mean(losses[-250:])) if losses else None,
        "resumed_from_step": start,
        "data_seconds": round(t_data, 1), "train_seconds": round(t_train, 1),
        "heldout": {
            "rmse_log_gamma": float(np.mean(rmse)),
            "spearman_gamma_hat": float(np.mean(rho_hat)),
            "spearman_dd": float(np.mean(rho_dd)),
            "certified_inside_1.1_gamma_hat": float(np.mean(certified)),
            "tail_fallback_rate": float(np.mean(fb_rate)),
            "ms_plain_mean": float(np.mean(ms_plain)),
            "ms_learned_mean": float(np.mean(ms_learned)),
        },
    }
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(report, f, indent=1)
    log(json.dumps(report))


if __name__ == "__main__":
    main()
