#!/usr/bin/env python3
"""Benchmark of the gamma-index search on one MI355X.

One step = one full gamma map of a synthetic IMRT-like dose pair (dose maximum, mask,
gamma0, compaction, cell table, DD sort, search, pass counts), inputs resident in HBM.
Prints one JSON line: reference voxels per second, the search kernel's roofline, and the
FP64 CPU oracle timed on this host as a baseline.

  python bench.py [--steps K] [--warmup W] [--workload 3d_128x128x96_2.5mm] [--dd 0.03 --dta 3]
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TRAIN_SPACING_MM = 2.5   # grid spacing of the shipped network's training pairs
METRIC = "ref voxels/sec, 3D 3%/3mm: plain vs learned-radius at |Δγ|≤1e-5; %FP32 peak"

# FP32 operations per evaluated cell of the closed-form face projections (3D: 8 corner
# differences, 19 chain steps, 1 vertex, 7 edges, 12 triangles, 6 tetrahedra; FMA = 2,
# add/mul/rcp = 1, compares and min = 0).  2D: 4 corners, 5 steps, 1 vertex, 3 edges,
# 2 triangles.
FLOP_PER_CELL = {3: 392, 2: 82}
# The per-cell work of the reference formulation (every face of the Kuhn lattice projected
# with its own normal equations: 6 tetrahedra with a 3x3 Gram solve and the condition check,
# 12 triangles, 7 edges, 1 vertex), fixed before any tuning; the roofline fraction is quoted
# on it, with the closed-form count beside it.
FLOP_PER_CELL_REFERENCE = {3: 1100, 2: 150}
PEAK_FP32_TFLOPS = 157.3    # MI355X vector FP32 (packed)
PEAK_BF16_TFLOPS = 2500.0   # MI355X dense BF16 matrix cores

# HBM bytes per launch of the dominant kernel, from the FETCH_SIZE and WRITE_SIZE counter
# runs summarised in the named profile (each counter scaled by what it reads for a plain
# 256 MiB device copy).  They hold only for the kernel source they were taken on: when its
# hash differs the traffic is reported as null.
TRAFFIC = {
    "3d_128x128x96_2.5mm": {
        "bytes": (15.64 + 2.25) * 1e6,
        "source": "paper_1012_1900_amd/csrc/k_search.hip",
        "sha256": "7e435a71fae7fe288f525dff3d5614aa0fcc235f56c40e4590c7dd95eee89105",
        "profile": "profiles/pmc_hbm_bytes_128x128x96_2.5mm_3pct3mm.md",
    },
}

# The mixed batch: 64 pairs, 2D or 3D, 3%/3mm, 2%/2mm or 1%/1mm, global or local.
MIXED = ("mixed_64_pairs", 40000, 64)

WORKLOADS = {
    "3d_128x128x96_2.5mm": ("3d_128x128x96_2.5mm", 100, "3D 128x128x96 at 2.5 mm, 7-beam synthetic IMRT-like pair (seed 100)"),
    "3d_256x256x192_1.25mm": ("3d_256x256x192_1.25mm", 200, "3D 256x256x192 at 1.25 mm, 7-beam synthetic IMRT-like pair (seed 200)"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def work_counts(cfg, seed, dd, dta):
    path = os.path.join(ROOT, "tests", "golden", "work_counts.json")
    try:
        with open(path) as f:
            table = json.load(f)
    except OSError:
        return None
    return table.get(f"{cfg}/seed{seed}/{dd * 100:g}%/{dta:g}mm/global/thr0.1")


def traffic_bytes(workload, kernel_default):
    t = TRAFFIC.get(workload)
    if t is None or not kernel_default:
        return None
    import hashlib
    try:
        with open(os.path.join(ROOT, t["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != t["sha256"]:
                return None
    except OSError:
        return None
    return t["bytes"]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def accuracy(g, o):
    """Error of a GPU gamma map (device tensor) against the FP64 oracle's: the largest
    |dgamma| over the masked nodes, the nodes beyond 1e-5 + 1e-5 gamma, mask agreement, and
    the pass counts (outside the 1e-5 band around gamma = 1, and that band's size)."""
    import numpy as np
    gh = g.detach().cpu().numpy().astype(np.float64).ravel()
    go = o.gamma.ravel()
    m = go >= 0
    same_mask = bool(np.array_equal(m, gh >= 0))
    err = np.abs(gh[m] - go[m])
    beyond = int((err > 1e-5 + 1e-5 * go[m]).sum())
    band = np.abs(go - 1.0) <= 1e-5
    outside = m & ~band
    pass_diff = int(((gh[outside] <= 1.0) != (go[outside] <= 1.0)).sum())
    return {"max_abs_dgamma": float(err.max()) if err.size else 0.0, "n_beyond_tol": beyond,
            "same_mask": same_mask, "n_pass_gpu": int((gh[m] <= 1.0).sum()), "n_pass_oracle": int(o.n_pass),
            "pass_decisions_differ_outside_band": pass_diff, "n_borderline_oracle": int(band[m].sum()),
            "ok": bool(same_mask and beyond == 0 and pass_diff == 0)}


def oracle_gamma(pair, dd, dta):
    import oracle
    oracle.build()
    return oracle.gamma(pair.ref, pair.eval, pair.spacing, dd, dta, 0.1)


def cpu_baseline(pair, dd, dta, reps, seconds):
    """The FP64 oracle as it stands, on every host core, over the whole workload, repeated
    until at least `seconds` of CPU time have passed (and at least `reps` times); the rate is
    the mean over every repetition."""
    import oracle
    oracle.build()
    n, total = 0, 0.0
    while n < max(1, reps) or total < seconds:
        t = time.perf_counter()
        o = oracle.gamma(pair.ref, pair.eval, pair.spacing, dd, dta, 0.1)
        total += time.perf_counter() - t
        n += 1
    return {
        "value": n * o.n_evaluated / total,
        "unit": "ref voxels/s",
        "cores": oracle.max_threads(),
        "cpu_count": os.cpu_count(),
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": f"whole workload ({o.n_evaluated} masked nodes, {o.cells_visited} cells) "
                  f"{n} times, {total:.1f} s in all, mean rate",
    }, o


# ---- sweeps of the paper's scaling studies --------------------------------------------------

# resolution levels of the scaling study (Sec. 3.5): the same box as the 3D workloads
# (240 x 320 x 320 mm, z slowest) sampled at the paper's four grid sizes
SWEEP_RESOLUTIONS = ((144, 128, 128), (72, 256, 256), (144, 256, 256), (72, 512, 512))
SWEEP_BOX_MM = (240.0, 320.0, 320.0)


def _time_maps(gx, torch, ref, ev, spacing, dd, dta, steps, warmup):
    """ms per queued map (graph replays, results collected inside the timed region), the
    phase times of one timed map, and that map's gamma and result."""
    for _ in range(warmup):
        gx.gammax_map(ref, ev, spacing, dd, dta, 0.1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = [gx.gammax_map_async(ref, ev, spacing, dd, dta, 0.1) for _ in range(steps)]
    for t in tickets:
        t.wait()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    g, r = gx.gammax_map(ref, ev, spacing, dd, dta, 0.1, timing=True)
    return ms, g, r


def _sweep_point(gx, torch, np, ref, ev, spacing, dd, dta, args, **extra):
    steps = min(args.steps, gx.ASYNC_SLOTS)
    ms, g, r = _time_maps(gx, torch, ref, ev, spacing, dd, dta, steps, args.warmup)
    gh = g.double()
    gam = gh[gh >= 0]
    # the search proper (the paper's T_gamma): key-0 pass, sort, walk, guard; no prep
    ms_gamma = r.ms_search + r.ms_sort + r.ms_tail + r.ms_guard
    pt = dict(dd=dd, dta=dta, shape=list(ref.shape), spacing_mm=[round(h, 4) for h in spacing],
              n_grid=int(ref.numel()), n_evaluated=int(r.n_evaluated), ms_per_map=round(ms, 4),
              ms_gamma=round(ms_gamma, 4), n_cells=int(r.n_cells), n_tail=int(r.n_tail),
              sum_gamma3=float((gam ** 3).sum().item()), pass_rate=round(r.pass_rate, 6),
              max_gamma=round(r.max_gamma, 4))
    if args.sweep_oracle > 0:
        pt["cpu_baseline"] = _sweep_oracle(np, ref, ev, spacing, dd, dta, g, r, args.sweep_oracle)
    pt.update(extra)
    print(json.dumps(pt), flush=True)
    return pt


def _sweep_oracle(np, ref, ev, spacing, dd, dta, g, r, n_sample):
    """The FP64 oracle beside a sweep point, on a sample of the evaluated nodes (random,
    seeded): its time per node on the host cores, its gamma against the GPU's at those
    nodes, and its visited cells per node against the GPU's total per evaluated node."""
    import oracle

    gh = g.detach().cpu().numpy().ravel()
    masked = np.flatnonzero(gh >= 0)
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(masked, size=min(n_sample, masked.size), replace=False))
    rh, eh = ref.detach().cpu().numpy(), ev.detach().cpu().numpy()
    t0 = time.perf_counter()
    o = oracle.gamma(rh, eh, spacing, dd, dta, 0.1, subset=idx)
    sec = time.perf_counter() - t0
    err = np.abs(gh[idx].astype(np.float64) - o.gamma)
    bar = 1e-5 + 1e-5 * o.gamma
    cells_o = float(o.cells.astype(np.float64).mean())
    return {"kind": "oracle", "sample": f"{idx.size} evaluated nodes drawn at random (seed 7)",
            "cores": oracle.max_threads(), "value": round(idx.size / sec, 1), "unit": "ref voxels/s",
            "max_abs_dgamma": float(err.max()), "n_beyond_tol": int((err > bar).sum()),
            "same_mask": bool(np.all(o.gamma >= 0)),
            "cells_per_node_oracle": round(cells_o, 3),
            "cells_per_node_gpu": round(r.n_cells / max(r.n_evaluated, 1), 3)}


def _fit_line(x, y):
    import numpy as np
    x, y = np.asarray(x, dtype=np.float64), np.asarray(y, dtype=np.float64)
    a, b = np.polyfit(x, y, 1)
    pred = a * x + b
    ss = float(((y - y.mean()) ** 2).sum())
    r2 = 1.0 - float(((y - pred) ** 2).sum()) / ss if ss > 0 else 1.0
    return float(a), float(b), r2


def run_sweep(args):
    """The paper's scaling studies on synthetic pairs, one JSON line per point and a last
    line with the fits:
    * criteria: DD x DTA in {1,2,3}% x {1,2,3} mm on the 256x256x192 workload (Table 3);
    * resolution: the 3D generator over one box at four grid sizes, T ~ N^a (Fig. 2);
    * shift: evaluation dose + s Dmax inside the 10 % region, s = -10 % ... +10 % in 1 %
      steps, on the 256x256x192 workload, T against sum(gamma^3) (Fig. 1b);
    * order: the same pair at five of those shifts, the sort and the walk past the key-0
      cells under each ordering key: none, |DD|, the bound after the key-0 cells, the
      network's gamma_hat, the gamma of the locally linear evaluated dose, and the true
      gamma (a perfect predictor)."""
    import numpy as np
    import torch

    import paper_1012_1900_amd as gx
    from dosegen import make_config_pair, make_pair_3d

    dev = torch.device("cuda", 0)
    kind = args.sweep
    pts = []
    if kind in ("criteria", "shift", "order"):
        cfg, seed, _ = WORKLOADS["3d_256x256x192_1.25mm"]
        pair = make_config_pair(cfg, seed)
        ref = torch.from_numpy(pair.ref).to(dev)
    if kind == "criteria":
        ev = torch.from_numpy(pair.eval).to(dev)
        for dd in (0.01, 0.02, 0.03):
            for dta in (1.0, 2.0, 3.0):
                pts.append(_sweep_point(gx, torch, np, ref, ev, pair.spacing, dd, dta, args))
        t = {(p["dd"], p["dta"]): p["ms_gamma"] for p in pts}
        summary = dict(sweep="criteria", proportional_ms_gamma=[t[(0.01, 1.0)], t[(0.02, 2.0)], t[(0.03, 3.0)]])
    elif kind == "resolution":
        for shape in SWEEP_RESOLUTIONS:
            spacing = tuple(b / n for b, n in zip(SWEEP_BOX_MM, shape))
            log(f"generating {shape}")
            p = make_pair_3d(WORKLOADS["3d_256x256x192_1.25mm"][1], shape=shape, spacing=spacing)
            r_, e_ = torch.from_numpy(p.ref).to(dev), torch.from_numpy(p.eval).to(dev)
            pts.append(_sweep_point(gx, torch, np, r_, e_, spacing, args.dd, args.dta, args))
            del r_, e_
        n = [p["n_grid"] for p in pts]
        a_map, _, r2_map = _fit_line(np.log(n), np.log([p["ms_per_map"] for p in pts]))
        a_g, _, r2_g = _fit_line(np.log(n), np.log([p["ms_gamma"] for p in pts]))
        a_c, _, r2_c = _fit_line(np.log(n), np.log([p["n_cells"] for p in pts]))
        summary = dict(sweep="resolution", exponent_ms_per_map=round(a_map, 3), r2_ms_per_map=round(r2_map, 4),
                       exponent_ms_gamma=round(a_g, 3), r2_ms_gamma=round(r2_g, 4),
                       exponent_cells=round(a_c, 3), r2_cells=round(r2_c, 4))
    elif kind == "shift":
        ev0 = torch.from_numpy(pair.eval).to(dev)
        dmax = float(pair.ref.max())
        region = ref >= 0.1 * dmax
        for k in range(-10, 11):
            ev = torch.where(region, ev0 + (0.01 * k) * dmax, ev0)
            pts.append(_sweep_point(gx, torch, np, ref, ev, pair.spacing, args.dd, args.dta, args, shift=k / 100))
        s3 = [p["sum_gamma3"] for p in pts]
        a, b, r2 = _fit_line(s3, [p["ms_gamma"] for p in pts])
        ac, bc, r2c = _fit_line(s3, [p["n_cells"] for p in pts])
        summary = dict(sweep="shift", ms_gamma_vs_sum_gamma3=dict(slope=a, intercept_ms=round(b, 4), r2=round(r2, 4)),
                       cells_vs_sum_gamma3=dict(slope=ac, intercept=round(bc, 1), r2=round(r2c, 4)))
    elif kind == "order":
        ev0 = torch.from_numpy(pair.eval).to(dev)
        dmax = float(pair.ref.max())
        region = ref >= 0.1 * dmax
        model = None
        if os.path.exists(args.weights):
            model = gx.Model(np.load(args.weights, allow_pickle=False))
        crit = (args.dd, args.dta)
        reps = max(3, min(args.steps, 20))
        for k in (-10, -5, 0, 5, 10):
            ev = torch.where(region, ev0 + (0.01 * k) * dmax, ev0)
            truth, _ = gx.gammax_map(ref, ev, pair.spacing, *crit, 0.1)
            # gamma of the evaluated dose taken as linear around each node: |dD| over the
            # norm of (Delta D, DTA |grad D_e|)
            grads = torch.gradient(ev, spacing=list(pair.spacing))
            g2 = sum(g * g for g in grads)
            lin = ((ev - ref).abs() / torch.sqrt((args.dd * dmax) ** 2 + g2 * args.dta ** 2)).contiguous()
            keys = [("none", {}), ("dd", {"sort": "dd"}), ("bound", {"sort": "bound"})]
            if model is not None:
                keys.append(("gamma_hat", {"sort": "predicted", "model": model, "cnn_pool": 2}))
            keys += [("gamma_lin", {"sort": "given", "order_key": lin}),
                     ("gamma_true", {"sort": "given", "order_key": truth.clamp_min(0.0).contiguous()})]
            if args.tail_lanes:
                for _, kw in keys:
                    kw["tail_lanes"] = args.tail_lanes
            row = dict(shift=k / 100, tail_lanes=args.tail_lanes)
            for name, kw in keys:
                for _ in range(args.warmup):
                    gx.gammax_map(ref, ev, pair.spacing, *crit, 0.1, **kw)
                ph = []
                for _ in range(reps):
                    g, r = gx.gammax_map(ref, ev, pair.spacing, *crit, 0.1, timing=True, **kw)
                    ph.append((r.ms_sort, r.ms_tail, r.ms_cnn))
                if not torch.equal(g, truth):
                    raise RuntimeError(f"order {name}: gamma differs from the unsorted map")
                m = np.mean(np.asarray(ph), axis=0)
                row[name] = dict(ms_sort=round(float(m[0]), 4), ms_tail=round(float(m[1]), 4),
                                 ms_cnn=round(float(m[2]), 4))
            row["n_tail"] = int(r.n_tail)
            print(json.dumps(row), flush=True)
            pts.append(row)
        names = [n for n in pts[0] if isinstance(pts[0][n], dict)]
        summary = dict(sweep="order", ms_tail_mean={n: round(float(np.mean([p[n]["ms_tail"] for p in pts])), 4)
                                                    for n in names})
    elif kind == "grids":
        # the 128x128x96 pair against evaluation doses on other grids over the same box
        cfg, seed, _ = WORKLOADS["3d_128x128x96_2.5mm"]
        pair = make_config_pair(cfg, seed)
        ref = torch.from_numpy(pair.ref).to(dev)
        rs = pair.ref.shape
        for ev_sp, shift in (((2.5, 2.5, 2.5), (0.0, 0.0, 0.0)), ((2.5, 2.5, 2.5), (1.25, 1.25, 1.25)),
                             ((1.25, 1.25, 1.25), (0.0, 0.0, 0.0)), ((5.0, 5.0, 5.0), (0.0, 0.0, 0.0))):
            es = tuple(max(2, int(round(n * h / e))) for n, h, e in zip(rs, pair.spacing, ev_sp))
            pe = make_pair_3d(seed, shape=es, spacing=ev_sp)
            origin = tuple((n - 1) / 2 * h - (m - 1) / 2 * e + d
                           for n, h, m, e, d in zip(rs, pair.spacing, es, ev_sp, shift))
            ev = torch.from_numpy(pe.eval).to(dev)
            out = torch.empty_like(ref)
            for _ in range(args.warmup):
                gx.gammax_map_grids(ref, ev, pair.spacing, ev_sp, origin, args.dd, args.dta, 0.1, out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                _, r = gx.gammax_map_grids(ref, ev, pair.spacing, ev_sp, origin, args.dd, args.dta, 0.1, out=out)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / args.steps
            pt = dict(ev_spacing_mm=list(ev_sp), ev_shape=list(es), shift_mm=list(shift), ms_per_map=round(ms, 4),
                      ref_vox_per_s=round(r.n_evaluated / (ms * 1e-3), 1), n_evaluated=int(r.n_evaluated),
                      n_cells=int(r.n_cells), table_len=int(r.table_len), pass_rate=round(r.pass_rate, 6),
                      max_gamma=round(r.max_gamma, 4))
            print(json.dumps(pt), flush=True)
            pts.append(pt)
            del ev, out
        summary = dict(sweep="grids", ms_per_map=[p["ms_per_map"] for p in pts])
    else:
        raise SystemExit(f"unknown sweep {kind}")
    print(json.dumps(summary), flush=True)


def _mixed_pair(spec):
    from dosegen import make_batch_pair
    p = make_batch_pair(spec)
    return p.ref, p.eval, p.spacing


def run_mixed(args):
    """The mixed batch through gammax_map_many (a cached context per pair, the maps on the
    current stream and three internal ones), every result collected inside the timed
    region: the aggregate ref voxels/s.
    The per-pair GPU time (HIP events around each map, one context per pair, maps queued
    round-robin on --streams streams) is reported at p50 / p99."""
    import multiprocessing as mp

    import numpy as np

    from dosegen import batch_specs

    name, seed, n = MIXED
    specs = batch_specs(seed, n, 1.0)
    log(f"generating {n} pairs")
    # the inputs are made in worker processes before this process touches the GPU
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        pairs = pool.map(_mixed_pair, specs)

    import torch

    import paper_1012_1900_amd as gx

    dev = torch.device("cuda", 0)
    streams = [torch.cuda.current_stream(dev)] + [torch.cuda.Stream(dev) for _ in range(max(1, args.streams) - 1)]
    data = []
    for k, (sp, (r, e, h)) in enumerate(zip(specs, pairs)):
        rt = torch.from_numpy(r).to(dev)
        et = torch.from_numpy(e).to(dev)
        data.append(dict(ref=rt, ev=et, out=torch.empty_like(rt), spacing=h, dd=sp.dd, dta=sp.dta,
                         local=sp.local, ctx=gx.Context(0), stream=streams[k % len(streams)], spec=sp))
    del pairs
    torch.cuda.synchronize()

    def one(q):
        return gx.gammax_map_async(q["ref"], q["ev"], q["spacing"], q["dd"], q["dta"], 0.1, q["local"],
                                   sort=args.sort, out=q["out"], ctx=q["ctx"], stream=q["stream"])

    log("warm-up (tables and graphs)")
    many_ctx = gx.Context(0)
    kw = dict(sort=args.sort, ctx=many_ctx, outs=[q["out"] for q in data])
    for _ in range(max(1, args.warmup)):
        gx.gammax_map_many(data, **kw)
        for q in data:
            one(q).wait()
    torch.cuda.synchronize()
    log(f"timing {args.steps} passes over the batch")
    M = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, rs = gx.gammax_map_many(data, **kw)
        M += sum(r.n_evaluated for r in rs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-pair GPU time: events around each queued map
    ms, tails = [], []
    for q in data:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(q["stream"])
        t = one(q)
        e1.record(q["stream"])
        tails.append(t.wait().n_tail)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    ms = np.array(ms)
    slow = [dict(shape=list(data[k]["spec"].shape), spacing_mm=round(data[k]["spec"].spacing[0], 3),
                 criteria=f"{data[k]['dd'] * 100:g}%/{data[k]['dta']:g}mm", local=data[k]["local"],
                 n_tail=int(tails[k]), ms=round(float(ms[k]), 4)) for k in np.argsort(-ms)[:5]]
    # the same batch as one captured graph (gammax_batch): plain, then with the learned
    # radius of the shipped network; results compared with the queued maps bit for bit
    outs_many = [q["out"].clone() for q in data]
    outs_b = [torch.empty_like(q["ref"]) for q in data]

    def batch_leg(**bkw):
        bctx = gx.Context(0)
        for _ in range(max(1, args.warmup)):
            gx.gammax_batch(data, ctx=bctx, outs=outs_b, sort=args.sort, **bkw)
        torch.cuda.synchronize()
        Mb, done = 0, None
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, rs = gx.gammax_batch(data, ctx=bctx, outs=outs_b, sort=args.sort, **bkw)
            Mb += sum(r.n_evaluated for r in rs)
            done = np.array([r.ms_done for r in rs])
        torch.cuda.synchronize()
        wb = time.perf_counter() - t0
        same = all(torch.equal(a, b) for a, b in zip(outs_b, outs_many))
        return {"value": round(Mb / wb, 1), "ms_per_step": round(1e3 * wb / args.steps, 4),
                "pair_done_ms_p50": round(float(np.percentile(done, 50)), 4),
                "pair_done_ms_p99": round(float(np.percentile(done, 99)), 4),
                "pair_done_ms_max": round(float(done.max()), 4),
                "n_fallback": int(sum(r.n_fallback for r in rs)),
                "identical_to_queued_maps": bool(same)}

    log("gammax_batch (one captured graph), plain")
    batch_plain = batch_leg()
    batch_learned = None
    if not args.no_learned and os.path.exists(args.weights):
        log("gammax_batch, learned radius")
        model = gx.Model(np.load(args.weights, allow_pickle=False))
        batch_learned = batch_leg(radius="learned", model=model)
        batch_learned["weights"] = os.path.relpath(args.weights, ROOT)
    nodes = sum(q["ref"].numel() for q in data)
    line = {
        "metric": "ref voxels/sec, mixed batch of 64 pairs (2D/3D, 3/3-2/2-1/1, global/local)",
        "value": round(M / wall, 1),
        "unit": "ref voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{n} mixed pairs (seeds {seed + 1}-{seed + n}): 2D 128-200^2 or 3D 128-200^2 x 96-150 "
                        "at 1-2 mm, criteria 3%/3mm, 2%/2mm or 1%/1mm, global or local, 10% cutoff",
            "submission": "gammax_map_many: a cached context per pair, the maps on four streams; a step is "
                          "one call over all pairs",
            "pairs": n,
            "grid_nodes": int(nodes),
            "evaluated_per_step": int(M // args.steps),
            "pair_ms_p50": round(float(np.percentile(ms, 50)), 4),
            "pair_ms_p99": round(float(np.percentile(ms, 99)), 4),
            "pair_ms_max": round(float(ms.max()), 4),
            "streams": len(streams),
            "sort": args.sort,
            "slowest_pairs": slow,
            "batch_graph": {
                "submission": "gammax_batch: one captured HIP graph per batch (every pair's compaction, one "
                              "key-0 launch over all pairs' nodes in cost order, every pair's tail, guard and "
                              "counts), replayed; per-pair completion times from the device clock",
                "plain": batch_plain,
                "learned": batch_learned,
            },
        },
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + [MIXED[0]], default="3d_128x128x96_2.5mm")
    ap.add_argument("--dd", type=float, default=0.03)
    ap.add_argument("--dta", type=float, default=3.0)
    ap.add_argument("--sort", choices=["dd", "bound", "none"], default="none")
    ap.add_argument("--precision", choices=["fp32", "guarded", "fp64"], default="guarded")
    ap.add_argument("--tail-lanes", type=int, default=0, choices=[0, 1, 8, 16, 32, 64])
    ap.add_argument("--cell-lanes", type=int, default=0, choices=[0, 1, 4, 8])
    ap.add_argument("--projection", choices=["faces", "ju"], default="faces",
                    help="key-0 pass: every owned face without branches, or Ju et al.'s recursion")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-radius leg")
    ap.add_argument("--no-c2", action="store_true", help="skip the 256x256x192 leg")
    ap.add_argument("--cnn-pool", type=int, choices=[0, 2], default=None,
                    help="learned leg: network input pooling (default: 2 on a grid at half the training "
                         "spacing, else 0; 0 runs the per-node network at every tail node)")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1012_1900_amd", "weights",
                                                      "cnn_3d_2.5mm_3pct3mm.npy"))
    ap.add_argument("--cpu-reps", type=int, default=2, help="fewest oracle repetitions")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="least CPU time the oracle baseline runs for")
    ap.add_argument("--sweep-oracle", type=int, default=4096,
                    help="sweeps: evaluated nodes per point on which the FP64 oracle runs beside the GPU (0: none)")
    ap.add_argument("--sweep", choices=["criteria", "resolution", "shift", "order", "grids"], default=None,
                    help="run one of the paper's scaling studies instead of the benchmark line")
    ap.add_argument("--concurrent", type=int, default=16,
                    help="also time this many copies of the map per gammax_map_many call (0: skip)")
    ap.add_argument("--streams", type=int, default=4,
                    help="mixed batch: spread the pairs round-robin over this many streams (the GPU "
                         "runs 4 hardware queues per process)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (a profiler reference "
                         "for the HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the gamma search of one dose pair is measured on a "
              "single MI355X (--gpus 1).", file=sys.stderr)
        sys.exit(2)

    if args.workload == MIXED[0]:
        run_mixed(args)
        return
    if args.sweep:
        run_sweep(args)
        return

    import numpy as np
    import torch

    import paper_1012_1900_amd as gx
    from dosegen import make_config_pair

    cfg, seed, desc = WORKLOADS[args.workload]
    log(f"generating {desc}")
    pair = make_config_pair(cfg, seed)
    nd = pair.ref.ndim
    dev = torch.device("cuda", 0)
    ref = torch.from_numpy(pair.ref).to(dev)
    ev = torch.from_numpy(pair.eval).to(dev)
    out = torch.empty_like(ref)
    torch.cuda.synchronize()

    if args.copy_mib > 0:
        n_copy = args.copy_mib * (1 << 20) // 4
        src = torch.ones(n_copy, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def leg(p, r_dev, e_dev, o_dev, extra, steps):
        """W warm-up maps; `steps` timed maps queued back to back (gammax_map_async: the host
        work of the next map overlaps the GPU's work on the current one, every result
        collected inside the timed region); `steps` synchronous maps (gammax_map: one host round trip each); then
        `steps` maps with HIP events per phase.  Returns (seconds per queued map, seconds per
        synchronous map, the last queued map's result, the phase results)."""
        kw = dict(sort=args.sort, precision=args.precision, tail_lanes=args.tail_lanes,
                  cell_lanes=args.cell_lanes, projection=args.projection, out=o_dev)
        kw.update(extra)
        for _ in range(args.warmup):
            gx.gammax_map(r_dev, e_dev, p.spacing, args.dd, args.dta, 0.1, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        queue = collections.deque()
        results = []
        for _ in range(steps):
            if len(queue) == gx.ASYNC_SLOTS:
                results.append(queue.popleft().wait())
            queue.append(gx.gammax_map_async(r_dev, e_dev, p.spacing, args.dd, args.dta, 0.1, **kw))
        while queue:
            results.append(queue.popleft().wait())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(steps):
            gx.gammax_map(r_dev, e_dev, p.spacing, args.dd, args.dta, 0.1, **kw)
        torch.cuda.synchronize()
        sync = (time.perf_counter() - t0) / steps
        phases = []
        for _ in range(steps):
            _, r = gx.gammax_map(r_dev, e_dev, p.spacing, args.dd, args.dta, 0.1, timing=True, **kw)
            phases.append(r)
        torch.cuda.synchronize()
        return wall / steps, sync, results[-1], phases

    def mean(f, ph):
        return float(np.mean([getattr(q, f) for q in ph]))

    model = None
    if nd == 3 and not args.no_learned and os.path.exists(args.weights):
        model = gx.Model(np.load(args.weights, allow_pickle=False))

    def learned_leg(p, r_dev, e_dev, o_dev, g_plain, sec_plain, steps):
        """The learned radius on the same pair: speculative walk inside 1.1 gamma_hat, the
        tail ordered by the prediction (the network's inference inside the timed map)."""
        # the network was trained on a 2.5 mm grid: a grid at half that spacing feeds it the
        # pair average-pooled 2x2x2 and interpolates its prediction back
        cnn_pool = 2 if all(abs(2.0 * h - TRAIN_SPACING_MM) < 1e-9 for h in p.spacing) else 0
        if args.cnn_pool is not None:
            cnn_pool = args.cnn_pool
        log(f"learned radius (cnn_pool {cnn_pool})")
        lsec, lsync, lr_last, lph = leg(p, r_dev, e_dev, o_dev,
                                        dict(radius="learned", sort="predicted", model=model, cnn_pool=cnn_pool),
                                        steps)
        ms_cnn = mean("ms_cnn", lph)
        # algorithmic MACs of the network at one tail node, from its 9^3 patch: layer l
        # produces (7 - 2 l)^3 outputs of its per-output MACs
        macs_node = sum((7 - 2 * l) ** 3 * m
                        for l, m in enumerate((2 * 16 * 27, 16 * 16 * 27, 16 * 16 * 27, 16 * 27)))
        macs = macs_node * int(lr_last.n_tail)
        if cnn_pool:
            # pooled input: the whole coarse grid, 15,120 MACs per coarse node
            coarse = int(np.prod([(n + 1) // 2 for n in p.ref.shape]))
            macs = coarse * sum(m for m in (2 * 16 * 27, 16 * 16 * 27, 16 * 16 * 27, 16 * 27))
        cnn_tflops = 2 * macs / (ms_cnn * 1e-3) / 1e12
        res = {
            "value": round(lr_last.n_evaluated / lsec, 1),
            "ms_per_step": round(1e3 * lsec, 4),
            "ms_per_step_sync": round(1e3 * lsync, 4),
            "speedup_vs_plain": round(sec_plain / lsec, 3),
            "n_tail": int(lr_last.n_tail),
            "n_fallback": int(lr_last.n_fallback),
            "identical_to_plain": bool(torch.equal(o_dev, g_plain)),
            "phases_ms": {k: round(mean(k, lph), 4) for k in ("ms_prep", "ms_cnn", "ms_search", "ms_sort",
                                                              "ms_tail", "ms_guard")},
            "weights": os.path.relpath(args.weights, ROOT),
            "cnn_pool": cnn_pool,
            "cnn_roofline": {"bound": "mfma", "achieved": round(cnn_tflops, 2), "peak": PEAK_BF16_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(cnn_tflops / PEAK_BF16_TFLOPS, 4),
                             "algorithmic_flop_per_launch": int(2 * macs),
                             "flop_per_tail_node": None if cnn_pool else int(2 * macs_node),
                             "avg_launch_ms": round(ms_cnn, 5)},
        }
        log(f"learned: {res['ms_per_step']} ms/step, {res['n_fallback']}/{res['n_tail']} fallbacks")
        return res

    log(f"plain search: warmup {args.warmup}, timing {args.steps} steps")
    sec, sync_sec, r_last, phases = leg(pair, ref, ev, out, {}, args.steps)
    sync_ms = 1e3 * sync_sec
    g_plain = out.clone()
    ms_per_step = 1e3 * sec
    M = r_last.n_evaluated
    value = M / sec
    ms_search = mean("ms_search", phases)
    log(f"{M} nodes, {ms_per_step:.3f} ms/step, search {ms_search:.4f} ms")

    # the same map many times at once (gammax_map_many: a context per copy, the maps on four
    # streams, so one map's latency-bound phases overlap another's key-0 pass); reported
    # beside the value, which stays the one-map-at-a-time rate
    concurrent = None
    if args.concurrent > 1:
        nc = args.concurrent
        many = [dict(ref=ref, ev=ev, spacing=pair.spacing, dd=args.dd, dta=args.dta) for _ in range(nc)]
        mkw = dict(sort=args.sort, precision=args.precision, tail_lanes=args.tail_lanes)
        mctx = gx.Context(0)
        for _ in range(max(1, args.warmup)):
            gx.gammax_map_many(many, ctx=mctx, **mkw)
        torch.cuda.synchronize()
        calls = max(1, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(calls):
            gs, rs = gx.gammax_map_many(many, ctx=mctx, **mkw)
        torch.cuda.synchronize()
        csec = (time.perf_counter() - t0) / (calls * nc)
        if not all(torch.equal(g, g_plain) for g in gs):
            raise RuntimeError("a concurrent map differs from the single map")
        concurrent = {"maps_per_call": nc, "calls": calls, "value": round(M / csec, 1),
                      "unit": "ref voxels/s", "ms_per_map": round(1e3 * csec, 4),
                      "submission": "gammax_map_many of the same pair, a cached context per copy, four streams"}
        log(f"concurrent: {1e3 * csec:.4f} ms/map over {nc} maps per call")
        del mctx

    learned = None
    g_learned = None
    if model is not None:
        learned = learned_leg(pair, ref, ev, out, g_plain, sec, args.steps)
        g_learned = out.clone()

    wc = work_counts(cfg, seed, args.dd, args.dta)
    cells = wc["cells_visited"] if wc else None
    roofline = None
    if wc:
        # dominant kernel: the pass over the key-0 cells of every node
        flops = wc["cells_visited_key0"] * FLOP_PER_CELL_REFERENCE[nd]
        flops_cf = wc["cells_visited_key0"] * FLOP_PER_CELL[nd]
        achieved = flops / (ms_search * 1e-3) / 1e12
        achieved_cf = flops_cf / (ms_search * 1e-3) / 1e12
        kern = "k_zero_group" if args.cell_lanes in (4, 8) else ("k_zero3" if nd == 3 else "k_zero2")
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                    "traffic": traffic_bytes(args.workload, kern == "k_zero3" and args.dd == 0.03
                                             and args.dta == 3.0 and args.precision == "guarded"),
                    "kernel": f"{kern} (key-0 cells of every node)",
                    "flop_per_cell": FLOP_PER_CELL_REFERENCE[nd],
                    "algorithmic_flop_per_launch": flops, "avg_launch_ms": round(ms_search, 5),
                    "closed_form": {"flop_per_cell": FLOP_PER_CELL[nd], "achieved": round(achieved_cf, 3),
                                    "frac": round(achieved_cf / PEAK_FP32_TFLOPS, 4)}}

    cpu = None
    acc = None
    if not args.no_cpu:
        log("cpu baseline (FP64 oracle)")
        cpu, o = cpu_baseline(pair, args.dd, args.dta, args.cpu_reps, args.cpu_seconds)
        if cells is None:
            cells = o.cells_visited
        acc = {"plain": accuracy(g_plain, o)}
        if g_learned is not None:
            acc["learned"] = accuracy(g_learned, o)
            learned["accuracy"] = acc["learned"]
        log(f"accuracy against the oracle: {acc}")

    # the 256x256x192 pair (the learned radius's target workload): plain and learned maps,
    # each checked against the oracle
    c2 = None
    if not args.no_c2 and args.workload != "3d_256x256x192_1.25mm" and nd == 3:
        cfg2, seed2, desc2 = WORKLOADS["3d_256x256x192_1.25mm"]
        log(f"generating {desc2}")
        pair2 = make_config_pair(cfg2, seed2)
        ref2 = torch.from_numpy(pair2.ref).to(dev)
        ev2 = torch.from_numpy(pair2.eval).to(dev)
        out2 = torch.empty_like(ref2)
        steps2 = max(5, args.steps)
        log("256x256x192 plain")
        sec2, sync2, r2, ph2 = leg(pair2, ref2, ev2, out2, {}, steps2)
        g2 = out2.clone()
        c2 = {"workload": f"{desc2}, {args.dd * 100:g}%/{args.dta:g}mm global, 10% cutoff",
              "n_evaluated": int(r2.n_evaluated),
              "plain": {"value": round(r2.n_evaluated / sec2, 1), "ms_per_step": round(1e3 * sec2, 4),
                        "ms_per_step_sync": round(1e3 * sync2, 4), "n_tail": int(r2.n_tail),
                        "phases_ms": {k: round(mean(k, ph2), 4) for k in ("ms_prep", "ms_search", "ms_sort",
                                                                          "ms_tail", "ms_guard")}},
              "learned": None}
        if model is not None:
            c2["learned"] = learned_leg(pair2, ref2, ev2, out2, g2, sec2, steps2)
        if not args.no_cpu:
            log("256x256x192 oracle")
            t0 = time.perf_counter()
            o2 = oracle_gamma(pair2, args.dd, args.dta)
            c2["oracle_s"] = round(time.perf_counter() - t0, 2)
            c2["plain"]["accuracy"] = accuracy(g2, o2)
            if c2["learned"] is not None:
                c2["learned"]["accuracy"] = accuracy(out2, o2)
        del ref2, ev2, out2, g2

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "ref voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision != "fp64" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{desc}, {args.dd * 100:g}%/{args.dta:g}mm global, 10% cutoff, plain search",
            "submission": "maps queued back to back (gammax_map_async), every result collected in the timed region",
            "ms_per_step_sync": round(sync_ms, 4),
            "concurrent_maps": concurrent,
            "grid_vox_per_s": round(pair.ref.size / sec, 1),
            "search_only_vox_per_s": round(M / (ms_search * 1e-3), 1),
            "shape": list(pair.ref.shape),
            "spacing_mm": list(pair.spacing),
            "n_evaluated": int(M),
            "sort": args.sort,
            "precision": args.precision,
            "projection": args.projection,
            "cells_visited_oracle": cells,
            "n_tail": int(phases[-1].n_tail),
            "phases_ms": {k: round(mean(k, phases), 4) for k in ("ms_prep", "ms_table", "ms_search", "ms_sort",
                                                                 "ms_tail", "ms_guard")},
        },
        "accuracy": acc["plain"] if acc else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "learned": learned,
        "c2": c2,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
