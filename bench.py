#!/usr/bin/env python
"""Benchmark: MLS r^-6 energy-and-force evaluations per second on one MI355X.

One step = one full evaluation (binning, local pair sum, anterpolation,
restrictions, level stencils, coarsest all-to-all, prolongations,
interpolation, energy) of the 1,000,000-atom homogeneous LJ cube at density
0.8 (a = 3, h = 1 -> 112^3 finest grid, cubic basis, 5 levels), inputs
resident in HBM.  The evaluation is captured into a graph; after W warm-up
replays, K replays are timed in equal blocks with events and the median block
gives the rate.  Both precisions are timed; ``value`` is the FP32-mixed rate,
with the FP64 rate, their ratio, the accuracy of each against the FP64 oracle
and the discretisation error against the exact sum beside it.

    python bench.py [--steps K] [--warmup W] [--blocks B] [--gpus 1]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"hbm": 8000.0, "fp64": 78.6, "fp32": 157.3}   # GB/s, TFLOP/s (MI355X published)
PAIR_FLOPS = 39        # flops of one ordered in-cutoff pair in the pair kernel's formula
STENCIL_FLOPS = 2      # one multiply-add per tap and grid point


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def count_pairs(pos, box, a):
    """Ordered pairs (i != j) closer than a (minimum image; a < L/2)."""
    from scipy.spatial import cKDTree
    import numpy as np
    t = cKDTree(np.mod(pos, box), boxsize=box)
    return int(t.count_neighbors(t, a)) - len(pos)


def work_model(plan_info, n, pairs, order):
    """Algorithmic work per evaluation for each stage (flops or bytes)."""
    g = plan_info["grid"]
    l = plan_info["levels"]
    pts = [(g[0] >> k) * (g[1] >> k) * (g[2] >> k) for k in range(l)]
    sum_lt = sum(pts[:-1])
    p3 = order ** 3
    return {
        "pair": dict(bound="alu", flops=PAIR_FLOPS * pairs),
        "stencil": dict(bound="alu", flops=STENCIL_FLOPS * plan_info["taps"] * sum_lt),
        # read sorted x,y,z,xi (32 B) per atom, p^3 grid updates (8 B read + 8 B write)
        "anterpolation": dict(bound="hbm", bytes=32 * n + 16 * min(p3 * n, pts[0])),
        # read atoms + E^1 once, write F (24), u, dE/dc6 (8+8), read e0/floc (32)
        "interpolation": dict(bound="hbm", bytes=32 * n + 8 * pts[0] + 40 * n + 32 * n),
        "restriction": dict(bound="hbm", bytes=8 * sum(pts[:-1]) + 8 * sum(pts[1:])),
        "prolongation": dict(bound="hbm", bytes=16 * sum(pts[:-1]) + 8 * sum(pts[1:])),
        "binning": dict(bound="hbm", bytes=112 * n),
        # FP64 in both precisions
        "coarsest": dict(bound="alu", flops=2 * pts[-1] ** 2, fp64=True),
    }


def stage_rooflines(stage_ms, model, precision):
    """Achieved rate of every timed stage against its roofline: ALU stages in
    TFLOP/s of the stage's algorithmic flops (against the published FP64
    peak, or for FP32 against the published 157.3 TFLOP/s, which needs packed
    FP32, and the 78.6 TFLOP/s of unpacked FP32 that this build issues);
    HBM stages in GB/s of algorithmic bytes against 8 TB/s."""
    out = {}
    for st, ms in stage_ms.items():
        m = model.get(st)
        if m is None or ms <= 0:
            continue
        dt = ms * 1e-3
        if m["bound"] == "hbm":
            a = m["bytes"] / dt / 1e9
            out[st] = {"bound": "hbm", "ms": ms, "bytes": m["bytes"], "achieved": a, "unit": "GB/s",
                       "peak": PEAK["hbm"], "frac": a / PEAK["hbm"]}
        else:
            a = m["flops"] / dt / 1e12
            f32 = precision == "mixed" and not m.get("fp64")
            peak = PEAK["fp32" if f32 else "fp64"]
            r = {"bound": "alu", "ms": ms, "flops": m["flops"], "achieved": a, "unit": "TFLOP/s", "peak": peak,
                 "frac": a / peak}
            if f32:
                r["peak_unpacked_fp32"] = PEAK["fp64"]
                r["frac_unpacked_fp32"] = a / PEAK["fp64"]
            out[st] = r
    return out


# kernels that carry each stage of the 10^6-atom cube (cell width a/2 there)
STAGE_KERNEL = {("pair", "mixed"): ["void k_one<PairTrimF32<2, false, false> >"],
                ("pair", "fp64"): ["void k_one<PairTrimF64<2, false, false> >"],
                ("stencil", "mixed"): ["void k_stencil_tile<float, 6, 16, 8>"],
                ("stencil", "fp64"): ["void k_stencil_tile<double, 6, 8, 8>"],
                ("anterpolation", "mixed"): ["void k_one<AnterpTile<4, float, 2744> >", "void k_one<AnterpCollect>"],
                ("anterpolation", "fp64"): ["void k_one<AnterpTile<4, double, 2744> >", "void k_one<AnterpCollect>"],
                ("interpolation", "mixed"): ["void k_one<InterpTile<4, float, 2744> >"],
                ("interpolation", "fp64"): ["void k_one<InterpTile<4, double, 2744> >"]}


def measured_traffic(stage, precision):
    """HBM bytes per launch of the stage's kernels, from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE record (calibrated on a plain copy); None
    when no record exists or any kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    names = STAGE_KERNEL.get((stage, precision))
    if names is None or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    csrc = os.path.join(ROOT, "paper_1308_4005_amd", "csrc")
    for f, h in rec["sources_sha1"].items():
        fp = os.path.join(csrc, f)
        if not os.path.exists(fp) or hashlib.sha1(open(fp, "rb").read()).hexdigest() != h:
            return None
    total = 0.0
    for name in names:
        k = rec["kernels"].get(name)
        if k is None:
            return None
        total += k["read_bytes"] + k["write_bytes"]
    return total


def time_graph(run, steps, warmup, blocks, dev):
    """Capture ``run`` (one evaluation) into a graph, replay it ``warmup``
    times, then time ``steps`` replays in ``blocks`` equal blocks with events;
    returns (median block ms per replay, every block's ms per replay)."""
    import statistics
    import torch
    run()                                   # eager once: lazily created streams exist before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for _ in range(warmup):
        g.replay()
    per = max(1, steps // blocks)
    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(blocks + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for b in range(blocks):
        for _ in range(per):
            g.replay()
        ev[b + 1].record(stream)
    torch.cuda.synchronize()
    block_ms = [ev[b].elapsed_time(ev[b + 1]) / per for b in range(blocks)]
    del g
    return statistics.median(block_ms), block_ms


def time_precision(w, prm, precision, steps, warmup, dev, continuity=2, stages=True, blocks=0):
    """Evaluations of one plan on the workload.  With ``blocks`` > 0 the
    evaluation is captured into a graph and ``ms`` is the median block of
    replays; ``eager_ms`` is always the rate of plain evaluate calls."""
    import torch
    from paper_1308_4005_amd import Plan, Result
    plan = Plan(w.box, prm["a"], prm["h"], prm["order"], prm["levels"], precision=precision,
                n_max=w.n, device=dev.index, continuity=continuity)
    pos = torch.tensor(w.pos, dtype=torch.float64, device=dev)
    c6 = torch.tensor(w.c6, dtype=torch.float64, device=dev)
    out = Result(torch.empty(1, dtype=torch.float64, device=dev),
                 torch.empty((w.n, 3), dtype=torch.float64, device=dev))
    for _ in range(warmup):
        plan.evaluate(pos, c6, out=out)
    eager_steps = steps if blocks == 0 else max(5, steps // 5)
    stream = torch.cuda.current_stream(dev)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(eager_steps):
        plan.evaluate(pos, c6, out=out)
    t1.record(stream)
    torch.cuda.synchronize()
    eager_ms = t0.elapsed_time(t1) / eager_steps
    ms, block_ms = eager_ms, None
    if blocks > 0:
        ms, block_ms = time_graph(lambda: plan.evaluate(pos, c6, out=out), steps, warmup, blocks, dev)
    # stage breakdown: library hipEvents at every stage boundary (in this mode
    # the stages run one after another on one stream)
    stage_ms = {}
    if stages:
        plan.set_timing(True)
        for _ in range(min(steps, 200)):
            plan.evaluate(pos, c6, out=out)
        torch.cuda.synchronize()
        stage_ms, cnt = plan.read_timing()
        plan.set_timing(False)
        stage_ms = {k: v / max(cnt, 1) for k, v in stage_ms.items()}
    E = float(out.energy.cpu()[0])
    F = out.forces.cpu().numpy()
    info = plan.info
    plan.close()
    return dict(ms=ms, eager_ms=eager_ms, block_ms=block_ms, stage_ms=stage_ms, E=E, F=F, info=info)


def time_stencil_mfma(w, prm, dev, steps):
    """Stencil stage of a mixed plan on the MFMA recast of the FP32 tile
    (selected by MLS_STENCIL_MFMA=1 at plan creation), library hipEvents as
    for the other stage times; None where the window exceeds its range."""
    import torch
    from paper_1308_4005_amd import Plan, Result
    old = os.environ.get("MLS_STENCIL_MFMA")
    os.environ["MLS_STENCIL_MFMA"] = "1"
    try:
        plan = Plan(w.box, prm["a"], prm["h"], prm["order"], prm["levels"], precision="mixed", n_max=w.n,
                    device=dev.index)
    finally:
        if old is None:
            del os.environ["MLS_STENCIL_MFMA"]
        else:
            os.environ["MLS_STENCIL_MFMA"] = old
    if plan.info["stencil_path"] != "tile_mfma_f32":
        plan.close()
        return None
    pos = torch.tensor(w.pos, dtype=torch.float64, device=dev)
    c6 = torch.tensor(w.c6, dtype=torch.float64, device=dev)
    out = Result(torch.empty(1, dtype=torch.float64, device=dev),
                 torch.empty((w.n, 3), dtype=torch.float64, device=dev))
    for _ in range(3):
        plan.evaluate(pos, c6, out=out)
    plan.set_timing(True)
    for _ in range(steps):
        plan.evaluate(pos, c6, out=out)
    torch.cuda.synchronize()
    stage_ms, cnt = plan.read_timing()
    plan.close()
    return stage_ms["stencil"] / max(cnt, 1)


def time_batched(ws, precision, steps, warmup, dev):
    """The batched form on the many-box workload: one graph replay per step
    (all boxes), after autotuning on the first call; beside it the same boxes
    evaluated one single plan after another on the same stream."""
    import numpy as np
    import torch
    from paper_1308_4005_amd import BatchPlan, Plan, Result
    bp = BatchPlan([w.box for w in ws], [w.n for w in ws], 3.0, 1.0, 4, 0, precision=precision, autotune=True,
                   device=dev.index)
    pos = torch.tensor(np.concatenate([w.pos for w in ws]), dtype=torch.float64, device=dev)
    c6 = torch.tensor(np.concatenate([w.c6 for w in ws]), dtype=torch.float64, device=dev)
    out = bp.evaluate(pos, c6)
    for _ in range(warmup):
        bp.evaluate(pos, c6, out=out)
    stream = torch.cuda.current_stream(dev)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        bp.evaluate(pos, c6, out=out)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    tuning = bp.tuning()
    E_batch = out.energies.cpu().numpy()
    bp.close()
    # the same boxes through single plans, one evaluate call per box
    plans, outs = [], []
    off = np.concatenate([[0], np.cumsum([w.n for w in ws])])
    for b, w in enumerate(ws):
        plans.append(Plan(w.box, 3.0, 1.0, 4, 0, precision=precision, n_max=w.n, device=dev.index))
        outs.append(Result(torch.empty(1, dtype=torch.float64, device=dev),
                           torch.empty((w.n, 3), dtype=torch.float64, device=dev)))
    views = [(pos[off[b]:off[b + 1]], c6[off[b]:off[b + 1]]) for b in range(len(ws))]

    def sweep():
        for pl, (p, c), o in zip(plans, views, outs):
            pl.evaluate(p, c, out=o)
    sweep()
    seq_steps = max(2, min(20, steps // 4))
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(seq_steps):
        sweep()
    t1.record(stream)
    torch.cuda.synchronize()
    ms_seq = t0.elapsed_time(t1) / seq_steps
    E_seq = np.array([float(o.energy.cpu()[0]) for o in outs])
    for pl in plans:
        pl.close()
    n = int(off[-1])
    return {"ms_per_step": ms, "batch_evals_per_s": 1000.0 / ms, "particle_evals_per_s": n * 1000.0 / ms,
            "sequential_single_plans_ms": ms_seq, "speedup_vs_sequential": ms_seq / ms,
            "max_rel_energy_diff_vs_single": float(np.max(np.abs(E_batch - E_seq) / np.abs(E_seq))),
            "tuning": tuning}


def lb_species(n, seed):
    """Two species drawn 50/50: epsilon in {1.0, 0.6}, sigma in {1.0, 1.25}."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return np.where(rng.uniform(size=n) < 0.5, 1.0, 0.6), np.where(rng.uniform(size=n) < 0.5, 1.0, 1.25)


def time_lb(w, prm, steps, warmup, dev, precision="fp64"):
    """Lorentz-Berthelot mixing (mls_evaluate_lb) on the same positions with
    two species drawn 50/50 (seed 17): epsilon in {1.0, 0.6}, sigma in
    {1.0, 1.25}."""
    import torch
    from paper_1308_4005_amd import Plan, Result
    eps, sig = lb_species(w.n, 17)
    plan = Plan(w.box, prm["a"], prm["h"], prm["order"], prm["levels"], n_max=w.n, device=dev.index,
                mixing="lorentz-berthelot", precision=precision)
    pos = torch.tensor(w.pos, dtype=torch.float64, device=dev)
    te = torch.tensor(eps, dtype=torch.float64, device=dev)
    ts = torch.tensor(sig, dtype=torch.float64, device=dev)
    out = Result(torch.empty(1, dtype=torch.float64, device=dev),
                 torch.empty((w.n, 3), dtype=torch.float64, device=dev))
    for _ in range(warmup):
        plan.evaluate_lb(pos, te, ts, out=out)
    stream = torch.cuda.current_stream(dev)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        plan.evaluate_lb(pos, te, ts, out=out)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    E = float(out.energy.cpu()[0])
    plan.close()
    return {"workload": f"{w.name} positions, two species 50/50: eps {{1.0, 0.6}}, sigma {{1.0, 1.25}} (seed 17)",
            "precision": precision, "ms_per_step": ms, "evals_per_s": 1000.0 / ms, "energy": E}


def time_batched_lb(ws, precision, steps, warmup, dev):
    """The batched Lorentz-Berthelot form (mls_batch_evaluate_lb) on the
    many-box workload, two species per box as for the single plan (seed 17
    over the concatenated atoms), after autotuning on the first call."""
    import numpy as np
    import torch
    from paper_1308_4005_amd import BatchPlan
    bp = BatchPlan([w.box for w in ws], [w.n for w in ws], 3.0, 1.0, 4, 0, precision=precision, autotune=True,
                   device=dev.index, mixing="lorentz-berthelot")
    n = sum(w.n for w in ws)
    eps, sig = lb_species(n, 17)
    t = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    pos, te, ts = t(np.concatenate([w.pos for w in ws])), t(eps), t(sig)
    out = bp.evaluate_lb(pos, te, ts)
    for _ in range(warmup):
        bp.evaluate_lb(pos, te, ts, out=out)
    stream = torch.cuda.current_stream(dev)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(steps):
        bp.evaluate_lb(pos, te, ts, out=out)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    bp.close()
    return {"precision": precision, "boxes": len(ws), "atoms": n, "ms_per_step": ms,
            "batch_evals_per_s": 1000.0 / ms, "particle_evals_per_s": n * 1000.0 / ms}


def time_md(w, prm, precision, steps, warmup, dev, blocks, chunk=50, dt=0.001):
    """Molecular dynamics on the workload (mls_md_run): LJ atoms with
    C6 = 4, C12 = 4 (epsilon = sigma = 1), unit masses, velocities drawn
    from N(0, 0.8) (seed 29), repulsion cutoff a.  One graph replay runs
    ``chunk`` velocity-Verlet steps; ``ms_per_step`` is the median block of
    replays divided by ``chunk`` (a call evaluates the forces chunk + 1
    times: once at its starting positions, then once per step).  Also times
    one mls_evaluate_md (dispersion plus repulsion) the same way, and
    multiple time stepping (mls_md_run_mts, grid part every 4 steps) in
    48-step calls continuing the same trajectory."""
    import numpy as np
    import torch
    from paper_1308_4005_amd import Plan, Result
    rng = np.random.default_rng(29)
    plan = Plan(w.box, prm["a"], prm["h"], prm["order"], prm["levels"], precision=precision, n_max=w.n,
                device=dev.index)
    x = torch.tensor(w.pos, dtype=torch.float64, device=dev)
    v = torch.tensor(rng.normal(scale=np.sqrt(0.8), size=(w.n, 3)), dtype=torch.float64, device=dev)
    c6 = torch.tensor(w.c6, dtype=torch.float64, device=dev)
    c12 = torch.full((w.n,), 4.0, dtype=torch.float64, device=dev)
    im = torch.ones(w.n, dtype=torch.float64, device=dev)
    F = torch.empty((w.n, 3), dtype=torch.float64, device=dev)
    ep = torch.empty(chunk + 1, dtype=torch.float64, device=dev)
    ek = torch.empty(chunk + 1, dtype=torch.float64, device=dev)
    out = Result(torch.empty(1, dtype=torch.float64, device=dev), torch.empty((w.n, 3), dtype=torch.float64, device=dev))
    ms_ev, _ = time_graph(lambda: plan.evaluate_md(x, c6, c12, out=out), steps, warmup, blocks, dev)
    ms, block_ms = time_graph(lambda: plan.md_run(x, v, c6, c12, im, dt, chunk, forces=F, epot=ep, ekin=ek),
                              max(blocks, steps // chunk), max(1, warmup // chunk), blocks, dev)
    torch.cuda.synchronize()
    flags = plan.status()
    tot = (ep + ek).cpu().numpy()
    # multiple time stepping: the grid part every k_slow = 4 steps
    k_slow, chunk_m = 4, 48
    epm = torch.empty(chunk_m // k_slow + 1, dtype=torch.float64, device=dev)
    ekm = torch.empty(chunk_m // k_slow + 1, dtype=torch.float64, device=dev)
    ms_m, block_m = time_graph(lambda: plan.md_run_mts(x, v, c6, c12, im, dt, chunk_m, k_slow, forces=F, epot=epm,
                                                       ekin=ekm),
                               max(blocks, steps // chunk_m), max(1, warmup // chunk_m), blocks, dev)
    torch.cuda.synchronize()
    flags |= plan.status()
    totm = (epm + ekm).cpu().numpy()
    # multiple time stepping per level: level 1 every 2 steps, levels 2..l
    # every 4 steps
    k_mid, k_sl = 2, 2
    epl = torch.empty(chunk_m // (k_mid * k_sl) + 1, dtype=torch.float64, device=dev)
    ekl = torch.empty(chunk_m // (k_mid * k_sl) + 1, dtype=torch.float64, device=dev)
    ms_l, block_l = time_graph(lambda: plan.md_run_mts_levels(x, v, c6, c12, im, dt, chunk_m, k_mid, k_sl, forces=F,
                                                              epot=epl, ekin=ekl),
                               max(blocks, steps // chunk_m), max(1, warmup // chunk_m), blocks, dev)
    torch.cuda.synchronize()
    flags |= plan.status()
    totl = (epl + ekl).cpu().numpy()
    plan.close()
    # neighbour reuse: velocity Verlet with plans that keep one binning while
    # no atom has moved more than skin/2 (0.07 keeps the 70 half-cells per
    # side of the 10^6-atom cube, 0.3 widens them), same trajectory start
    reuse = {}
    for skin in (0.07, 0.3):
        rp = Plan(w.box, prm["a"], prm["h"], prm["order"], prm["levels"], precision=precision, n_max=w.n,
                  device=dev.index, skin=skin)
        xr_ = torch.tensor(w.pos, dtype=torch.float64, device=dev)
        vr_ = torch.tensor(rng.normal(scale=np.sqrt(0.8), size=(w.n, 3)), dtype=torch.float64, device=dev)
        ms_r, block_r = time_graph(lambda: rp.md_run(xr_, vr_, c6, c12, im, dt, chunk, forces=F, epot=ep, ekin=ek),
                                   max(blocks, steps // chunk), max(1, warmup // chunk), blocks, dev)
        torch.cuda.synchronize()
        flags |= rp.status()
        reuse[str(skin)] = {"ms_per_step": ms_r / chunk, "steps_per_s": 1000.0 * chunk / ms_r,
                            "cells": list(rp.info["cells"]), "block_ms_per_step": [b / chunk for b in block_r]}
        rp.close()
    return {"workload": f"{w.name} positions, LJ C6 = C12 = 4, unit masses, velocities N(0, 0.8) (seed 29), "
                        f"repulsion cutoff {prm['a']}, dt {dt}",
            "precision": precision, "ms_per_step": ms / chunk, "steps_per_s": 1000.0 * chunk / ms,
            "block_ms_per_step": [b / chunk for b in block_ms], "steps_per_replay": chunk,
            "evaluate_md_ms": ms_ev, "flags": flags,
            "last_replay_total_energy_spread_rel": float((tot.max() - tot.min()) / abs(tot.mean())),
            "multiple_time_stepping": {
                "k_slow": k_slow, "ms_per_step": ms_m / chunk_m, "steps_per_s": 1000.0 * chunk_m / ms_m,
                "block_ms_per_step": [b / chunk_m for b in block_m], "steps_per_replay": chunk_m,
                "last_replay_total_energy_spread_rel": float((totm.max() - totm.min()) / abs(totm.mean()))},
            "neighbour_reuse": {"note": "mls_md_run with a skin: binning kept while no atom moved more than "
                                        "skin/2, checked every step", "by_skin": reuse,
                                "without_skin_ms_per_step": ms / chunk},
            "multiple_time_stepping_per_level": {
                "k_mid": k_mid, "k_slow": k_sl, "ms_per_step": ms_l / chunk_m, "steps_per_s": 1000.0 * chunk_m / ms_l,
                "block_ms_per_step": [b / chunk_m for b in block_l], "steps_per_replay": chunk_m,
                "last_replay_total_energy_spread_rel": float((totl.max() - totl.min()) / abs(totl.mean()))}}


def run_selection(w, head, steps, dev, target=1e-4):
    """Accuracy-targeted (a, h) (Sec. III.E) for this workload at the headline
    precision, then the evaluation rate at the chosen parameters."""
    import torch
    from paper_1308_4005_amd.params import select_parameters
    pos = torch.tensor(w.pos, dtype=torch.float64, device=dev)
    c6 = torch.tensor(w.c6, dtype=torch.float64, device=dev)
    t = time.time()
    s = select_parameters(pos, c6, w.box, target, precision=head, device=dev.index)
    wall = time.time() - t
    prm = dict(a=s.a, h=s.h, order=4, levels=0)
    r = time_precision(w, prm, head, max(50, steps // 5), 5, dev, stages=False, blocks=5)
    out = {"target_rms_rel_F": target, "a": s.a, "h": s.h, "levels": s.levels, "measured_rms_rel_F": s.error,
           "C_local_s": s.C_local, "C_grids_s": s.C_grids, "C_accuracy": s.C, "iterations": len(s.history),
           "selection_wall_s": wall, "ms_per_step": r["ms"], "evals_per_s": 1000.0 / r["ms"],
           "reference": f"error against an evaluation with a cutoff 1.7x larger (same h), {head}"}
    # the same selection on the 32,000-atom cube whose exact periodic forces
    # (Ewald, 512 sampled atoms) are stored: the error of eq:accuracy-tolerance
    import numpy as np
    from paper_1308_4005_amd import Plan
    from paper_1308_4005_amd import workloads as W
    path = os.path.join(ROOT, "tests", "golden", "cube32k_exact.json")
    if os.path.exists(path):
        gold = json.load(open(path))
        w32 = W.cube(gold["n"], gold["density"], seed=gold["seed"])
        p32 = torch.tensor(w32.pos, dtype=torch.float64, device=dev)
        c32 = torch.tensor(w32.c6, dtype=torch.float64, device=dev)
        s32 = select_parameters(p32, c32, w32.box, target, precision=head, device=dev.index)
        plan = Plan(w32.box, s32.a, s32.h, 4, 0, precision=head, n_max=w32.n, device=dev.index)
        F = plan.evaluate(p32, c32).forces.cpu().numpy()[np.asarray(gold["sample"])]
        plan.close()
        Fx = np.asarray(gold["forces"])
        out["exact_check_cube32k"] = {
            "a": s32.a, "h": s32.h, "levels": s32.levels, "proxy_rms_rel_F": s32.error,
            "exact_rms_rel_F": float(np.sqrt(np.sum((F - Fx) ** 2) / np.sum(Fx ** 2))),
            "reference": "exact periodic sum by Ewald at 512 sampled atoms (tests/golden/cube32k_exact.json)"}
    return out


def golden_errors(E, F, gold):
    import numpy as np
    if gold is None:
        return None
    idx = np.asarray(gold["sample"])
    Fr = np.asarray(gold["forces"])
    Fs = F[idx]
    diff = np.linalg.norm(Fs - Fr, axis=1)
    nref = np.linalg.norm(Fr, axis=1)
    return dict(dE=abs(E - gold["energy"]) / abs(gold["energy"]),
                rms_rel_F=float(np.sqrt(np.sum(diff ** 2) / np.sum(nref ** 2))),
                paper_dF=float(np.mean(diff / nref)),
                max_F=float(np.max(diff) / gold["force_rms"]),
                sampled_atoms=int(len(idx)))


def discretisation(prm, precisions, dev):
    """Error of the library's output against the exact periodic sum (Ewald,
    stored for 512 atoms of the 32,000-atom cube at density 0.8) with the
    headline a, h and order; the error does not depend on the system size."""
    import numpy as np
    import torch
    from paper_1308_4005_amd import Plan
    from paper_1308_4005_amd import workloads as W
    path = os.path.join(ROOT, "tests", "golden", "cube32k_exact.json")
    if not os.path.exists(path):
        return None
    gold = json.load(open(path))
    w = W.cube(gold["n"], gold["density"], seed=gold["seed"])
    pos = torch.tensor(w.pos, dtype=torch.float64, device=dev)
    c6 = torch.tensor(w.c6, dtype=torch.float64, device=dev)
    idx = np.asarray(gold["sample"])
    Fx = np.asarray(gold["forces"])
    nref = np.linalg.norm(Fx, axis=1)
    out = {"workload": f"cube32k: {w.n} atoms, L={w.box[0]:.4f}, density {gold['density']}, seed {gold['seed']}",
           "reference": "exact periodic sum by Ewald at 512 sampled atoms"}
    for p in precisions:
        plan = Plan(w.box, prm["a"], prm["h"], prm["order"], 0, precision=p, n_max=w.n, device=dev.index)
        r = plan.evaluate(pos, c6)
        torch.cuda.synchronize()
        diff = np.linalg.norm(r.forces.cpu().numpy()[idx] - Fx, axis=1)
        out[p] = {"rms_rel_F": float(np.sqrt(np.sum(diff ** 2) / np.sum(nref ** 2))),
                  "paper_dF": float(np.mean(diff / nref)), "max_F": float(np.max(diff) / np.sqrt(np.mean(nref ** 2))),
                  "levels": plan.info["levels"], "h_eff": list(plan.info["h_eff"])}
        plan.close()
    return out


def cpu_baseline(prm, target):
    """The FP64 oracle, timed on a bounded sample of the headline workload:
    evaluations (median of 3) of a 125,000-atom cube (one eighth of the atoms) with the same
    density, a, effective spacing and order, and a hierarchy one level
    shorter that ends in the same coarsest grid (56^3 -> 7^3 in four levels
    against 112^3 -> 7^3 in five).  Every stage of the method is linear in
    N except the coarsest all-to-all, whose size is the same in both, so the
    rate is extrapolated by the atom ratio."""
    from threadpoolctl import threadpool_limits
    from oracle import mls as oracle_mls
    from paper_1308_4005_amd import workloads as W
    n_s = target.n // 8
    w = W.cube(n_s, 0.8, seed=33)
    levels = max(1, prm["levels"] - 1)
    times = []
    with threadpool_limits(limits=1):
        for _ in range(3):
            t0 = time.perf_counter()
            r = oracle_mls.mls(w.pos, w.c6, w.box, prm["a"], prm["h"], prm["order"], levels)
            times.append(time.perf_counter() - t0)
    dt = sorted(times)[1]
    avail = len(os.sched_getaffinity(0))
    return {"value": (1.0 / dt) * (w.n / target.n), "unit": "evals/s (1M-atom equivalent)",
            "cores": 1, "cores_available": avail, "kind": "oracle", "extrapolated": True,
            "sample": f"EXTRAPOLATED: oracle.mls FP64 evaluations of a {w.n}-atom cube (rho 0.8, L="
                      f"{w.box[0]:.3f}, a={prm['a']}, h={prm['h']} -> grid {list(map(int, r['n1']))}, "
                      f"p={prm['order']}, {levels} levels, coarsest "
                      f"{[int(x) >> (levels - 1) for x in r['n1']]}): median of 3 runs {dt:.1f} s; scaled by {w.n}/{target.n} "
                      f"atoms to the {target.n}-atom headline; numpy single thread (BLAS limited to 1, no "
                      f"process pool) of {avail} cores available"}


SWEEP_A = (2.5, 3.0, 4.0)
SWEEP_H = (0.8, 1.0, 1.25)
SWEEP_P = (4, 6)


def _tag(x):
    return f"{x:g}".replace(".", "p")


def precision_sweep(w, dev, steps, blocks):
    """The precision-at-scale sweep on the 10^6-atom cube: a in {2.5, 3, 4},
    h in {0.8, 1, 1.25}, p in {4, 6}, five levels.  Per setting and precision:
    ms per evaluation (graph replays), and the energy and force errors against
    the FP64 oracle at the stored sample of 512 atoms (tests/golden/
    cube1M_a*_h*_p*_l5.json, written by the oracle alone) and of the mixed
    path against the FP64 path on all atoms."""
    import numpy as np
    out = []
    for a in SWEEP_A:
        for h in SWEEP_H:
            for p in SWEEP_P:
                prm = dict(a=a, h=h, order=p, levels=5)
                gpath = os.path.join(ROOT, "tests", "golden", f"cube1M_a{_tag(a)}_h{_tag(h)}_p{p}_l5.json")
                gold = json.load(open(gpath)) if os.path.exists(gpath) else None
                row = {"a": a, "h": h, "order": p}
                F = {}
                for prec in ("fp64", "mixed"):
                    r = time_precision(w, prm, prec, steps, 3, dev, stages=False, blocks=blocks)
                    F[prec] = (r["E"], r["F"])
                    row[prec] = {"ms_per_step": r["ms"], "evals_per_s": 1000.0 / r["ms"],
                                 "vs_oracle": golden_errors(r["E"], r["F"], gold)}
                    row["grid"] = list(r["info"]["grid"])
                    row["taps"] = r["info"]["taps"]
                    row[prec]["stencil_path"] = r["info"]["stencil_path"]
                (Ed, Fd), (Em, Fm) = F["fp64"], F["mixed"]
                dif = np.linalg.norm(Fm - Fd, axis=1)
                row["mixed_vs_fp64_gpu"] = {"dE": abs(Em - Ed) / abs(Ed),
                                            "rms_rel_F": float(np.sqrt(np.sum(dif ** 2) / np.sum(Fd ** 2)))}
                row["mixed_over_fp64"] = row["fp64"]["ms_per_step"] / row["mixed"]["ms_per_step"]
                log(f"[bench] sweep a={a} h={h} p={p}: fp64 {row['fp64']['ms_per_step']:.3f} ms, mixed "
                    f"{row['mixed']['ms_per_step']:.3f} ms, mixed-vs-fp64 rms F {row['mixed_vs_fp64_gpu']['rms_rel_F']:.1e}"
                    f", oracle sample {'yes' if gold else 'missing'}")
                out.append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="timed graph replays (split into --blocks blocks)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--blocks", type=int, default=5, help="timed blocks; the median block is reported")
    ap.add_argument("--workload", default="cube1M")
    ap.add_argument("--a", type=float, default=3.0)
    ap.add_argument("--h", type=float, default=1.0)
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--levels", type=int, default=5)
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "mixed"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="leave out the batched-form measurement")
    ap.add_argument("--no-family", action="store_true", help="leave out the smoothing-family measurement")
    ap.add_argument("--no-lb", action="store_true", help="leave out the Lorentz-Berthelot measurement")
    ap.add_argument("--no-select", action="store_true", help="leave out the parameter-selection measurement")
    ap.add_argument("--no-md", action="store_true", help="leave out the molecular-dynamics measurement")
    ap.add_argument("--no-sweep", action="store_true", help="leave out the 18-setting precision sweep")
    ap.add_argument("--sweep-steps", type=int, default=100, help="graph replays per sweep setting")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: MLS here is a single-GPU path "
              "(the multi-GPU decomposition is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1308_4005_amd import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t = time.time()
    w = W.named(args.workload)
    log(f"[bench] workload {w.name}: n={w.n} box={w.box.round(4).tolist()} ({time.time() - t:.1f}s)")
    prm = dict(a=args.a, h=args.h, order=args.order, levels=args.levels)
    gname = f"{args.workload}_a{args.a:g}_h{args.h:g}_p{args.order}_l{args.levels}"
    gpath = os.path.join(ROOT, "tests", "golden", gname + ".json")
    gold = json.load(open(gpath)) if os.path.exists(gpath) else None

    precisions = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    res = {}
    for p in precisions:
        log(f"[bench] timing {p}: warmup {args.warmup}, steps {args.steps} in {args.blocks} blocks")
        res[p] = time_precision(w, prm, p, args.steps, args.warmup, dev, blocks=args.blocks)
        log(f"[bench] {p}: {res[p]['ms']:.3f} ms/eval (graph, median block), eager {res[p]['eager_ms']:.3f} stages {json.dumps({k: round(v, 4) for k, v in res[p]['stage_ms'].items()})}")

    head = "mixed" if "mixed" in res else precisions[0]
    info = res[head]["info"]
    pairs = count_pairs(w.pos, w.box, args.a) if min(w.box) > 2 * args.a else None
    model = work_model(info, w.n, pairs or 0, args.order)
    # dominant kernel of the headline precision
    sm = res[head]["stage_ms"]
    dom = max(sm, key=sm.get)
    m = model[dom]
    dt_s = sm[dom] * 1e-3
    if m["bound"] == "hbm":
        achieved = m["bytes"] / dt_s / 1e9
        peak = PEAK["hbm"]
        unit = "GB/s"
    else:
        achieved = m["flops"] / dt_s / 1e12
        peak = PEAK["fp32" if head == "mixed" else "fp64"]
        unit = "TFLOP/s"
    roofline = {"bound": m["bound"], "kernel": dom, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": measured_traffic(dom, head), "traffic_unit": "bytes",
                "work_per_launch": m.get("flops", m.get("bytes")),
                "avg_launch_ms": sm[dom]}
    if m["bound"] != "hbm" and head == "mixed":
        roofline["peak_unpacked_fp32"] = PEAK["fp64"]
        roofline["frac_unpacked_fp32"] = achieved / PEAK["fp64"]
    per_stage_roofline = {p: stage_rooflines(res[p]["stage_ms"], model, p) for p in res}
    # the level stencil of the mixed plan two ways: the VALU tile (the
    # default) and its MFMA recast
    stencil_variants = None
    if "mixed" in res:
        mf = time_stencil_mfma(w, prm, dev, min(args.steps, 100))
        vt = res["mixed"]["stage_ms"].get("stencil")
        stencil_variants = {"tile_f32_valu_ms": vt, "tile_mfma_f32_ms": mf,
                            "flops_per_launch": model["stencil"]["flops"]}
        log(f"[bench] stencil stage: VALU tile {vt} ms, MFMA tile {mf} ms")

    accuracy = {}
    for p in res:
        accuracy[p] = golden_errors(res[p]["E"], res[p]["F"], gold)
    if "mixed" in res and "fp64" in res:
        Fd, Fm = res["fp64"]["F"], res["mixed"]["F"]
        dif = np.linalg.norm(Fm - Fd, axis=1)
        accuracy["mixed_vs_fp64_gpu"] = dict(
            dE=abs(res["mixed"]["E"] - res["fp64"]["E"]) / abs(res["fp64"]["E"]),
            rms_rel_F=float(np.sqrt(np.sum(dif ** 2) / np.sum(Fd ** 2))))

    log("[bench] discretisation error against the exact sum (32,000-atom cube)")
    disc = discretisation(prm, precisions, dev)

    # the smoothing-function family (continuity C^1..C^4, Sec. III.B) at the
    # headline precision; k = 2 is the headline itself
    family = None
    if not args.no_family:
        family = {"precision": head, "ms_per_step": {}, "energy": {}}
        for k in (1, 2, 3, 4):
            if k == 2:
                r = res[head]
            else:
                log(f"[bench] continuity C^{k}")
                r = time_precision(w, prm, head, max(50, args.steps // 5), 5, dev, continuity=k, stages=False,
                                   blocks=args.blocks)
            family["ms_per_step"][f"C{k}"] = r["ms"]
            family["energy"][f"C{k}"] = r["E"]

    batch_ws = []

    def batch_workload():
        # the 256-box workload, built once (the batched and the batched
        # Lorentz-Berthelot timings share it)
        if not batch_ws:
            batch_ws.extend(W.named_batch("batch256"))
        return batch_ws

    lb = None
    if not args.no_lb:
        log("[bench] Lorentz-Berthelot mixing")
        lb = {p: time_lb(w, prm, max(5, args.steps // 20), 2, dev, precision=p) for p in ("fp64", "mixed")}
        log(f"[bench] Lorentz-Berthelot: FP64 {lb['fp64']['ms_per_step']:.3f}, mixed "
            f"{lb['mixed']['ms_per_step']:.3f} ms/eval")
        if not args.no_batch:
            bws = batch_workload()
            lb["batched"] = {p: time_batched_lb(bws, p, max(5, args.steps // 20), 2, dev) for p in ("fp64", "mixed")}
            log(f"[bench] batched Lorentz-Berthelot ({len(bws)} boxes): FP64 "
                f"{lb['batched']['fp64']['ms_per_step']:.3f}, mixed {lb['batched']['mixed']['ms_per_step']:.3f} ms")

    md = None
    if not args.no_md:
        log("[bench] molecular dynamics (velocity Verlet, dispersion + repulsion)")
        md = time_md(w, prm, head, args.steps, args.warmup, dev, args.blocks)
        log(f"[bench] md: {md['ms_per_step']:.3f} ms/step, evaluate_md {md['evaluate_md_ms']:.3f} ms, "
            f"multiple time stepping (k=4) {md['multiple_time_stepping']['ms_per_step']:.3f} ms/step, per level "
            f"(2, 2) {md['multiple_time_stepping_per_level']['ms_per_step']:.3f} ms/step, neighbour reuse "
            f"{json.dumps({k: round(v['ms_per_step'], 4) for k, v in md['neighbour_reuse']['by_skin'].items()})}")

    selection = None
    if not args.no_select:
        log("[bench] parameter selection for RMS-relative force error 1e-4")
        selection = run_selection(w, head, args.steps, dev)
        log(f"[bench] selected a={selection['a']:.3f} h={selection['h']:.3f}: error "
            f"{selection['measured_rms_rel_F']:.2e}, {selection['ms_per_step']:.3f} ms/eval")

    batched = None
    if not args.no_batch:
        t = time.time()
        ws = batch_workload()
        log(f"[bench] batch256: {len(ws)} boxes, {sum(w.n for w in ws)} atoms ({time.time() - t:.1f}s)")
        batched = {"workload": "batch256: 256 periodic boxes, N ~ floor(exp U(ln 500, ln 20000)), box (L, L, aL) "
                               "with a ~ U(1,4), density ~ U(0.02,0.85), RSA min distance 0.8, C6=4; "
                               "a=3, h=1, p=4, levels by box size",
                   "boxes": len(ws), "atoms": int(sum(w.n for w in ws))}
        for p in precisions:
            log(f"[bench] batched {p}")
            batched[p] = time_batched(ws, p, args.steps, args.warmup, dev)
            log(f"[bench] batched {p}: {batched[p]['ms_per_step']:.3f} ms/step, sequential single plans "
                f"{batched[p]['sequential_single_plans_ms']:.3f} ms")

    sweep = None
    if not args.no_sweep and args.workload == "cube1M":
        log("[bench] precision-at-scale sweep (18 settings x 2 precisions)")
        sweep = precision_sweep(w, dev, args.sweep_steps, min(args.blocks, 5))

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle on a bounded sample)")
        cpu = cpu_baseline(prm, w)
        log(f"[bench] cpu baseline: {cpu['sample']}")

    ms = res[head]["ms"]
    line = {
        "metric": "MLS E+F evals/s at 1M atoms, FP32-mixed vs FP64, at stated RMS force error",
        "value": 1000.0 / ms,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-mixed" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n} LJ atoms, periodic cube L={w.box[0]:.4f}, density 0.8, "
                               f"RSA min distance 0.8, C6=4",
                   "a": args.a, "h": args.h, "h_eff": list(info["h_eff"]), "grid": list(info["grid"]),
                   "order": args.order, "levels": info["levels"], "taps": info["taps"],
                   "in_cutoff_pairs": pairs},
        "particle_evals_per_s": w.n * 1000.0 / ms,
        "timing": f"graph replays of one evaluation: {args.warmup} warm-up, then {args.steps} replays in "
                  f"{args.blocks} blocks timed with events; ms_per_step is the median block",
        "per_precision": {p: {"evals_per_s": 1000.0 / r["ms"], "ms_per_step": r["ms"], "block_ms": r["block_ms"],
                              "eager_ms_per_step": r["eager_ms"], "stage_ms": r["stage_ms"], "serial_ms_per_step": sum(r["stage_ms"].values()),
                              "energy": r["E"]} for p, r in res.items()},
        "mixed_over_fp64": (res["fp64"]["ms"] / res["mixed"]["ms"]) if len(res) == 2 else None,
        "accuracy": accuracy,
        "discretisation_error": disc,
        "roofline": roofline,
        "stage_roofline": per_stage_roofline,
        "stencil_variants": stencil_variants,
        "precision_sweep": sweep,
        "continuity_family": family,
        "lorentz_berthelot": lb,
        "molecular_dynamics": md,
        "parameter_selection": selection,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
