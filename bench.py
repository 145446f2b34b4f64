#!/usr/bin/env python
"""Benchmark of the QV-tree search hot path on one MI355X.

One step = one call of qv_plan_step: a full planning step (map signature,
then for each of the D levels the prediction/likelihood statistics, the
observation draws, and the child beliefs or the fused leaf scores, then the
expectimax backup) on the 64 x 64 workload: seeded random rectangles (20%
blocked), 8 actions with 8-neighbour slip, wall bits plus 32 landmarks,
depth 3, 4 samples per action, Gaussian start belief (sigma 5 cells), Q
from the library's own value iteration to a 1e-6 relative residual.  Inputs
are resident on the GPU before the timed region; the timed steps cycle over
a fixed set of draw seeds whose trees were counted during warm-up.

Prints one JSON line: belief-state updates/s (value), plans/s, V-node
expansions/s, the roofline of the dominant kernel (HIP events around its
launches inside the timed region), the per-kernel breakdown, the value
iteration, and the FP64 CPU oracle timed on a bounded sample of the same
workload.  Beside the headline: 256 uneven queries planned in one batched
call against the same queries planned one by one ("batch"), one evaluation
of the filter likelihood and its adjoint on 1024 logged runs ("filter"), and
planning on a 512 x 512 grid ("large").
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "belief-state updates/sec + plans/sec (1 GPU), % of HBM roofline"
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_rect64.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--seeds", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--banded", action="store_true",
                    help="force the banded multi-pass kernels (QV_PLAN_TILED)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (PMC byte-count calibration)")
    ap.add_argument("--only-headline", action="store_true",
                    help="skip the batch, filter and large-grid measurements")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--filter-steps", type=int, default=5)
    ap.add_argument("--large-steps", type=int, default=10)
    return ap.parse_args()


def gpu_q(B, torch, prob, dev):
    """Q-MDP table from the library's value iteration (tol 1e-6 relative)."""
    m = B.DeviceModel(prob, dev)
    Q = torch.empty(m.S * m.A, dtype=torch.float32, device=dev)
    ws = torch.empty(B.qv_vi_workspace_bytes(m, 10000), dtype=torch.uint8, device=dev)
    st, _, sweeps = B.qv_value_iterate(m, 1e-6, 10000, Q, ws)
    B.check(st, "qv_value_iterate")
    return Q, sweeps


def level_counts(tree, D):
    lf = tree["level_first"]
    return [int(tree["valid"][lf[d]:lf[d + 1]].sum()) for d in range(D + 1)]


def bench_batch(args, B, wl, torch, dev):
    """256 independent queries (sides 32..256, 10-30% blocked, N/E/S/W,
    wall bits, depth 2-3, 3 samples): one batched call (persistent launches,
    HIP graph per level, autotuned shape) against the same 256 queries
    planned one qv_plan_step call after another."""
    from paper_1810_00204_amd.planner import BatchPlanner, Planner
    probs = wl.make_batch(seed=0)
    Qs = [gpu_q(B, torch, p, dev)[0] for p in probs]
    seed = 1810
    bp = BatchPlanner(probs, Qs, device=dev, n=3, flags=B.QV_BATCH_GRAPH)
    tune_ms = bp.autotune(seed, reps=2)
    tc, ch = bp.shape()
    bp.plan(seed)
    counts = [level_counts(bp.tree(q), p.D) for q, p in enumerate(probs)]
    upd = sum(sum(c[1:]) * p.S for c, p in zip(counts, probs))
    for _ in range(2):
        bp.plan(seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batch_steps):
        bp.plan(seed)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / args.batch_steps
    # the plain per-query form: each query on its own (auto kernel choice)
    pls = [Planner(p, device=dev) for p in probs]
    for q, pl in enumerate(pls):
        pl.plan(Qs[q], seed=seed, query_id=q)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        for q, pl in enumerate(pls):
            pl.plan(Qs[q], seed=seed, query_id=q)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / reps
    nq = len(probs)
    return {"workload": "256 queries, sides U{32..256}, 10-30% blocked, 4 actions, wall bits, "
                        "D U{2,3}, n 3",
            "queries": nq, "mean_cells": sum(p.S for p in probs) / nq,
            "depth3_queries": sum(1 for p in probs if p.D == 3),
            "ms_per_batch": t_batch * 1e3, "plans_per_s": nq / t_batch,
            "belief_updates_per_s": upd / t_batch,
            "sequential_ms_per_batch": t_seq * 1e3, "sequential_plans_per_s": nq / t_seq,
            "speedup_vs_sequential": t_seq / t_batch,
            "shape": {"tile_cells": tc, "chunk": ch, "autotune_ms_per_batch": tune_ms},
            "graph": True}


def bench_filter(args, B, wl, torch, dev):
    """One evaluation = NLL and adjoint gradient of 1024 logged runs of 50
    steps on 128 x 128 (8 actions, 9 slip outcomes), checkpoints every 10."""
    from paper_1810_00204_amd.filter import FilterProblem
    ts = wl.make_trajectories(seed=0)
    fp = FilterProblem(ts.problem, ts.acts, ts.obs, device=dev, ckpt_every=10)
    th = torch.as_tensor(ts.theta)
    ph = torch.as_tensor(ts.phi)
    fp.run(th, ph)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.filter_steps):
        fp.run(th, ph, check=False)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.filter_steps
    ntraj, T = ts.acts.shape
    S = ts.problem.W * ts.problem.H
    return {"workload": f"{ntraj} runs x {T} steps, {ts.problem.W}x{ts.problem.H}, 8 actions, "
                        "checkpoint every 10",
            "ms_per_eval": dt * 1e3, "evals_per_s": 1.0 / dt,
            "filter_updates_per_s": ntraj * T * S / dt,
            "note": "one evaluation = forward filter, segment recomputation and adjoint"}


def bench_large(args, B, wl, torch, dev):
    """512 x 512 rectangles and corridors (25% blocked), 8 actions, 256
    landmarks, depth 3, 3 samples, 4-patch start belief."""
    from paper_1810_00204_amd.planner import Planner
    prob = wl.make_large(seed=0)
    pl = Planner(prob, device=dev)
    t0 = time.perf_counter()
    Q, res, sweeps = pl.value_iterate(tol=1e-6, max_sweeps=10000)
    torch.cuda.synchronize()
    vi_ms = (time.perf_counter() - t0) * 1e3
    pl.plan(Q)
    counts = level_counts(pl.tree(beliefs=False), prob.D)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.large_steps):
        pl.plan(Q)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.large_steps
    upd = sum(counts[1:]) * prob.S
    return {"workload": prob.name, "ms_per_plan": dt * 1e3, "plans_per_s": 1.0 / dt,
            "belief_updates_per_s": upd / dt, "nodes_per_level": counts,
            "value_iteration": {"sweeps": sweeps, "residual": res, "ms": vi_ms}}


def source_hash():
    from paper_1810_00204_amd.build import source_hash as h
    return h()


def kernel_work(name, prob, counts):
    """Algorithmic FP32 flops, HBM bytes and the bounding resource of one
    launch of a per-level planning kernel ("<kernel>@L<d>"), from the numbers
    of valid nodes per level.  None for others."""
    if "@L" not in name:
        return None
    base, lvl = name.rsplit("@L", 1)
    d = int(lvl)
    S, A, D = prob.S, prob.A, prob.D
    P, C = counts[d], counts[d + 1]
    leaf = d == D - 1
    stencil = P * A * S * 18.0          # 9 FMA per (parent, action, cell)
    stats = P * A * S * 3.0             # bin add, R(b,a) FMA
    child = C * S * 6.0                 # O product, normalisation
    score = C * S * 2.0 * A             # A FMAs against Q per leaf cell
    # leaf scores from the nine basis histograms (k_leaf_parent): per
    # (parent, cell) the eight inflow sums s_k (8), lambda s_k (9), 9 (AM+1)
    # accumulations with Q (2 flops each) and R(b,a) (2 A); per parent the
    # transform HQ_a = sum_k T'(a,k) E_k (A 16 (AM+1) 9 FMAs); per leaf child
    # 16 A FMAs
    AM = 4 if A <= 4 else 8
    basis = (P * S * (8.0 + 9.0 + 18.0 * (AM + 1) + 2.0 * A)
             + P * A * 16.0 * (AM + 1) * 18.0 + C * 32.0 * A)
    if "k_leaf_parent" in base:
        return basis, P * S * 4.0, "alu"
    if "k_node" in base:
        if leaf:
            return stencil + stats + child + score, P * S * 4.0, "alu"
        return stencil + stats + child, P * S * 4.0 + C * S * 4.0, "hbm"
    if "k_stats" in base:
        return stencil + stats, P * S * 4.0, "alu"
    if "k_update" in base:
        return stencil + child, P * S * 4.0 + C * S * 4.0, "hbm"
    if "k_leaf" in base:
        return stencil + child + score, P * S * 4.0, "alu"
    return None


def cpu_baseline(prob, Q32, seeds):
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    upd = 0
    for s in seeds:
        res = oracle.plan(prob, Q32, seed=s)
        d = res["dump"]
        upd += sum(int(d.level(d.valid, k).sum()) for k in range(1, prob.D + 1)) * prob.S
    dt = time.perf_counter() - t0
    return {"value": upd / dt, "unit": "belief-state updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{len(seeds)} full planning steps (draw seeds {seeds[0]}..{seeds[-1]}) of "
                      f"the same workload by the single-threaded FP64 oracle, {dt:.1f} s",
            "plans_per_s": len(seeds) / dt, "seconds": dt}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the planning path runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1810_00204_amd import binding as B
    from paper_1810_00204_amd import workloads as wl
    from paper_1810_00204_amd.planner import Planner

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    B.lib()
    dev = "cuda:0"
    prob = wl.make_rect(seed=0)
    pl = Planner(prob, device=dev, flags=B.QV_PLAN_TILED if args.banded else 0)

    # offline Q-MDP values (timed on its own)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Q, res, sweeps = pl.value_iterate(tol=1e-6, max_sweeps=10000)
    torch.cuda.synchronize()
    vi_ms = (time.perf_counter() - t0) * 1e3

    seeds = [prob.seed + i for i in range(args.seeds)]
    counts = {}
    for i in range(max(args.warmup, len(seeds))):
        s = seeds[i % len(seeds)]
        pl.plan(Q, seed=s)
        if s not in counts:
            t = pl.tree(beliefs=False)
            lf = t["level_first"]
            counts[s] = [int(t["valid"][lf[d]:lf[d + 1]].sum()) for d in range(prob.D + 1)]
    torch.cuda.synchronize()

    K = args.steps
    step_seeds = [seeds[k % len(seeds)] for k in range(K)]
    # timed region: K planning steps, nothing else on the stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in step_seeds:
        pl.plan(Q, seed=s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the same K steps again with HIP events bracketing every kernel launch
    # on the launch stream: per-kernel durations for the roofline
    B.qv_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in step_seeds:
        pl.plan(Q, seed=s)
    torch.cuda.synchronize()
    wall_ev = time.perf_counter() - t0
    st, ktimes = B.qv_timing_read()
    B.qv_timing_enable(False)
    B.check(st, "qv_timing_read")

    # work done in the timed region
    upd = sum(sum(counts[s][1:]) for s in step_seeds) * prob.S
    # the stricter count: posteriors written out (levels 1..D-1); leaf
    # posteriors are scored through wall-reading histograms, not formed cell by cell
    upd_stored = sum(sum(counts[s][1:prob.D]) for s in step_seeds) * prob.S
    exp = sum(sum(counts[s][:-1]) for s in step_seeds)
    kids = sum(sum(counts[s][1:]) for s in step_seeds)

    # per-kernel algorithmic work and measured time
    kern = {}
    tot_ms = sum(v[1] for v in ktimes.values())
    for name, (launches, ms) in ktimes.items():
        e = {"launches": launches, "avg_us": 1e3 * ms / launches,
             "share": ms / tot_ms if tot_ms else None}
        work = [kernel_work(name, prob, counts[s]) for s in step_seeds]
        if work[0] is not None:
            fl = sum(w[0] for w in work)
            by = sum(w[1] for w in work)
            e.update({"bound": work[0][2], "alg_gflop_per_launch": fl / len(work) / 1e9,
                      "alg_mb_per_launch": by / len(work) / 1e6,
                      "tflops": fl / (ms * 1e-3) / 1e12, "gbs": by / (ms * 1e-3) / 1e9})
        kern[name] = e
    dom = max(ktimes, key=lambda k: ktimes[k][1])
    roof = {"kernel": dom}
    if kern[dom].get("bound") == "alu":
        roof.update({"bound": "alu", "achieved": kern[dom]["tflops"], "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s"})
    else:
        roof.update({"bound": "hbm", "achieved": kern[dom].get("gbs", 0.0), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s"})
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("source_hash") == source_hash() and dom in tr.get("kernels", {}):
            roof["traffic"] = tr["kernels"][dom]["bytes_per_launch"]
    hbm_k = [k for k, v in kern.items() if v.get("bound") == "hbm"]
    hbm_frac = {k: kern[k]["gbs"] / PEAK_HBM_GBS for k in hbm_k}

    if args.copy_calibration:
        a = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()

    line = {
        "metric": METRIC, "value": upd / wall, "unit": "belief-state updates/s",
        "n_gpus": 1, "steps": K, "warmup": args.warmup, "ms_per_step": wall * 1e3 / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": prob.name, "grid": f"{prob.W}x{prob.H}", "actions": prob.A,
                   "landmarks": prob.L, "depth": prob.D, "samples_per_action": prob.n,
                   "blocked_fraction": round(float(prob.occ.mean()), 4),
                   "draw_seeds": len(seeds), "parallelism": "single GPU",
                   "kernels": "banded" if args.banded else "auto",
                   "source_hash": source_hash()},
        "ms_per_step_with_kernel_events": wall_ev * 1e3 / K,
        "plans_per_s": K / wall, "v_node_expansions_per_s": exp / wall,
        "stored_belief_updates_per_s": upd_stored / wall,
        "child_nodes_per_s": kids / wall,
        "hbm_frac_by_kernel": hbm_frac,
        "roofline": roof, "kernels": kern,
        "value_iteration": {"sweeps": sweeps, "residual": res, "ms": vi_ms,
                            "sweeps_per_s": sweeps / (vi_ms * 1e-3)},
    }
    if not args.only_headline:
        line["batch"] = bench_batch(args, B, wl, torch, dev)
        line["filter"] = bench_filter(args, B, wl, torch, dev)
        line["large"] = bench_large(args, B, wl, torch, dev)
    if not args.no_cpu_baseline:
        Q32 = Q.cpu().numpy().reshape(prob.S, prob.A)
        line["cpu_baseline"] = cpu_baseline(prob, Q32, seeds[:4])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
