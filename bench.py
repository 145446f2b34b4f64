#!/usr/bin/env python
"""Benchmark of the QV-tree search hot path on one MI355X.

One step = one call of qv_plan_step: a full planning step (map signature,
then for each of the D levels the prediction/likelihood statistics, the
observation draws, and the child beliefs or the fused leaf scores, then the
expectimax backup) on the 512 x 512 workload: seeded random rectangles
(sides 4..32) alternating with corridor walls (lengths 32..256) until 25% of
the cells are blocked, 8 actions with 8-neighbour slip, wall bits plus 256
landmarks, depth 3, 3 samples per action, start belief an equal mixture of
four disjoint 20 x 20 patches, Q from the library's own value iteration to a
1e-6 relative residual.  Inputs are resident on the GPU before the timed
region; the timed steps cycle over a fixed set of draw seeds whose trees
were counted during warm-up.

Prints one JSON line.  `value` is the rate of belief-state updates produced:
posterior cells Phi(b,a,z)(s) written out at levels 1..D-1 (all S cells of
every valid child, blocked ones included).  The last level scores its
children through wall-reading histograms without forming their posteriors;
the count that includes them is `evaluated_belief_updates_per_s`.  Beside it:
plans/s, V-node expansions/s, the per-kernel table (HIP events around every
launch, on the launch stream, over a second pass of the same steps), the
roofline of the dominant kernel, the value iteration, the FP64 CPU oracle
timed on a bounded sample of the same workload (one thread and all cores),
the 64 x 64 workload ("rect64"), 256 uneven queries in one batched call
("batch"), and one evaluation of the filter likelihood with its adjoint
("filter").
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "belief-state updates/sec + plans/sec (1 GPU), % of HBM roofline"
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PROFILES = os.path.join(ROOT, "profiles")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seeds", type=int, default=8)
    ap.add_argument("--workload", choices=["large512", "rect64"], default="large512",
                    help="the headline workload (default: the 512 x 512 grid)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-runs", type=int, default=5)
    ap.add_argument("--banded", action="store_true",
                    help="force the banded multi-pass kernels (QV_PLAN_TILED)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run plain device copies (PMC byte-count calibration)")
    ap.add_argument("--only-headline", action="store_true",
                    help="skip the side measurements (rect64, batch, filter)")
    ap.add_argument("--side-steps", type=int, default=200)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--filter-steps", type=int, default=5)
    ap.add_argument("--loop-runs", type=int, default=10)
    ap.add_argument("--loop-expansions", type=int, default=128)
    return ap.parse_args()


def make_problem(name):
    from paper_1810_00204_amd import workloads as wl
    return {"large512": lambda: wl.make_large(seed=0),
            "rect64": lambda: wl.make_rect(seed=0)}[name]()


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on a bounded sample of the headline workload
# ---------------------------------------------------------------------------

_PROBLEMS = {}


def _oracle_stored_levels(args):
    """The oracle's expansions of every V-node of levels 0..D-2 of one plan
    (draw seed `seed`): exactly the posteriors the GPU writes out.  Returns
    (belief-state updates produced, expansions, seconds)."""
    name, seed = args
    import oracle
    if name not in _PROBLEMS:
        _PROBLEMS[name] = make_problem(name)
    prob = _PROBLEMS[name]
    t0 = time.perf_counter()
    frontier = [(prob.b0.astype("float64"), 0)]
    upd = exp = 0
    for d in range(prob.D - 1):
        nxt = []
        for b, slot in frontier:
            e = oracle.expand_node(prob, b, d, slot, seed=seed, beliefs=True)
            exp += 1
            for c in range(prob.K):
                if e["valid"][c]:
                    upd += prob.S
                    nxt.append((e["beliefs"][c], slot * prob.K + c))
        frontier = nxt
    return upd, exp, time.perf_counter() - t0


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, seeds, runs):
    """Single-thread and all-core legs, median of `runs` runs each.  A run of
    the single-thread leg is one plan's stored levels; a run of the all-core
    leg is that for `cores` draw seeds at once, one process per seed.  Runs
    before the GPU is touched (the worker processes are forked)."""
    import multiprocessing as mp
    import oracle
    oracle.build(force=False)
    cores = min(len(os.sched_getaffinity(0)), 16)
    one = [_oracle_stored_levels((name, seeds[i % len(seeds)])) for i in range(runs)]
    r1 = statistics.median(u / t for u, _, t in one)
    ctx = mp.get_context("fork")
    allc = []
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_stored_levels, [(name, seeds[0])] * cores)   # warm the workers
        for i in range(runs):
            t0 = time.perf_counter()
            res = pool.map(_oracle_stored_levels,
                           [(name, seeds[(i + j) % len(seeds)]) for j in range(cores)])
            allc.append(sum(u for u, _, _ in res) / (time.perf_counter() - t0))
    rall = statistics.median(allc)
    upd1, exp1 = one[0][0], one[0][1]
    return {"value": rall, "unit": "belief-state updates/s", "cores": cores, "kind": "oracle",
            "sample": (f"the stored levels (0..D-2) of one plan: {exp1} V-node expansions "
                       f"producing {upd1} belief-state updates, by the FP64 oracle; single-thread "
                       f"leg = one plan per run, all-core leg = {cores} plans (one per process, "
                       f"distinct draw seeds) per run; median of {runs} runs each"),
            "single_thread": {"value": r1, "runs_s": [t for _, _, t in one]},
            "all_cores": {"value": rall, "runs_per_s": allc},
            "cpu_model": _cpu_model(), "affinity_cores": len(os.sched_getaffinity(0))}


# ---------------------------------------------------------------------------
# GPU measurements
# ---------------------------------------------------------------------------

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


def kernel_work(name, prob, counts):
    """Algorithmic work of one launch of a per-level planning kernel
    ("<kernel>@L<d>"): (FP32 flops, HBM bytes, bound), from the numbers of
    valid nodes per level.  The figures are the method's, not this build's
    algorithm's:
      * a belief-state update (one child posterior cell) costs 4 B written
        plus 8/K B of parent reads (the parent is read once for the
        statistics and once for the update, shared by K child slots): the
        statistics pass is charged 4/K B per update, the update pass 4 + 4/K;
      * the prediction is 9 FMA (18 flops) per (parent, action, cell);
      * a leaf child's score is 2 + 2|A| flops per cell (posterior cell and
        its dot products with Q).
    None for kernels outside the levels."""
    if "@L" not in name:
        return None
    base, lvl = name.rsplit("@L", 1)
    d = int(lvl)
    S, A, D, K = prob.S, prob.A, prob.D, prob.A * prob.n
    P, C = counts[d], counts[d + 1]
    leaf = d == D - 1
    stencil = P * A * S * 18.0
    upd_bytes = C * S * (4.0 + 8.0 / K)
    score = C * S * (2.0 + 2.0 * A)
    if "k_leaf_parent" in base or ("k_node" in base and leaf) or base.startswith("k_leaf<"):
        return stencil + score, P * S * 4.0, "alu"
    if "k_node" in base:
        return stencil + C * S * 2.0, upd_bytes, "hbm"
    if "k_stats" in base:
        return stencil, C * S * 4.0 / K, "hbm"
    if "k_update" in base:
        return stencil + C * S * 2.0, C * S * (4.0 + 4.0 / K), "hbm"
    return None


def traffic_of(workload, kernel, src_hash):
    """Counter-measured HBM bytes per launch of `kernel` from the committed
    rocprofv3 summary, if it was taken on these sources; else None."""
    path = os.path.join(PROFILES, f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    tr = json.load(open(path))
    if tr.get("source_hash") != src_hash:
        return None
    k = tr.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_launch"]


def plan_bench(B, torch, dev, prob, steps, warmup, nseeds, flags, workload_key, src_hash):
    """K timed planning steps of one workload; then the same K steps with
    kernel events for the per-kernel table and the roofline."""
    from paper_1810_00204_amd.planner import Planner
    pl = Planner(prob, device=dev, flags=flags)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Q, res, sweeps = pl.value_iterate(tol=1e-6, max_sweeps=10000)
    torch.cuda.synchronize()
    vi_ms = (time.perf_counter() - t0) * 1e3

    seeds = [prob.seed + i for i in range(nseeds)]
    counts = {}
    for i in range(max(warmup, len(seeds))):
        s = seeds[i % len(seeds)]
        pl.plan(Q, seed=s)
        if s not in counts:
            counts[s] = level_counts(pl.tree(beliefs=False), prob.D)
    torch.cuda.synchronize()

    step_seeds = [seeds[k % len(seeds)] for k in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in step_seeds:
        pl.plan(Q, seed=s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the same steps with HIP events bracketing every kernel launch on its stream
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

    D, S = prob.D, prob.S
    stored = sum(sum(counts[s][1:D]) for s in step_seeds) * S
    evaluated = sum(sum(counts[s][1:]) for s in step_seeds) * S
    exp = sum(sum(counts[s][:-1]) for s in step_seeds)
    kids = sum(sum(counts[s][1:]) for s in step_seeds)

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
            e["frac"] = (e["tflops"] / PEAK_FP32_TFLOPS if e["bound"] == "alu"
                         else e["gbs"] / PEAK_HBM_GBS)
            tb = traffic_of(workload_key, name, src_hash)
            if tb is not None:
                e["counter_mb_per_launch"] = tb / 1e6
                e["counter_over_alg_bytes"] = tb / (by / len(work))
        kern[name] = e
    dom = max((k for k in kern if "bound" in kern[k]), key=lambda k: ktimes[k][1])
    roof = {"kernel": dom, "bound": kern[dom]["bound"]}
    if roof["bound"] == "alu":
        roof.update({"achieved": kern[dom]["tflops"], "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s"})
    else:
        roof.update({"achieved": kern[dom]["gbs"], "peak": PEAK_HBM_GBS, "unit": "GB/s"})
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = traffic_of(workload_key, dom, src_hash)
    return {
        "wall": wall, "steps": steps, "Q": Q,
        "stored_updates_per_s": stored / wall,
        "evaluated_updates_per_s": evaluated / wall,
        "ms_per_step": wall * 1e3 / steps,
        "ms_per_step_with_kernel_events": wall_ev * 1e3 / steps,
        "plans_per_s": steps / wall, "v_node_expansions_per_s": exp / wall,
        "child_nodes_per_s": kids / wall,
        "nodes_per_level": counts[seeds[0]],
        "roofline": roof, "kernels": kern,
        "value_iteration": {"sweeps": sweeps, "residual": res, "ms": vi_ms,
                            "sweeps_per_s": sweeps / (vi_ms * 1e-3)},
    }


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
            "evaluated_belief_updates_per_s": upd / t_batch,
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


def progress(msg):
    """A line on stderr as each part of the run ends (stdout carries only the
    JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bench_closed_loop(args, B, wl, torch, dev):
    """Closed-loop runs of the experiment model of Sec. V on the synthetic
    100 x 40 map (nine actions, 0.95 sensor, the paper's stage reward):
    plan, act in the simulated world, observe, update the belief, until the
    robot stops or 400 steps; the comparison-table quantities over the runs,
    for the anytime search (FIB upper bound, blind-policy lower bound, a
    budget of expansions per step) and for the fixed-depth plan (Q-MDP
    leaves).  Runs r use world seed 1000 + r and draw seed 2000 + r."""
    from paper_1810_00204_amd.experiment import ClosedLoop, SearchLoop, summarize
    from paper_1810_00204_amd.planner import Planner
    prob = wl.make_paper(seed=0)
    pl = Planner(prob, device=dev)
    Q, _, qs = pl.value_iterate(tol=1e-6)
    F, _, fs = pl.fib_iterate(tol=1e-6)
    Lb, _, ls = pl.blind_iterate(tol=1e-6)
    desc = (f"{prob.name}: synthetic {prob.W}x{prob.H} map, 9 actions, wall bits read correctly "
            "w.p. 0.95, r in {-2,-1,0}, gamma 0.95, start belief uniform over free cells, "
            "stop on the stay action, 400-step cap")
    sl = SearchLoop(prob, F, Lb, expansions=args.loop_expansions, n=prob.n)
    runs = [sl.run(wl.Environment(prob, seed=1000 + r), seed=2000 + r, max_steps=400)
            for r in range(args.loop_runs)]
    search = summarize(runs)
    search.update({"planner": f"best-first search, {args.loop_expansions} expansions per step, "
                              f"n {prob.n}, U = FIB, L = blind policies, action = argmax L_Q"})
    cl = ClosedLoop(prob, Q)
    runs = [cl.run(wl.Environment(prob, seed=1000 + r), seed=2000 + r, max_steps=400)
            for r in range(args.loop_runs)]
    plan = summarize(runs)
    plan.update({"planner": f"fixed-depth plan, D {prob.D}, n {prob.n}, Q-MDP leaves"})
    return {"workload": desc, "search": search, "plan": plan,
            "sweeps": {"value_iteration": qs, "fib": fs, "blind": ls}}


def bench_search(B, torch, dev, wl, expansions=256):
    """Best-first expansions/s on the 100 x 40 experiment map (9 actions,
    n 3): one search of `expansions` expansions from the uniform belief."""
    from paper_1810_00204_amd.planner import Planner, SearchPlanner
    prob = wl.make_paper(seed=0)
    pl = Planner(prob, device=dev)
    F, _, _ = pl.fib_iterate(tol=1e-6)
    Lb, _, _ = pl.blind_iterate(tol=1e-6)
    sp = SearchPlanner(prob, F, Lb, max_nodes=1 + expansions * prob.A * prob.n, device=dev)
    sp.init()
    sp.expand(8, seed=1, query_id=0)
    torch.cuda.synchronize()
    sp.init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sp.expand(expansions, seed=1, query_id=0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    g = sp.records()
    return {"workload": f"{prob.name}, uniform start belief", "expansions": g["expansions"],
            "ms": dt * 1e3, "expansions_per_s": g["expansions"] / dt,
            "nodes": int(g["next"]), "child_nodes_per_s": (int(g["next"]) - 1) / dt}


def bench_fib(B, torch, dev, prob):
    """The fast informed bound of the headline workload: sweeps to a 1e-6
    relative residual in one cooperative launch."""
    m = B.DeviceModel(prob, dev)
    al = torch.empty(m.S * m.A, dtype=torch.float32, device=dev)
    ws = torch.empty(B.qv_fib_workspace_bytes(m, 10000), dtype=torch.uint8, device=dev)
    B.check(B.qv_fib_iterate(m, 1e-6, 10000, al, ws)[0], "qv_fib_iterate")   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, res, sw = B.qv_fib_iterate(m, 1e-6, 10000, al, ws)
    B.check(st, "qv_fib_iterate")
    ms = (time.perf_counter() - t0) * 1e3
    return {"sweeps": sw, "residual": res, "ms": ms, "sweeps_per_s": sw / (ms * 1e-3),
            "cell_action_backups_per_s": sw * m.S * m.A / (ms * 1e-3)}


def source_hash():
    from paper_1810_00204_amd.build import source_hash as h
    return h()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the planning path runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    prob = make_problem(args.workload)
    seeds = [prob.seed + i for i in range(args.seeds)]
    # the CPU legs first, in forked workers, before anything touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(args.workload, seeds, args.cpu_runs)
    if cpu is not None:
        progress(f"cpu baseline done: {cpu['value']:.3e} updates/s on {cpu['cores']} cores")

    import torch
    from paper_1810_00204_amd import binding as B
    from paper_1810_00204_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    B.lib()
    dev = "cuda:0"
    src = source_hash()
    flags = B.QV_PLAN_TILED if args.banded else 0
    r = plan_bench(B, torch, dev, prob, args.steps, args.warmup, args.seeds, flags,
                   args.workload, src)
    progress(f"{prob.name}: {r['ms_per_step']:.4f} ms per plan")

    if args.copy_calibration:
        for mib in (256, 512):
            a = torch.empty(mib << 20, dtype=torch.uint8, device=dev)
            b = torch.empty_like(a)
            for _ in range(3):
                b.copy_(a)
            torch.cuda.synchronize()
            del a, b

    line = {
        "metric": METRIC, "value": r["stored_updates_per_s"], "unit": "belief-state updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": prob.name, "grid": f"{prob.W}x{prob.H}", "actions": prob.A,
                   "landmarks": prob.L, "depth": prob.D, "samples_per_action": prob.n,
                   "blocked_fraction": round(float(prob.occ.mean()), 4),
                   "draw_seeds": len(seeds), "parallelism": "single GPU",
                   "kernels": "banded" if args.banded else "auto", "source_hash": src},
        "value_counts": "posterior cells written out (levels 1..D-1, all S cells per valid child)",
        "evaluated_belief_updates_per_s": r["evaluated_updates_per_s"],
        "ms_per_step_with_kernel_events": r["ms_per_step_with_kernel_events"],
        "plans_per_s": r["plans_per_s"], "v_node_expansions_per_s": r["v_node_expansions_per_s"],
        "child_nodes_per_s": r["child_nodes_per_s"], "nodes_per_level": r["nodes_per_level"],
        "roofline": r["roofline"], "kernels": r["kernels"],
        "value_iteration": r["value_iteration"],
    }
    if not args.only_headline:
        side = "rect64" if args.workload == "large512" else "large512"
        sp = make_problem(side)
        rs = plan_bench(B, torch, dev, sp, args.side_steps, args.warmup, args.seeds, flags,
                        side, src)
        line[side] = {"workload": sp.name, "ms_per_plan": rs["ms_per_step"],
                      "plans_per_s": rs["plans_per_s"],
                      "stored_belief_updates_per_s": rs["stored_updates_per_s"],
                      "evaluated_belief_updates_per_s": rs["evaluated_updates_per_s"],
                      "nodes_per_level": rs["nodes_per_level"], "roofline": rs["roofline"],
                      "kernels": rs["kernels"], "value_iteration": rs["value_iteration"]}
        progress(f"{sp.name}: {rs['ms_per_step']:.4f} ms per plan")
        line["batch"] = bench_batch(args, B, wl, torch, dev)
        progress(f"batch: {line['batch']['ms_per_batch']:.3f} ms per batch")
        line["filter"] = bench_filter(args, B, wl, torch, dev)
        progress(f"filter: {line['filter']['ms_per_eval']:.3f} ms per evaluation")
        line["fib"] = bench_fib(B, torch, dev, prob)
        progress(f"fib: {line['fib']['sweeps']} sweeps in {line['fib']['ms']:.2f} ms")
        line["search"] = bench_search(B, torch, dev, wl)
        progress(f"search: {line['search']['expansions_per_s']:.0f} expansions/s")
        line["closed_loop"] = bench_closed_loop(args, B, wl, torch, dev)
        progress(f"closed loop: failure rate search {line['closed_loop']['search']['failure_rate']:.2f}, "
                 f"plan {line['closed_loop']['plan']['failure_rate']:.2f}")
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
