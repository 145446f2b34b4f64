"""Short text summaries of rocprofv3 output for profiles/.

  python -m paper_1810_00204_amd.rocprof_summary stats <kernel_stats.csv> \\
      --cmd "<the rocprofv3 command>" --out profiles/<kernel>_<workload>.md

writes the per-kernel duration table (calls, total, average, share);

  python -m paper_1810_00204_amd.rocprof_summary traffic \\
      --fetch <FETCH_SIZE counter_collection.csv> --write <WRITE_SIZE ...csv> \\
      --copy-bytes 536870912 --workload rect64 --cmd-fetch "..." --cmd-write "..." \\
      --out profiles/traffic_rect64.json

turns the two counter passes into HBM bytes per launch of each planning
kernel, per tree level.  Both counters read in KiB per dispatch; each is
scaled by what it reads for a plain device copy of --copy-bytes bytes (the
largest copy dispatch of the run), so the result is in bytes actually
moved.  Levels are told apart by grid size, from the tree shape of the
workload.
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

BLOCK = 256        # threads per workgroup of the banded planning kernels
NODE_BLOCK = 512   # k_node (inner levels) and k_leaf_parent workgroups


def short_name(full: str) -> str:
    """'void qv::k_node<8, true>(qv::DevModel, ...)' -> 'k_node<8, true>'."""
    s = full.strip()
    if s.startswith("void "):
        s = s[5:]
    depth = 0
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            s = s[:i]
            break
    return re.sub(r"^qv::", "", s)


def level_grids(workload: str):
    """{(kernel family, grid threads): level} for the planning kernels."""
    from paper_1810_00204_amd import workloads as wl
    prob = {"rect64": lambda: wl.make_rect(seed=0),
            "large512": lambda: wl.make_large(seed=0),
            "small10": lambda: wl.make_small(seed=0)}[workload]()
    A, K, D = prob.A, prob.A * prob.n, prob.D
    th = max(1, min(prob.H, 1024 // prob.W))
    tiles = (prob.H + th - 1) // th
    leaf_rows = max(1, min(prob.H, 8192 // prob.W))
    leaf_tiles = (prob.H + leaf_rows - 1) // leaf_rows
    out = {}
    for d in range(D):
        slots = K ** d
        # per-parent levels of few items run on thinner bands (as the planner)
        th_d, tiles_d = th, tiles
        while th_d > 1 and slots * tiles_d < 512:
            th_d = (th_d + 1) // 2
            tiles_d = (prob.H + th_d - 1) // th_d
        out[("k_node", slots * A * NODE_BLOCK)] = d
        if d == 0:   # level 0 also carries the leaf-band sort workgroups
            out[("k_node", (slots * A + leaf_tiles) * NODE_BLOCK)] = d
        for fam in ("k_stats", "k_update", "k_leaf"):
            out[(fam, slots * tiles * A * BLOCK)] = d
        for fam in ("k_stats_parent", "k_update_parent"):
            out[(fam, slots * tiles_d * BLOCK)] = d
        # a level of few items splits each (parent, band)'s actions over G
        # workgroups of the update launch
        G = 1
        while G < 4 and G * 2 <= A and slots * tiles_d * G * 2 <= 1024:
            G *= 2
        out[("k_update_parent", slots * tiles_d * G * BLOCK)] = d
        if d == 0:   # the level-0 statistics launch also carries the leaf-band sort
            out[("k_stats_parent", (slots * tiles_d + leaf_tiles) * BLOCK)] = d
        out[("k_stats_draws", slots * A * 64)] = d
    for d in range(1, D - 1):   # basis inner levels (the leaf kernel with R for Q)
        out[("k_leaf_parent", K ** d * leaf_tiles * NODE_BLOCK)] = d
        out[("k_inner_finish", K ** d * A * BLOCK)] = d
    out[("k_leaf_parent", K ** (D - 1) * leaf_tiles * NODE_BLOCK)] = D - 1
    out[("k_leaf_finish", K ** (D - 1) * NODE_BLOCK)] = D - 1
    return out


def family(name: str) -> str:
    return name.split("<", 1)[0]


def cmd_stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel statistics: {args.title}", "",
             "Command (from the repository root on the GPU host):", "",
             "```", args.cmd, "```", "",
             "| kernel | calls | total ms | average us | share |",
             "|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:args.top]:
        lines.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | "
                     f"{100.0 * float(r['TotalDurationNs']) / tot:.1f}% |")
    if args.trace:
        # the planning kernels by level, from the dispatches of the trace (a
        # kernel that runs at several levels has one row per level)
        grids = level_grids(args.workload)
        per = collections.defaultdict(list)
        for r in csv.DictReader(open(args.trace)):
            name = short_name(r["Kernel_Name"])
            lvl = grids.get((family(name), int(r["Grid_Size_X"])))
            if lvl is not None:
                per[f"{name}@L{lvl}"].append(
                    (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
        lines += ["", "Planning kernels by level (dispatch durations from the kernel trace):", "",
                  "| kernel@level | calls | average us |", "|---|---|---|"]
        for key, ds in sorted(per.items(), key=lambda kv: -sum(kv[1])):
            lines.append(f"| `{key}` | {len(ds)} | {sum(ds) / len(ds):.2f} |")
    open(args.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def cmd_markers(args):
    """Host time inside each roctx range (QVTS_ROCTX=1): the enqueueing of a
    plan and of each of its levels."""
    per = collections.defaultdict(list)
    for r in csv.DictReader(open(args.csv)):
        per[r["Function"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    lines = [f"# rocprofv3 marker trace: {args.title}", "",
             "Command (from the repository root on the GPU host):", "",
             "```", args.cmd, "```", "",
             "Host time between the push and the pop of each range (the launches are",
             "asynchronous: this is the cost of enqueueing, not of the kernels).", "",
             "| range | count | mean us | max us |", "|---|---|---|---|"]
    for name in sorted(per):
        ds = per[name]
        lines.append(f"| `{name}` | {len(ds)} | {sum(ds) / len(ds):.1f} | {max(ds):.1f} |")
    open(args.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _counter(path, copy_bytes):
    rows = list(csv.DictReader(open(path)))
    copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
    if not copies:
        raise SystemExit(f"{path}: no device copy dispatch to calibrate against")
    ref_kib = max(copies)
    scale = copy_bytes / ref_kib   # bytes per counter unit
    per = collections.defaultdict(list)
    for r in rows:
        per[(short_name(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return per, scale, ref_kib


def cmd_traffic(args):
    from paper_1810_00204_amd.build import source_hash
    grids = level_grids(args.workload)
    fetch, fs, fref = _counter(args.fetch, args.copy_bytes)
    write, ws, wref = _counter(args.write, args.copy_bytes)
    kern = {}
    for (name, grid), vals in fetch.items():
        lvl = grids.get((family(name), grid))
        if lvl is None:
            continue
        key = f"{name}@L{lvl}"
        wv = write.get((name, grid), [0.0])
        fb = fs * sum(vals) / len(vals)
        wb = ws * sum(wv) / len(wv)
        kern[key] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                     "dispatches": len(vals)}
    out = {"source_hash": source_hash(), "workload": args.workload,
           "copy_bytes": args.copy_bytes,
           "counter_reading_of_copy_kib": {"FETCH_SIZE": fref, "WRITE_SIZE": wref},
           "bytes_per_counter_unit": {"FETCH_SIZE": fs, "WRITE_SIZE": ws},
           "commands": {"FETCH_SIZE": args.cmd_fetch, "WRITE_SIZE": args.cmd_write},
           "kernels": kern}
    json.dump(out, open(args.out, "w"), indent=1)
    print(json.dumps(out, indent=1))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    s.add_argument("--title", default="")
    s.add_argument("--top", type=int, default=12)
    s.add_argument("--out", required=True)
    s.add_argument("--trace", default="", help="kernel trace csv: adds per-level rows")
    s.add_argument("--workload", default="rect64")
    mk = sub.add_parser("markers")
    mk.add_argument("csv")
    mk.add_argument("--cmd", required=True)
    mk.add_argument("--title", default="")
    mk.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-bytes", type=int, default=512 << 20)
    t.add_argument("--workload", default="rect64")
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--out", required=True)
    a = ap.parse_args()
    {"stats": cmd_stats, "traffic": cmd_traffic, "markers": cmd_markers}[a.mode](a)


if __name__ == "__main__":
    main()
