"""Per-kernel summaries of rocprofv3 CSV output, as markdown tables.

    python -m paper_2508_13615_amd.profsum stats  <prefix_kernel_stats.csv> [--top N]
    python -m paper_2508_13615_amd.profsum pmc    <prefix_counter_collection.csv> <out.json>
    python -m paper_2508_13615_amd.profsum traffic <fetch.json> <write.json> <stats.csv>
    python -m paper_2508_13615_amd.profsum sweep-pmc <fetch.json> <write.json> <source_sha256>
    python -m paper_2508_13615_amd.profsum counters <prefix_counter_collection.csv> [more.csv ...]
    python -m paper_2508_13615_amd.profsum sweep-lines <fetch.json> <write.json> [qubits]
    python -m paper_2508_13615_amd.profsum engine-bounds <bench_line.json> <name>=<counters.csv> ... [--qubits N]

``stats`` tabulates the kernel statistics that ``rocprofv3 --stats`` writes.
``pmc`` folds a per-dispatch counter CSV (one counter per run) into
per-kernel aggregates, small enough to keep.  ``traffic`` combines a
FETCH_SIZE and a WRITE_SIZE aggregate with the kernel times: both counters are
scaled by what they read for the library's streaming copy in the same run,
which copies one whole state (as many bytes read as written), so that the
scaled write of the copy equals its scaled read.  ``sweep-pmc`` gives the same
per launch for every kernel, with a machine-readable block (bytes per
launch, scale factors, and the hash of the kernel sources the counters were
taken with) that ``bench.py`` reads for ``roofline.traffic``.  ``counters``
tabulates several counters per kernel (any number of runs, each with its own
counter set): totals over the run and, where SQ_WAVES was collected, per
wavefront.  ``sweep-lines`` sets each sweep kernel's measured traffic (all
its dispatches of one benchmark step) beside the algorithmic and the
line-granular bytes of the gate cases the benchmark launches on it (the case
list and kernel choice come from bench.py and the library's host-only
sv_plan_info).  ``engine-bounds`` sets the circuits benchmark's engine runs
(seconds per run from its bench line, one counter run per circuit holding
SQ_INSTS_VALU, SQ_INSTS_SALU and SQ_WAVES) against their HBM floor (every
forward pass reads and writes the state once, the observable pass reads it:
(2 passes + 1) S at 8 TB/s) and their VALU issue floor (a wave64 VALU
instruction takes 4 cycles of a 16-lane SIMD; 1024 SIMDs at 2.4 GHz); the
benchmark runs each circuit 4 times (a warm-up and 3 timed runs), so counter
totals are divided by 4.  Pass and layout counts come from the library's
host-only batch planner with the shipped tuning table.
"""
from __future__ import annotations

import csv
import json
import sys

# The reference of known size: the library's streaming copy (sv_stream_bench
# mode 0) of one whole state, which the benchmark runs before the sweep; its
# instantiations k_stream<0, U> all read and write the same bytes.
COPY_PREFIX = "k_stream<0,"


def copy_reference(counter_json: dict) -> float:
    """Per-dispatch value of the streaming copy (median over its launch shapes)."""
    vals = sorted(v["mean"] for k, v in counter_json.items() if k.startswith(COPY_PREFIX))
    if not vals:
        raise SystemExit("no streaming-copy dispatch (k_stream<0, ...>) in the counter data")
    return vals[len(vals) // 2]


def short_name(k: str) -> str:
    """Kernel name without return type, namespace and parameter list."""
    k = k.replace("void ", "").replace("svk::", "")
    return k.split("(")[0] if "(" in k and not k.startswith("__") else k[:80]


def read_stats(path: str) -> dict:
    out = {}
    for r in csv.DictReader(open(path)):
        out[short_name(r["Name"])] = {"calls": int(r["Calls"]), "total_ms": float(r["TotalDurationNs"]) / 1e6,
                                      "avg_ms": float(r["AverageNs"]) / 1e6, "min_ms": float(r["MinNs"]) / 1e6,
                                      "max_ms": float(r["MaxNs"]) / 1e6, "pct": float(r["Percentage"])}
    return out


def stats_table(path: str, top: int = 40) -> str:
    s = sorted(read_stats(path).items(), key=lambda kv: -kv[1]["total_ms"])[:top]
    rows = ["| kernel | calls | avg ms | min ms | max ms | total ms | % |", "|---|---|---|---|---|---|---|"]
    for k, v in s:
        rows.append(f"| `{k}` | {v['calls']} | {v['avg_ms']:.4f} | {v['min_ms']:.4f} | {v['max_ms']:.4f} | "
                    f"{v['total_ms']:.1f} | {v['pct']:.2f} |")
    return "\n".join(rows)


def pmc_aggregate(path: str) -> dict:
    agg = {}
    for r in csv.DictReader(open(path)):
        k = short_name(r["Kernel_Name"])
        v = float(r["Counter_Value"])
        a = agg.setdefault(k, {"counter": r["Counter_Name"], "dispatches": 0, "sum": 0.0, "min": float("inf"),
                               "max": 0.0})
        a["dispatches"] += 1
        a["sum"] += v
        a["min"] = min(a["min"], v)
        a["max"] = max(a["max"], v)
    for a in agg.values():
        a["mean"] = a["sum"] / a["dispatches"]
    return agg


def traffic_table(fetch_json: str, write_json: str, stats_csv: str, min_ms: float = 1.0) -> str:
    f = json.load(open(fetch_json))
    w = json.load(open(write_json))
    st = read_stats(stats_csv)
    copy_f, copy_w = copy_reference(f), copy_reference(w)
    # one copy reads and writes the same bytes: WRITE_SIZE counts them at face value
    ff = copy_w / copy_f
    head = (f"Scale factors from the streaming copy `{COPY_PREFIX} U>` (one whole state copied): FETCH_SIZE "
            f"{copy_f:.0f} KiB, WRITE_SIZE {copy_w:.0f} KiB per dispatch, so fetch x{ff:.4f}, write x1.0000.\n\n")
    rows = ["| kernel | dispatches | total ms | read GiB | written GiB | measured GB/s |", "|---|---|---|---|---|---|"]
    for k, t in sorted(st.items(), key=lambda kv: -kv[1]["total_ms"]):
        if k not in f or k not in w or t["total_ms"] < min_ms:
            continue
        rd = f[k]["sum"] * ff * 1024 / 2 ** 30
        wr = w[k]["sum"] * 1024 / 2 ** 30
        gbps = (rd + wr) * 2 ** 30 / 1e9 / (t["total_ms"] / 1e3)
        rows.append(f"| `{k}` | {f[k]['dispatches']} | {t['total_ms']:.1f} | {rd:.1f} | {wr:.1f} | {gbps:.0f} |")
    return head + "\n".join(rows)


def sweep_pmc(fetch_json: str, write_json: str, sha: str) -> str:
    f = json.load(open(fetch_json))
    w = json.load(open(write_json))
    copy_f, copy_w = copy_reference(f), copy_reference(w)
    ff = copy_w / copy_f
    rows = ["| kernel | dispatches | FETCH KiB (raw) | WRITE KiB (raw) | read GiB (scaled) | written GiB (scaled) | "
            "traffic GB |", "|---|---|---|---|---|---|---|"]
    blk = {"fetch_factor": ff, "write_factor": 1.0, "source_sha256": sha, "kernels": {}}
    for k in sorted(f, key=lambda k: -f[k]["dispatches"]):
        if k.startswith("k_stream") or k not in w or not k.startswith("k_"):
            continue
        rd = f[k]["mean"] * ff * 1024
        wr = w[k]["mean"] * 1024
        rows.append(f"| `{k}` | {f[k]['dispatches']} | {f[k]['mean']:.0f} | {w[k]['mean']:.0f} | {rd / 2**30:.3f} | "
                    f"{wr / 2**30:.3f} | {(rd + wr) / 1e9:.2f} |")
        blk["kernels"][k] = {"dispatches": f[k]["dispatches"], "fetch_kib_raw": f[k]["mean"],
                             "write_kib_raw": w[k]["mean"], "read_bytes": rd, "write_bytes": wr,
                             "traffic_bytes": rd + wr}
    head = (f"The scale factors come from the library's streaming copy (`{COPY_PREFIX} U>`, sv_stream_bench) in "
            f"the same runs, which copies one whole state: FETCH_SIZE reads {copy_f:.0f} KiB for it (fetch factor "
            f"{ff:.4f}), WRITE_SIZE {copy_w:.0f} KiB (factor 1.0000).  Means per dispatch over the run.\n\n")
    return head + "\n".join(rows) + "\n\nMachine-readable (bytes per dispatch after scaling):\n\n```json\n" + \
        json.dumps(blk, indent=1) + "\n```\n"


def counters_table(paths) -> str:
    """Per kernel: every counter's total over its dispatches; per wavefront
    where the same run collected SQ_WAVES."""
    tot = {}   # kernel -> counter -> sum
    waves = {}  # (path, kernel) -> SQ_WAVES sum
    per_run = {}
    for path in paths:
        for r in csv.DictReader(open(path)):
            k = short_name(r["Kernel_Name"])
            c = r["Counter_Name"]
            v = float(r["Counter_Value"])
            tot.setdefault(k, {})
            tot[k][c] = tot[k].get(c, 0.0) + v
            per_run.setdefault((path, k), {})
            per_run[(path, k)][c] = per_run[(path, k)].get(c, 0.0) + v
            if c == "SQ_WAVES":
                waves[(path, k)] = waves.get((path, k), 0.0) + v
    names = sorted({c for v in tot.values() for c in v})
    rows = ["| kernel | counter | total | per wavefront |", "|---|---|---|---|"]
    for k in sorted(tot, key=lambda k: -tot[k].get("SQ_INSTS_VALU", 0.0)):
        if not k.startswith("k_"):
            continue
        for c in names:
            if c not in tot[k]:
                continue
            pw = ""
            for (path, kk), cnts in per_run.items():
                if kk == k and c in cnts and waves.get((path, k)):
                    pw = f"{cnts[c] / waves[(path, k)]:.1f}"
            rows.append(f"| `{k}` | {c} | {tot[k][c]:.4g} | {pw} |")
    return "\n".join(rows)


def sweep_lines(fetch_json: str, write_json: str, n: int = 30) -> str:
    import os

    import numpy as np

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    import paper_2508_13615_amd as sv
    import workloads as W
    f = json.load(open(fetch_json))
    w = json.load(open(write_json))
    ff = copy_reference(w) / copy_reference(f)
    S = (1 << n) * 16
    agg = {}
    for c in bench.sweep_cases(n, np.random.default_rng(1002), W):
        g, tg, ct, _, _ = c
        name = g if not ct else ({1: "CNOT", 2: "Toffoli"}[len(ct)] if g == "X" else g)
        for k, alg, line, nm in ((bench.kernel_of(sv, g, tg, ct, n=n), 2 * S * bench.touched_fraction(g, len(ct)),
                                  2 * S * bench.line_fraction(g, tg, ct, 3), name),
                                 (bench.kernel_of(sv, g, bench.dense_of(c, None)[0], (), True, n), 2 * S, 2 * S,
                                  "general")):
            a = agg.setdefault(k, [0, 0.0, 0.0, {}])
            a[0] += 1
            a[1] += alg
            a[2] += line
            a[3][nm] = a[3].get(nm, 0) + 1
    rows = ["| kernel | cases | measured / algorithmic | measured / line-granular | gate cases |", "|---|---|---|---|---|"]
    for k, (cnt, alg, line, names) in sorted(agg.items(), key=lambda kv: -kv[1][0]):
        if k not in f or k not in w:
            continue
        meas = (f[k]["mean"] * ff + w[k]["mean"]) * 1024 * f[k]["dispatches"]
        rows.append(f"| `{k}` | {cnt} | {meas / alg:.3f} | {meas / line:.3f} | "
                    + ", ".join(f"{nm} {c}" for nm, c in sorted(names.items())) + " |")
    return "\n".join(rows)


def engine_bounds(bench_line: str, runs: dict, n: int = 30, layers: int = 10) -> str:
    import os

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    import paper_2508_13615_amd as sv
    with open(bench_line) as f:
        secs = json.loads(f.read().strip().splitlines()[-1])["circuits32_s"]
    _, jobs = bench.circuit_jobs(n, layers)
    # forward pass kernels of 16 amplitudes per thread, both instances (with and
    # without the out-of-tile control test), summed
    kern = {"c128": "k_pass_fwd<double, 4", "c64": "k_pass_fwd<float, 4"}
    ebytes = {"c128": 16, "c64": 8}
    rows = ["| circuit | dtype | s per run (HIP events) | passes | gate ops (fused) | layout changes | "
            "HBM floor at 8 TB/s | VALU issue floor | VALU / wave / pass | SALU / wave / pass | VALU busy |",
            "|---|---|---|---|---|---|---|---|---|---|---|"]
    for name, path in runs.items():
        tot = {}
        for r in csv.DictReader(open(path)):
            k = short_name(r["Kernel_Name"])
            tot.setdefault(k, {})
            tot[k][r["Counter_Name"]] = tot[k].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        ops, th = jobs[name]
        for dt in ("c128", "c64"):
            c = {}
            for k, v in tot.items():
                if k.startswith(kern[dt]):
                    for cn, cv in v.items():
                        c[cn] = c.get(cn, 0.0) + cv
            plan = sv.batch_plan([(n, ops, len(th), "sum_z")], dt, with_grad=False)
            t = secs[f"{name}_{dt}"]
            hbm = (2 * plan["passes"] + 1) * (1 << n) * ebytes[dt] / 8e12
            valu = c["SQ_INSTS_VALU"] / 4 * 4 / (1024 * 2.4e9)
            rows.append(f"| {name} | {dt} | {t:.4f} | {plan['passes']} | {plan['fused_ops']} | "
                        f"{plan['layout_changes']} | {hbm:.4f} s | {valu:.4f} s | "
                        f"{c['SQ_INSTS_VALU'] / c['SQ_WAVES']:.0f} | {c['SQ_INSTS_SALU'] / c['SQ_WAVES']:.0f} | "
                        f"{valu / t:.2f} |")
    return "\n".join(rows)


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        top = int(argv[argv.index("--top") + 1]) if "--top" in argv else 40
        print(stats_table(argv[1], top))
    elif len(argv) == 3 and argv[0] == "pmc":
        json.dump(pmc_aggregate(argv[1]), open(argv[2], "w"), indent=1)
    elif len(argv) == 4 and argv[0] == "traffic":
        print(traffic_table(argv[1], argv[2], argv[3]))
    elif len(argv) == 4 and argv[0] == "sweep-pmc":
        print(sweep_pmc(argv[1], argv[2], argv[3]))
    elif len(argv) >= 2 and argv[0] == "counters":
        print(counters_table(argv[1:]))
    elif len(argv) >= 3 and argv[0] == "engine-bounds":
        n = int(argv[argv.index("--qubits") + 1]) if "--qubits" in argv else 30
        runs = dict(a.split("=", 1) for a in argv[2:] if "=" in a)
        print(engine_bounds(argv[1], runs, n))
    elif len(argv) in (3, 4) and argv[0] == "sweep-lines":
        print(sweep_lines(argv[1], argv[2], int(argv[3]) if len(argv) == 4 else 30))
    else:
        sys.exit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
