"""Per-kernel summaries of rocprofv3 CSV output, as markdown tables.

    python -m paper_2508_13615_amd.profsum stats  <prefix_kernel_stats.csv> [--top N]
    python -m paper_2508_13615_amd.profsum pmc    <prefix_counter_collection.csv> <out.json>
    python -m paper_2508_13615_amd.profsum traffic <fetch.json> <write.json> <stats.csv>
    python -m paper_2508_13615_amd.profsum sweep-pmc <fetch.json> <write.json> <source_sha256>

``stats`` tabulates the kernel statistics that ``rocprofv3 --stats`` writes.
``pmc`` folds a per-dispatch counter CSV (one counter per run) into
per-kernel aggregates, small enough to keep.  ``traffic`` combines a
FETCH_SIZE and a WRITE_SIZE aggregate with the kernel times: both counters are
scaled by what they read for the runtime's copy kernel in the same run, which
copies one whole state (as many bytes read as written), so that the scaled
write of the copy equals its scaled read.  ``sweep-pmc`` gives the same
per launch for every kernel, with a machine-readable block (bytes per
launch, scale factors, and the hash of the kernel sources the counters were
taken with) that ``bench.py`` reads for ``roofline.traffic``.
"""
from __future__ import annotations

import csv
import json
import sys

COPY_KERNEL = "__amd_rocclr_copyBuffer"


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
    copy_f, copy_w = f[COPY_KERNEL]["max"], w[COPY_KERNEL]["max"]
    # one copy reads and writes the same bytes: WRITE_SIZE counts them at face value
    ff = copy_w / copy_f
    head = (f"Scale factors from `{COPY_KERNEL}` (one whole state copied): FETCH_SIZE {copy_f:.0f} KiB, "
            f"WRITE_SIZE {copy_w:.0f} KiB per dispatch, so fetch x{ff:.4f}, write x1.0000.\n\n")
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
    copy_f, copy_w = f[COPY_KERNEL]["max"], w[COPY_KERNEL]["max"]
    ff = copy_w / copy_f
    rows = ["| kernel | dispatches | FETCH KiB (raw) | WRITE KiB (raw) | read GiB (scaled) | written GiB (scaled) | "
            "traffic GB |", "|---|---|---|---|---|---|---|"]
    blk = {"fetch_factor": ff, "write_factor": 1.0, "source_sha256": sha, "kernels": {}}
    for k in sorted(f, key=lambda k: -f[k]["dispatches"]):
        if k == COPY_KERNEL or k not in w or not k.startswith("k_"):
            continue
        rd = f[k]["mean"] * ff * 1024
        wr = w[k]["mean"] * 1024
        rows.append(f"| `{k}` | {f[k]['dispatches']} | {f[k]['mean']:.0f} | {w[k]['mean']:.0f} | {rd / 2**30:.3f} | "
                    f"{wr / 2**30:.3f} | {(rd + wr) / 1e9:.2f} |")
        blk["kernels"][k] = {"dispatches": f[k]["dispatches"], "fetch_kib_raw": f[k]["mean"],
                             "write_kib_raw": w[k]["mean"], "read_bytes": rd, "write_bytes": wr,
                             "traffic_bytes": rd + wr}
    head = (f"The scale factors come from the runtime's copy kernel (`{COPY_KERNEL}`) in the same runs, which "
            f"copies one whole state: FETCH_SIZE reads {copy_f:.0f} KiB for it (fetch factor {ff:.4f}), "
            f"WRITE_SIZE {copy_w:.0f} KiB (factor 1.0000).  Means per dispatch over the run.\n\n")
    return head + "\n".join(rows) + "\n\nMachine-readable (bytes per dispatch after scaling):\n\n```json\n" + \
        json.dumps(blk, indent=1) + "\n```\n"


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
    else:
        sys.exit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
