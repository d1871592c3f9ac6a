"""Autotuner for libsv's launch shapes.

For every kernel class (paired, subset phase, two-target, general,
wavefront-paired, LDS-staged), both dtypes and the three run-length tiers (bytes
spanned by a run of consecutive touched amplitudes: < 64 B, < 1 KiB, larger),
it times representative gates under each candidate shape
(block x groups-per-thread x non-temporal flag) with HIP events and keeps the
fastest.  For the fused pass engine it times every tile shape (tile qubits x
amplitudes per thread), per dtype and per stage mix.  Batches with the
adjoint sweep are timed on the adjoint gradient of a 24-qubit, 8-layer
hardware-efficient ansatz, on a batch of 256 such circuits of 14-22 qubits
and on the adjoint gradient of a 28-qubit, 4-layer one (a state far larger
than the caches).  Forward-only batches are timed on a 30-qubit, 10-layer
ansatz, a 30-qubit QFT and the same batch of 256 without the adjoint.  The
result is written as JSON next to the library and loaded by
``paper_2508_13615_amd`` at import (``apply_table``).

Run on the GPU:  python -m paper_2508_13615_amd.autotune [--qubits 30] [--engine-only | --classes K ...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_mi355x.json")
CLASSES = {0: "paired", 1: "subset", 3: "two-target", 4: "general", 5: "wave", 6: "lds"}
BLOCKS = (64, 128, 256, 512)
UNROLLS = (1, 2, 4)


def apply_table(sv, path: str = TABLE) -> int:
    """Load a tuning table into the library; returns the number of entries."""
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        tab = json.load(f)
    for e in tab["entries"]:
        sv.tune_set(e["class"], e["dtype"], e["tier"], e["block"], e["unroll"], e["nt"])
    for e in tab.get("engine", []):
        sv.tune_engine_set(e["dtype"], e["with_grad"], e["tile_qubits"], e["amps_per_thread"])
    return len(tab["entries"]) + len(tab.get("engine", []))


def _candidates(kc: int, n: int, rng, np):
    """Gate cases of a kernel class with the lowest touched qubit swept from 0."""
    hi = n - 1
    for low in range(0, n - 2):
        if kc == 0:
            yield low, ("SWAP", (low, hi), (), (), None)
        elif kc == 1:
            yield low, ("Z", (low,), (), (), None)
        elif kc == 3:
            z = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
            yield low, ("U4", (hi, low), (), (), np.linalg.qr(z)[0])
        elif kc == 4 or kc == 6:
            yield low, ("GENERAL", (hi, low), (), (), None)
        else:
            ctl = (low,) if low >= 6 else ()
            yield low, ("H", (low % 6,), ctl, (), None)


def _lds_cases(sv, dtype: str, tier: int, n: int):
    """The LDS-staged kernel at the lowest qubit of `tier`, in each of its
    forms: 2-qubit matrices with none or one of the qubits above the staged
    chunk, 3-qubit matrices with one or two above it, and the SWAP move.  Its
    best block differs between these forms, so the tier's shape is chosen on
    all of them together; the unroll (lines staged per thread per round
    trip) acts on the 3-qubit form only."""
    lows = [lo for lo in range(0, 6) if sv.plan_info(n, dtype, "GENERAL", (n - 1, lo))["class"] == 6
            and sv.plan_info(n, dtype, "GENERAL", (n - 1, lo))["tier"] == tier]
    if not lows:
        return []
    lo = lows[0]  # at most 5; qubits lo + 1 .. 7 sit inside the chunk
    forms = [("GENERAL", (n - 1, lo)), ("GENERAL", (lo, 7)), ("GENERAL", (n - 1, n // 2, lo)),
             ("GENERAL", (lo, lo + 1, n - 1)), ("SWAP", (n - 1, lo))]
    out = []
    for g, tg in forms:
        info = sv.plan_info(n, dtype, g, tg)
        if info["class"] == 6 and info["tier"] == tier:
            out.append((g, tg, (), (), None))
    return out


def _cases(sv, kc: int, dtype: str, tier: int, n: int):
    """Up to two cases (lowest and highest reachable position) that libsv
    launches with kernel class `kc` in `tier`; [] if the tier is unreachable.
    The LDS-staged class takes one case per form of the kernel instead."""
    import numpy as np
    if kc == 6:
        return _lds_cases(sv, dtype, tier, n)
    rng = np.random.default_rng(11)
    hits = []
    for low, case in _candidates(kc, n, rng, np):
        g, tg, ct = case[0], case[1], case[2]
        info = sv.plan_info(n, dtype, g, tg, ct)
        if info["class"] == kc and info["tier"] == tier:
            hits.append(case)
    if len(hits) > 2:
        hits = [hits[0], hits[len(hits) // 2]]
    return hits


def _time_shape(sv, torch, st, kc, dtype, tier, shape, cases, dense, reps):
    import numpy as np
    sv.tune_set(kc, dtype, tier, *shape)
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(reps + 1):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for g, tg, ct, p, m in cases:
            if g == "GENERAL":
                st.apply_general(tg, dense[len(tg)])
            else:
                st.apply(g, tg, ct, p, m)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    return float(np.median(times[1:]))


def tune(qubits: int = 30, reps: int = 3, dtypes=("c128", "c64"), log=print, margin: float = 0.02,
         classes=tuple(CLASSES)) -> dict:
    """Two rounds per key: every candidate once (median of `reps`), then the
    four fastest and the library default again, interleaved, median of
    2*`reps`.  A candidate replaces the default only if it is `margin` faster."""
    import numpy as np
    import torch

    import paper_2508_13615_amd as sv

    entries = []
    # dense unitaries for the GENERAL cases, by qubit count
    dense = {k: np.linalg.qr(np.random.default_rng(3 + k).standard_normal((2 ** k, 2 ** k)) + 0j)[0] for k in (2, 3)}
    shapes = [(b, u, nt) for b in BLOCKS for u in UNROLLS for nt in (0, 1)]
    for dtype in dtypes:
        st = sv.State(qubits, dtype, basis=0)
        for kc in classes:
            for tier in range(3):
                cases = _cases(sv, kc, dtype, tier, qubits)
                if not cases:
                    log(f"[autotune] {dtype} {CLASSES[kc]:10s} tier {tier}: not reachable, default kept")
                    continue
                default = sv.tune_get(kc, dtype, tier)
                first = sorted((_time_shape(sv, torch, st, kc, dtype, tier, sh, cases, dense, reps), sh) for sh in shapes)
                finalists = [sh for _, sh in first[:4]]
                if default not in finalists:
                    finalists.append(default)
                acc = {sh: [] for sh in finalists}
                for _ in range(2):
                    for sh in finalists:
                        acc[sh].append(_time_shape(sv, torch, st, kc, dtype, tier, sh, cases, dense, reps))
                med = {sh: float(np.median(v)) for sh, v in acc.items()}
                best = min(med, key=med.get)
                if med[best] > (1.0 - margin) * med[default]:
                    best = default
                sv.tune_set(kc, dtype, tier, *best)
                block, unroll, nt = best
                entries.append({"class": kc, "class_name": CLASSES[kc], "dtype": dtype, "tier": tier,
                                "block": block, "unroll": unroll, "nt": nt,
                                "ms_per_case": med[best] / len(cases),
                                "default": list(default), "default_ms_per_case": med[default] / len(cases),
                                "cases": [(c[0], list(c[1]), list(c[2])) for c in cases]})
                log(f"[autotune] {dtype} {CLASSES[kc]:10s} tier {tier}: block {block} unroll {unroll} nt {nt} "
                    f"({med[best] / len(cases):.3f} ms per gate; default {default} "
                    f"{med[default] / len(cases):.3f})")
        del st
        torch.cuda.empty_cache()
    return {"device": torch.cuda.get_device_name(0), "qubits": qubits, "reps": reps, "margin": margin,
            "created": time.strftime("%Y-%m-%d %H:%M:%S"), "entries": entries}


# Engine tile shapes tried per dtype and stage mix: (tile_qubits,
# amps_per_thread).  Every one keeps forward workgroups, and with the adjoint
# reverse ones, within 64..512 threads.
def _engine_shape_ok(dtype, tq, apt, with_grad):
    rb = apt.bit_length() - 1
    rrb = min(rb, 3) if dtype == "c128" else rb
    return 6 <= tq - rb and tq - (min(rb, rrb) if with_grad else rb) <= 9


ENGINE_SHAPES = {(dt, g): [(t, a) for a in (8, 16) for t in range(9, 14) if _engine_shape_ok(dt, t, a, g)]
                 for dt in ("c128", "c64") for g in (True, False)}


def _engine_workloads(with_grad: bool):
    """(name, circuits) pairs for one stage mix: circuits as sv.Batch takes them."""
    import workloads as W
    spec = W.batch_spec(256, 1006, 14, 22, 4, 12)
    batch = [(c.n, W.hea_ops(c.n, c.layers), len(c.params), "sum_z") for c in spec]
    if with_grad:
        return [("adjoint_hea24", [(24, W.hea_ops(24, 8), W.hea_n_params(24, 8), "sum_zz")]),
                ("batch256", batch),
                ("adjoint_hea28", [(28, W.hea_ops(28, 4), W.hea_n_params(28, 4), "sum_zz")])]
    return [("hea30", [(30, W.hea_ops(30, 10), W.hea_n_params(30, 10), "sum_z")]),
            ("qft30", [(30, [W.Op("H", (), (q,)) for q in range(30)] + W.qft_ops(30), 0, "sum_z")]),
            ("batch256_forward", batch)]


def _time_engine(sv, circuits, dtype, shape, reps, with_grad=True):
    import numpy as np
    b = sv.Batch(circuits, dtype, tile_qubits=shape[0], amps_per_thread=shape[1], with_grad=with_grad)
    params = np.random.default_rng(7).uniform(0, 2 * np.pi, sum(c[2] for c in circuits))
    b.run(params)  # capture + first replay
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        b.run(params)
        times.append(time.perf_counter() - t0)
    del b
    return float(np.median(times))


def tune_engine(reps: int = 5, dtypes=("c128", "c64"), log=print, margin: float = 0.02) -> list:
    """Per dtype and stage mix: each shape's time on each workload of that mix,
    relative to the built-in default shape, averaged over the workloads; the
    best replaces the default only if it is `margin` faster.  Wall time of
    synchronous runs (parameters uploaded, expectation values and gradients
    read back) is what a caller sees."""
    import numpy as np
    import torch

    import paper_2508_13615_amd as sv

    out = []
    for dtype in dtypes:
        for grad in (True, False):
            mix = "adjoint" if grad else "forward"
            work = _engine_workloads(grad)
            sv.tune_engine_set(dtype, grad, 0, 0)
            default = sv.tune_engine_get(dtype, grad)
            shapes = ENGINE_SHAPES[(dtype, grad)]
            if default not in shapes:
                shapes = shapes + [default]
            t = {sh: {} for sh in shapes}
            for name, circs in work:
                for _ in range(2):  # two interleaved rounds, the faster kept
                    for sh in shapes:
                        v = _time_engine(sv, circs, dtype, sh, reps, grad)
                        t[sh][name] = min(v, t[sh].get(name, float("inf")))
                torch.cuda.empty_cache()
                log(f"[autotune] engine {dtype} {mix} {name}: {len(shapes)} shapes timed")
            score = {sh: float(np.mean([t[sh][n] / t[default][n] for n, _ in work])) for sh in shapes}
            for sh in shapes:
                log(f"[autotune] engine {dtype} {mix} tile_qubits {sh[0]:2d} amps_per_thread {sh[1]:2d}: "
                    + ", ".join(f"{n} {t[sh][n] * 1e3:.2f} ms" for n, _ in work) + f" (relative {score[sh]:.3f})")
            best = min(score, key=score.get)
            if score[best] > 1.0 - margin:
                best = default
            sv.tune_engine_set(dtype, grad, *best)
            out.append({"dtype": dtype, "with_grad": int(grad), "tile_qubits": best[0], "amps_per_thread": best[1],
                        "relative_to_default": score[best], "default": list(default),
                        "ms": {f"{sh[0]}x{sh[1]}": {n: t[sh][n] * 1e3 for n, _ in work} for sh in shapes}})
            log(f"[autotune] engine {dtype} {mix}: tile_qubits {best[0]} amps_per_thread {best[1]}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--qubits", type=int, default=30)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--engine-only", action="store_true",
                    help="tune only the fused engine's tile shape and keep the table's gate entries")
    ap.add_argument("--classes", type=int, nargs="+", choices=sorted(CLASSES),
                    help="tune only these gate kernel classes; the table's other entries, engine included, are kept")
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    if args.classes:
        with open(TABLE) as f:
            tab = json.load(f)
        new = tune(args.qubits, args.reps, log=log, classes=tuple(args.classes))
        keep = [e for e in tab["entries"] if e["class"] not in args.classes]
        tab["entries"] = sorted(keep + new["entries"], key=lambda e: (e["dtype"] != "c128", e["class"], e["tier"]))
        tab["created"] = new["created"]
    elif args.engine_only:
        with open(args.out) as f:
            tab = json.load(f)
        tab["engine"] = tune_engine(log=log)
    else:
        tab = tune(args.qubits, args.reps, log=log)
        tab["engine"] = tune_engine(log=log)
    with open(args.out, "w") as f:
        json.dump(tab, f, indent=1)
    print(f"wrote {args.out} ({len(tab['entries'])} gate entries, {len(tab['engine'])} engine entries)",
          file=sys.stderr)


if __name__ == "__main__":
    main()
