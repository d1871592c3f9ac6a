"""Autotuner for libsv's launch shapes.

For every kernel class (paired, subset phase, element-wise diagonal,
two-target, general), both dtypes and the three run-length tiers (bytes
spanned by a run of consecutive touched amplitudes: < 64 B, < 1 KiB, larger),
it times representative gates under each candidate shape
(block x groups-per-thread x non-temporal flag) with HIP events and keeps the
fastest.  The result is written as JSON next to the library and loaded by
``paper_2508_13615_amd`` at import (``apply_table``).

Run on the GPU:  python -m paper_2508_13615_amd.autotune [--qubits 30]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_mi355x.json")
CLASSES = {0: "paired", 1: "subset", 2: "diagonal", 3: "two-target", 4: "general"}
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
    return len(tab["entries"])


def _tier_qubit(dtype: str, tier: int) -> list:
    """Lowest touched qubits that fall in a tier (2^q * elem bytes)."""
    eb = 16 if dtype == "c128" else 8
    qs = [q for q in range(0, 30) if {0: eb << q < 64, 1: 64 <= eb << q < 1024, 2: eb << q >= 1024}[tier]]
    if tier == 2:
        return [qs[len(qs) // 3], qs[-1]]
    return [qs[0], qs[-1]]


def _cases(kc: int, dtype: str, tier: int, n: int):
    """(gate, targets, controls) cases whose lowest touched qubit lies in the tier."""
    import numpy as np
    out = []
    rng = np.random.default_rng(11)
    for low in _tier_qubit(dtype, tier):
        hi = n - 1 if low != n - 1 else n - 2
        if kc == 0:
            out.append(("RY", (low,), (), (0.3,), None))
            out.append(("X", (hi,), (low,), (), None))
        elif kc == 1:
            out.append(("Z", (low,), (), (), None))
        elif kc == 2:
            out.append(("RZ", (hi,), (low,), (0.3,), None))
        elif kc == 3:
            z = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
            out.append(("U4", (hi, low), (), (), np.linalg.qr(z)[0]))
        else:
            out.append(("GENERAL", (hi, low), (), (), None))
    return out


def tune(qubits: int = 30, reps: int = 3, dtypes=("c128", "c64"), log=print) -> dict:
    import numpy as np
    import torch

    import paper_2508_13615_amd as sv

    entries = []
    u4 = np.linalg.qr(np.random.default_rng(5).standard_normal((4, 4)) + 0j)[0]
    for dtype in dtypes:
        st = sv.State(qubits, dtype, basis=0)
        stream = torch.cuda.current_stream()
        for kc in CLASSES:
            for tier in range(3):
                cases = _cases(kc, dtype, tier, qubits)
                best = None
                for block in BLOCKS:
                    for unroll in UNROLLS:
                        for nt in (0, 1):
                            sv.tune_set(kc, dtype, tier, block, unroll, nt)
                            times = []
                            for _ in range(reps + 1):
                                e0 = torch.cuda.Event(enable_timing=True)
                                e1 = torch.cuda.Event(enable_timing=True)
                                e0.record(stream)
                                for g, tg, ct, p, m in cases:
                                    if g == "GENERAL":
                                        st.apply_general(tg, u4)
                                    else:
                                        st.apply(g, tg, ct, p, m)
                                e1.record(stream)
                                e1.synchronize()
                                times.append(e0.elapsed_time(e1))
                            t = float(np.median(times[1:]))
                            if best is None or t < best[0]:
                                best = (t, block, unroll, nt)
                t, block, unroll, nt = best
                sv.tune_set(kc, dtype, tier, block, unroll, nt)
                entries.append({"class": kc, "class_name": CLASSES[kc], "dtype": dtype, "tier": tier,
                                "block": block, "unroll": unroll, "nt": nt, "ms_per_case": t / len(cases),
                                "cases": [(c[0], list(c[1]), list(c[2])) for c in cases]})
                log(f"[autotune] {dtype} {CLASSES[kc]:10s} tier {tier}: block {block} unroll {unroll} nt {nt} "
                    f"({t / len(cases):.3f} ms per gate)")
        del st
        torch.cuda.empty_cache()
    return {"device": torch.cuda.get_device_name(0), "qubits": qubits, "reps": reps,
            "created": time.strftime("%Y-%m-%d %H:%M:%S"), "entries": entries}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--qubits", type=int, default=30)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=TABLE)
    args = ap.parse_args()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    tab = tune(args.qubits, args.reps, log=lambda *a: print(*a, file=sys.stderr, flush=True))
    with open(args.out, "w") as f:
        json.dump(tab, f, indent=1)
    print(f"wrote {args.out} ({len(tab['entries'])} entries)", file=sys.stderr)


if __name__ == "__main__":
    main()
