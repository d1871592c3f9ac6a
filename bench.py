#!/usr/bin/env python
"""Benchmark of the state-vector hot path on one MI355X.

One step = one pass of the single-gate sweep on a 30-qubit complex128 state
(16 GiB, seeded complex Gaussian, normalised): every gate class (H, X, Z, RZ,
RY, U2, CNOT, SWAP, U4, Toffoli) on every target 0..29, with the second qubit
or controls drawn from {0, 15, 29}; each case runs through the gate-specific
kernel and through the general dense kernel (the paper's two approaches,
Sec. 3.1), and the step ends with one expectation value (sum_i Z_i Z_{i+1}).
`value` is gates/s of the gate-specific kernels over the timed steps.

The last stdout line is one compact JSON object (the headline): value,
ms_per_step, roofline, cpu_baseline and one summary figure per section.
Everything else -- per class, per kernel, per target, every section in full --
goes to a detail JSON file (--detail, default gpurun_out/bench_detail.json).
Sections:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                average HIP-event-timed launch duration, against 8 TB/s;
                `traffic` is its measured HBM bytes per launch, read from the
                committed PMC summary (null once the sweep kernels' sources
                differ from the ones the counters were taken with);
  ceiling       the library's streaming kernel (sv_stream_bench) copying,
                reading and writing the state's bytes: the measured ceiling;
  classes       per gate class, gate-specific and general kernel as fractions
                of 8 TB/s; the half- and quarter-touch classes (Z, CNOT, SWAP,
                Toffoli) also over the cases whose lowest touched qubit is at
                or above the 128-byte line bits, where their algorithmic bytes
                are also their line-granular bytes;
  sweep_c64     the same sweep on a complex64 state (secondary, one step);
  adjoint       24 qubits, 8 layers RY+RZ + CNOT ladder, 384 params,
                sum Z_i Z_{i+1}: one adjoint-gradient call vs parameter shift
                (2 forward+expval runs per parameter) on the same GPU, on the
                op-by-op kernels, with the error of each dtype's gradient
                against the oracle's parameter-shift gradient on 16 sampled
                parameters (stored reference, tests/golden);
  adjoint_fused the same on the fused pass engine;
  batch         256 circuits of 14..22 qubits, forward + gradient in one
                graph launch, vs the same circuits one after another;
  circuits32    32-qubit HEA (10 layers), QFT and universal circuit;
  circuits20    the 20-qubit HEA and QFT in both dtypes against the oracle's
                stored results (max-abs amplitude error on 1024 sampled
                amplitudes, sum Z_i energy error);
  cpu_baseline  the oracle on the host cores on a bounded sample (and on one
                thread), with the host's CPU model and memory, and one oracle
                forward + expectation of the 24-qubit adjoint workload.
Progress lines go to stderr; stdout carries only the JSON line.
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

METRIC = "gates/sec & effective HBM GB/s at 30 qubits c128; adjoint grad vs param-shift s"
PEAK_GBPS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pmc_sweep30_c128.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_of(sv, gate, tg, ct, general=False, n=30, dtype="c128"):
    """The kernel instantiation libsv launches for a case (from sv_plan_info)."""
    if general:
        return sv.plan_info(n, dtype, "GENERAL", tg)["kernel"]
    return sv.plan_info(n, dtype, gate, tg, ct)["kernel"]


def touched_fraction(gate, nc):
    """Fraction of amplitudes a gate-specific kernel reads and writes."""
    if gate in ("X", "H", "RY", "RZ", "U2", "U4"):
        return 1.0 / (2 ** nc)
    if gate in ("Z", "SWAP"):
        return 0.5 / (2 ** nc)
    return 1.0


def line_fraction(gate, tg, ct, line_bits):
    """Fraction of the state's 128-byte lines holding an amplitude the gate
    touches (a line spans the lowest `line_bits` qubits): a constrained bit
    below the line size does not spare any line."""
    hi = [q for q in ct if q >= line_bits]
    f = 0.5 ** len(hi)
    if gate == "Z":
        f *= 0.5 if tg[0] >= line_bits else 1.0
    elif gate == "SWAP":
        f *= 0.5 if min(tg) >= line_bits else 1.0
    return f


def sweep_cases(n, rng, W):
    cases = []
    for t in range(n):
        for g in ("H", "X", "Z", "RZ", "RY", "U2"):
            p = (float(rng.uniform(0, 2 * math.pi)),) if g in ("RZ", "RY") else ()
            m = W.haar_unitary(1, rng) if g == "U2" else None
            cases.append((g, (t,), (), p, m))
        sec = W.second_qubit_choices(t, n)
        for c in sec:
            cases.append(("X", (t,), (c,), (), None))            # CNOT c -> t
            cases.append(("SWAP", (t, c), (), (), None))
            cases.append(("U4", (t, c), (), (), W.haar_unitary(2, rng)))
        for i in range(len(sec)):
            for j in range(i + 1, len(sec)):
                cases.append(("X", (t,), (sec[i], sec[j]), (), None))  # Toffoli
    return cases


def dense_of(case, oracle_free_matrix):
    """Dense matrix on (controls..., targets...) for the general kernel; built
    from the gate definitions in this file's own small table."""
    import numpy as np
    g, tg, ct, p, m = case
    r2 = math.sqrt(0.5)
    if g == "U2" or g == "U4":
        u = np.asarray(m, dtype=np.complex128)
    elif g == "X":
        u = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    elif g == "H":
        u = np.array([[r2, r2], [r2, -r2]], dtype=np.complex128)
    elif g == "Z":
        u = np.diag([1, -1]).astype(np.complex128)
    elif g == "RZ":
        u = np.diag([np.exp(-0.5j * p[0]), np.exp(0.5j * p[0])])
    elif g == "RY":
        c, s = math.cos(p[0] / 2), math.sin(p[0] / 2)
        u = np.array([[c, -s], [s, c]], dtype=np.complex128)
    elif g == "SWAP":
        u = np.eye(4, dtype=np.complex128)[[0, 2, 1, 3]]
    else:
        raise ValueError(g)
    k = len(ct)
    if k:
        # controlled-U on (controls..., targets...): identity except the last block
        d = 2 ** (k + len(tg))
        full = np.eye(d, dtype=np.complex128)
        full[d - u.shape[0]:, d - u.shape[0]:] = u
        u = full
    return tuple(ct) + tuple(tg), np.ascontiguousarray(u)


def run_sweep(sv, torch, state, cases, denses, timed, recs):
    """One step.  Appends one record per case to `recs` when timed:
    (name, specific kernel, general kernel, specific s, general s,
    algorithmic bytes, line-granular bytes, lowest touched qubit, target of a
    one-qubit gate or None), plus one ("expval", ...) record."""
    stream = torch.cuda.current_stream()
    ev = []
    for i, case in enumerate(cases):
        g, tg, ct, p, m = case
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        state.apply(g, tg, ct, p, m)
        e1.record(stream)
        qs, u = denses[i]
        state.apply_general(qs, u)
        e2.record(stream)
        ev.append((case, e0, e1, e2))
    e3 = torch.cuda.Event(enable_timing=True)
    e3.record(stream)
    zz = [(1.0, "ZZ", (q, q + 1)) for q in range(state.n - 1)]
    state.expval(zz)
    e4 = torch.cuda.Event(enable_timing=True)
    e4.record(stream)
    torch.cuda.synchronize()
    if not timed:
        return
    eb = 16 if state.dtype == "c128" else 8
    S = (1 << state.n) * eb
    lb = 3 if eb == 16 else 4  # qubits spanned by a 128-byte line
    for case, e0, e1, e2 in ev:
        g, tg, ct, p, m = case
        name = g if not ct else ({1: "CNOT", 2: "Toffoli"}[len(ct)] if g == "X" else g)
        qs = tuple(ct) + tuple(tg)
        recs.append((name, kernel_of(sv, g, tg, ct, n=state.n, dtype=state.dtype),
                     kernel_of(sv, g, qs, (), True, state.n, state.dtype), e0.elapsed_time(e1) * 1e-3,
                     e1.elapsed_time(e2) * 1e-3, 2 * S * touched_fraction(g, len(ct)),
                     2 * S * line_fraction(g, tg, ct, lb), min(qs), tg[0] if not ct and len(tg) == 1 else None))
    recs.append(("expval", "k_diag_obs_partial<%s>" % ("double" if eb == 16 else "float"), None,
                 e3.elapsed_time(e4) * 1e-3, 0.0, S, S, 0, None))


def summarize_sweep(recs, n, dtype, ceiling_gbps):
    """Whole-sweep, per class, per kernel and per target figures from
    run_sweep's records; GB/s are algorithmic, line_GBps line-granular."""
    eb = 16 if dtype == "c128" else 8
    lb = 3 if eb == 16 else 4
    S = (1 << n) * eb
    gates = [r for r in recs if r[0] != "expval"]
    t_spec = sum(r[3] for r in gates)
    t_gen = sum(r[4] for r in gates)
    tot = {"gates_per_s": len(gates) / t_spec, "effective_GBps": sum(r[5] for r in gates) / t_spec / 1e9,
           "line_GBps": sum(r[6] for r in gates) / t_spec / 1e9, "general_gates_per_s": len(gates) / t_gen}
    tot["effective_frac_of_8TBps"] = tot["effective_GBps"] / PEAK_GBPS
    tot["line_frac_of_8TBps"] = tot["line_GBps"] / PEAK_GBPS
    tot["effective_frac_of_ceiling"] = tot["effective_GBps"] / ceiling_gbps if ceiling_gbps else None
    per_class = {}
    for name in sorted({r[0] for r in gates}):
        rs = [r for r in gates if r[0] == name]
        ts, tg_ = sum(r[3] for r in rs), sum(r[4] for r in rs)
        bs, ls = sum(r[5] for r in rs), sum(r[6] for r in rs)
        d = {"specific": {"kernels": sorted({r[1] for r in rs}), "launches": len(rs), "avg_ms": 1e3 * ts / len(rs),
                          "GBps": bs / ts / 1e9, "frac_of_8TBps": bs / ts / 1e9 / PEAK_GBPS,
                          "line_GBps": ls / ts / 1e9},
             "general": {"kernels": sorted({r[2] for r in rs}), "launches": len(rs), "avg_ms": 1e3 * tg_ / len(rs),
                         "GBps": 2 * S * len(rs) / tg_ / 1e9, "frac_of_8TBps": 2 * S * len(rs) / tg_ / 1e9 / PEAK_GBPS}}
        d["speedup_specific_vs_general"] = tg_ / ts
        al = [r for r in rs if r[7] >= lb]
        if al and name in ("Z", "CNOT", "SWAP", "Toffoli"):
            ta, ba = sum(r[3] for r in al), sum(r[5] for r in al)
            d["specific_lowest_qubit_ge_line_bits"] = {"launches": len(al), "avg_ms": 1e3 * ta / len(al),
                                                        "GBps": ba / ta / 1e9, "frac_of_8TBps": ba / ta / 1e9 / PEAK_GBPS}
        per_class[name] = d
    by_kernel = {}
    for r in recs:
        for kern, t, byt in ((r[1], r[3], r[5]), (r[2], r[4], 2 * S)):
            if kern is None:
                continue
            a = by_kernel.setdefault(kern, [0.0, 0.0, 0])
            a[0] += t
            a[1] += byt
            a[2] += 1
    per_kernel = {k: {"launches": c, "avg_ms": 1e3 * t / c, "GBps": by / t / 1e9, "frac_of_8TBps": by / t / 1e9 / PEAK_GBPS,
                      "share_of_step_time": t / (t_spec + t_gen)}
                  for k, (t, by, c) in sorted(by_kernel.items(), key=lambda kv: -kv[1][0])}
    per_target = {}
    for r in gates:
        if r[8] is not None:
            per_target.setdefault(r[0], {}).setdefault(r[8], []).append((r[3], r[4]))
    per_target_ms = {g: {"specific": [round(1e3 * sum(x[0] for x in v[t]) / len(v[t]), 4) for t in sorted(v)],
                         "general": [round(1e3 * sum(x[1] for x in v[t]) / len(v[t]), 4) for t in sorted(v)]}
                     for g, v in per_target.items()}
    return tot, per_class, per_kernel, by_kernel, per_target_ms


def measure_ceiling(sv, torch, state):
    """The streaming kernel (sv_stream_bench) over the state's bytes: copy to
    a second buffer (bytes read + bytes written), read only, write only, and
    in place (read and write back, a full-touch gate's access pattern; run on
    the second buffer); best launch shape of a small set, median of 3 runs
    each.  `ceiling_GBps` is the in-place figure: the bound for a gate."""
    nbytes = state.tensor.numel() * state.tensor.element_size()
    other = torch.zeros_like(state.tensor)
    out = {"bytes": nbytes}
    for mode, label, factor in ((0, "copy", 2), (1, "read", 1), (2, "write", 1), (3, "inplace", 2)):
        best = None
        for block in (64, 128, 256, 512):
            for unroll in (1, 2, 4, 8):
                def run():
                    sv.stream_bench(mode, other if mode != 1 else None, state.tensor if mode in (0, 1) else None,
                                    nbytes, block, unroll)
                run()
                torch.cuda.synchronize()
                ts = []
                for _ in range(3):
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    run()
                    e1.record()
                    e1.synchronize()
                    ts.append(e0.elapsed_time(e1) * 1e-3)
                gbps = factor * nbytes / sorted(ts)[1] / 1e9
                if best is None or gbps > best[0]:
                    best = (gbps, block, unroll)
        out[f"{label}_GBps"] = best[0]
        out[f"{label}_shape"] = [best[1], best[2]]
    out["ceiling_GBps"] = out["inplace_GBps"]
    del other
    torch.cuda.empty_cache()
    return out


# The files the single-gate and reduction kernels are compiled from; the PMC
# summary records their hash, so a change to any of them voids its traffic.
SWEEP_KERNEL_SOURCES = ("k_gates.hip", "k_reduce.hip", "sv_core.h")


def kernel_sources_sha256():
    """SHA-256 over the sweep kernels' source files (file name + bytes, in
    the order above); the PMC summary records the value it was measured with."""
    import hashlib
    h = hashlib.sha256()
    for name in SWEEP_KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2508_13615_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_traffic(kernel, summary=PMC_SUMMARY):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC
    summary (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size), or
    None when there is no entry or the kernels changed since it was taken."""
    if not os.path.exists(summary):
        return None
    with open(summary) as f:
        text = f.read()
    a = text.find("```json")
    if a < 0:
        return None
    b = text.find("```", a + 7)
    blk = json.loads(text[a + 7:b])
    if blk.get("source_sha256") != kernel_sources_sha256():
        return None
    e = blk["kernels"].get(kernel)
    return None if e is None else e["traffic_bytes"]


def host_info():
    """CPU model, logical CPUs and memory of the host (from /proc)."""
    model, mem = None, None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                mem = round(int(line.split()[1]) / 2**20, 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "mem_GiB": mem}


def cpu_baseline(qubits_cpu, qubits_gpu, min_seconds=10.0):
    """The oracle on the host cores: X, H, RZ, CNOT, CZ and Toffoli at three
    targets on a Gaussian state, the list repeated until at least
    `min_seconds` of work has run; the rate is scaled to `qubits_gpu`
    (the oracle's work is linear in the amplitude count)."""
    import oracle
    import workloads as W
    psi = W.gaussian_state(qubits_cpu, 1001)
    sample = []
    ts = [0, qubits_cpu // 2, qubits_cpu - 1]
    for t in ts:
        c = 0 if t != 0 else qubits_cpu // 2
        c2 = qubits_cpu - 1 if t != qubits_cpu - 1 else qubits_cpu // 2
        sample += [("X", (t,), ()), ("H", (t,), ()), ("RZ", (t,), (), (0.7,)), ("X", (t,), (c,)),
                   ("Z", (t,), (c,)), ("X", (t,), (c, c2))]
    oracle.apply_gate(psi, "H", (1,))  # warm-up
    gates = 0
    t0 = time.perf_counter()
    while True:
        for s in sample:
            oracle.apply_gate(psi, s[0], s[1], s[2], s[3] if len(s) > 3 else ())
        gates += len(sample)
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    rate = gates / dt * 2.0 ** (qubits_cpu - qubits_gpu)
    scaled = ("" if qubits_cpu == qubits_gpu else
              f"; rate scaled by 2^{qubits_cpu - qubits_gpu} to {qubits_gpu} qubits (the oracle's work is linear "
              f"in the amplitude count)")
    return {"value": rate, "unit": "gates/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": (f"X, H, RZ, CNOT, CZ, Toffoli at t in {ts} on a {qubits_cpu}-qubit complex128 Gaussian state, "
                       f"{gates} gates in {dt:.1f} s{scaled}")}


def cpu_param_shift_estimate(n, layers):
    """One oracle forward pass + sum Z_i Z_{i+1} of the adjoint workload; the
    oracle's parameter-shift gradient would take 2 * params such runs."""
    import oracle
    import workloads as W
    ops = W.hea_ops(n, layers)
    th = W.uniform_angles(W.hea_n_params(n, layers), 1005)
    t0 = time.perf_counter()
    oracle.energy(n, ops, th, W.sum_zz(n))
    t = time.perf_counter() - t0
    runs = 2 * W.hea_n_params(n, layers)
    return {"forward_expval_s": t, "param_shift_runs": runs, "param_shift_s_extrapolated": t * runs,
            "cores": oracle.num_threads()}


GOLDEN = os.path.join(ROOT, "tests", "golden")


def golden_adjoint(n):
    """The oracle's stored gradients of the adjoint workload at n qubits
    (tests/golden/oracle_adjoint_hea.txt): energy, {j: parameter shift},
    {j: central difference}."""
    e, ps, fd = None, {}, {}
    path = os.path.join(GOLDEN, "oracle_adjoint_hea.txt")
    if not os.path.exists(path):
        return e, ps, fd
    with open(path) as f:
        for line in f:
            tok = line.split()
            if not tok or tok[0].startswith("#") or int(tok[1]) != n:
                continue
            if tok[0] == "energy":
                e = float(tok[2])
            else:
                (ps if tok[0] == "ps" else fd)[int(tok[2])] = float(tok[3])
    return e, ps, fd


def golden_circuits20():
    """The oracle's stored 20-qubit HEA and QFT results
    (tests/golden/oracle_circuits20.txt): {name: (energy, {index: amplitude})}."""
    out = {}
    with open(os.path.join(GOLDEN, "oracle_circuits20.txt")) as f:
        for line in f:
            tok = line.split()
            if not tok or tok[0].startswith("#"):
                continue
            e, amps = out.setdefault(tok[1], [None, {}])
            if tok[0] == "energy":
                out[tok[1]][0] = float(tok[2])
            else:
                amps[int(tok[2])] = complex(float(tok[3]), float(tok[4]))
    return out


def circuits20(sv, torch):
    """The 20-qubit HEA and QFT on the fused engine and on the op-by-op
    kernels, both dtypes, against the oracle's stored results: the error of
    every result per dtype (the complex64 precision form)."""
    import numpy as np
    import workloads as W
    n = 20
    ref = golden_circuits20()
    x = W.random_basis_index(n, 1004)
    prep = [W.Op("X", (), (q,)) for q in range(n) if (x >> q) & 1]
    jobs = {"hea": (W.hea_ops(n, 10), W.uniform_angles(W.hea_n_params(n, 10), 1003)),
            "qft": (prep + W.qft_ops(n), np.zeros(0))}
    out = {}
    for name, (ops, th) in jobs.items():
        e_ref, amps = ref[name]
        idx = np.array(sorted(amps))
        want = np.array([amps[i] for i in idx])
        for dt in ("c128", "c64"):
            b = sv.Batch([(n, ops, len(th), "sum_z")], dt, with_grad=False)
            e = float(b.run(th)[0][0])
            got = b.state(0)[idx].astype(np.complex128)
            del b
            st = sv.State(n, dt, basis=0)
            sv.Circuit(n, ops, len(th)).apply(st, th)
            e_op = st.expval(W.sum_z(n))
            got_op = st.numpy()[idx].astype(np.complex128)
            del st
            out[f"{name}_{dt}"] = {"engine_amp_err": float(np.max(np.abs(got - want))),
                                   "engine_energy_err": abs(e - e_ref),
                                   "op_by_op_amp_err": float(np.max(np.abs(got_op - want))),
                                   "op_by_op_energy_err": abs(e_op - e_ref)}
    torch.cuda.empty_cache()
    return out


def adjoint_compare(sv, torch, n, layers, ps_params, full_ps):
    import numpy as np
    import workloads as W
    ops = W.hea_ops(n, layers)
    npar = W.hea_n_params(n, layers)
    th = W.uniform_angles(npar, 1005)
    obs = W.sum_zz(n)
    out = {"qubits": n, "layers": layers, "params": npar, "ops": len(ops), "observable": "sum_i Z_i Z_{i+1}"}
    circ = sv.Circuit(n, ops, npar)
    grads = {}
    for dt in ("c128", "c64"):
        psi, lam = sv.State(n, dt), sv.State(n, dt)
        circ.adjoint_grad(psi, lam, th, obs)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        psi.set_basis(0)
        e, g = circ.adjoint_grad(psi, lam, th, obs)
        t_adj = time.perf_counter() - t0
        grads[dt] = (e, g)
        out[f"adjoint_s_{dt}"] = t_adj
        del psi, lam
    # parameter shift on the same GPU, same kernels: 2 forward+expval runs per parameter
    which = list(range(npar)) if full_ps else list(np.random.default_rng(1007).choice(npar, ps_params, replace=False))
    res = {}
    for dt in ("c128", "c64"):
        s = sv.State(n, dt)
        sobs = sv.Observable(obs)
        p = th.copy()
        s.set_basis(0)
        circ.apply(s, p)
        s.expval(sobs)  # warm-up
        torch.cuda.synchronize()
        gps = np.zeros(len(which))
        t0 = time.perf_counter()
        for i, j in enumerate(which):
            p[j] = th[j] + math.pi / 2
            s.set_basis(0)
            circ.apply(s, p)
            ep = s.expval(sobs)
            p[j] = th[j] - math.pi / 2
            s.set_basis(0)
            circ.apply(s, p)
            em = s.expval(sobs)
            p[j] = th[j]
            gps[i] = (ep - em) / 2
        t_ps = time.perf_counter() - t0
        res[dt] = gps
        out[f"param_shift_s_{dt}_measured"] = t_ps
        out[f"param_shift_s_{dt}"] = t_ps * npar / len(which)
        del s
    out["param_shift_params_timed"] = len(which)
    out["param_shift_extrapolated"] = len(which) != npar
    ref = res["c128"]
    e_or, ps_or, fd_or = golden_adjoint(n) if (n, layers) == (24, 8) else (None, {}, {})
    if ps_or:
        js = sorted(ps_or)
        g_or = np.array([ps_or[j] for j in js])
        g_fd = np.array([fd_or[j] for j in js])
        for dt in ("c128", "c64"):
            out[f"max_abs_err_adjoint_{dt}_vs_oracle_ps"] = float(np.max(np.abs(grads[dt][1][js] - g_or)))
            out[f"max_abs_err_adjoint_{dt}_vs_oracle_fd"] = float(np.max(np.abs(grads[dt][1][js] - g_fd)))
            out[f"abs_err_energy_{dt}_vs_oracle"] = abs(grads[dt][0] - e_or)
        out["oracle_params_checked"] = js
    out["max_abs_err_adjoint_c128_vs_ps_c128"] = float(np.max(np.abs(grads["c128"][1][which] - ref)))
    out["max_abs_err_adjoint_c64_vs_ps_c128"] = float(np.max(np.abs(grads["c64"][1][which] - ref)))
    out["max_abs_err_ps_c64_vs_ps_c128"] = float(np.max(np.abs(res["c64"] - ref)))
    out["expval_c128"] = grads["c128"][0]
    out["speedup_c128"] = out["param_shift_s_c128"] / out["adjoint_s_c128"]
    out["speedup_c64"] = out["param_shift_s_c64"] / out["adjoint_s_c64"]
    torch.cuda.empty_cache()
    return out


def _timed(torch, fn, reps=3):
    fn()  # warm-up (graph capture on first run)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2]


def adjoint_fused(sv, torch, n, layers, chunk):
    """Config 4 on the fused pass engine: one adjoint-gradient run against
    parameter shift with every shifted parameter set run as a batch of
    circuits (2 * params circuits, `chunk` per launch)."""
    import numpy as np
    import workloads as W
    ops = W.hea_ops(n, layers)
    npar = W.hea_n_params(n, layers)
    th = W.uniform_angles(npar, 1005)
    out = {"qubits": n, "layers": layers, "params": npar, "engine": "fused passes (sv_batch)"}
    grads = {}
    for dt in ("c128", "c64"):
        b = sv.Batch([(n, ops, npar, "sum_zz")], dt, with_grad=True)
        res = {}

        def run():
            res["eg"] = b.run(th)

        out[f"adjoint_s_{dt}"] = _timed(torch, run)
        grads[dt] = res["eg"]
        out[f"passes_{dt}"] = b.info()["passes"]
        del b
        torch.cuda.empty_cache()
        shifted = []
        for j in range(npar):
            for sgn in (1.0, -1.0):
                p = th.copy()
                p[j] += sgn * math.pi / 2
                shifted.append(p)
        bf = sv.Batch([(n, ops, npar, "sum_zz")] * chunk, dt, with_grad=False)
        bf.run(np.concatenate(shifted[:chunk]))  # capture
        torch.cuda.synchronize()
        es = []
        t0 = time.perf_counter()
        for k in range(0, len(shifted), chunk):
            part = shifted[k:k + chunk]
            while len(part) < chunk:
                part = part + [th]
            e, _ = bf.run(np.concatenate(part))
            es.extend(e[:min(chunk, len(shifted) - k)])
        out[f"param_shift_s_{dt}"] = time.perf_counter() - t0
        es = np.array(es)
        gps = (es[0::2] - es[1::2]) / 2.0
        out[f"max_abs_err_adjoint_vs_ps_{dt}"] = float(np.max(np.abs(grads[dt][1] - gps)))
        out[f"speedup_{dt}"] = out[f"param_shift_s_{dt}"] / out[f"adjoint_s_{dt}"]
        if dt == "c128":
            g_ref = gps
        del bf
        torch.cuda.empty_cache()
    out["param_shift_circuits"] = 2 * npar
    out["param_shift_circuits_per_launch"] = chunk
    out["max_abs_err_adjoint_c64_vs_ps_c128"] = float(np.max(np.abs(grads["c64"][1] - g_ref)))
    out["expval_c128"] = float(grads["c128"][0][0])
    return out


def config5(sv, torch, reps, sequential):
    """256 circuits, 14..22 qubits, 4..12 HEA layers, sum Z_i, forward +
    adjoint gradient in one graph launch; against the same circuits run one
    after another through the op-by-op path."""
    import numpy as np
    import workloads as W
    spec = W.batch_spec(256, 1006, 14, 22, 4, 12)
    circs = [(c.n, W.hea_ops(c.n, c.layers), len(c.params), "sum_z") for c in spec]
    params = np.concatenate([c.params for c in spec])
    out = {"circuits": len(spec), "qubits": "14..22", "layers": "4..12", "observable": "sum_i Z_i",
           "gates": int(sum(len(c[1]) for c in circs)), "params": int(len(params))}
    for dt in ("c128", "c64"):
        b = sv.Batch(circs, dt, with_grad=True)
        res = {}

        def run():
            res["eg"] = b.run(params)

        t = _timed(torch, run, reps)
        info = b.info()
        out[dt] = {"run_s": t, "circuits_per_s": len(spec) / t, "algorithmic_GBps": info["pass_bytes"] / t / 1e9,
                   "passes": info["passes"], "levels": info["levels"], "state_GB": info["state_bytes"] / 1e9}
        e_b, g_b = res["eg"]
        del b
        torch.cuda.empty_cache()
        if sequential:
            objs = [(sv.Circuit(c.n, W.hea_ops(c.n, c.layers), len(c.params)), sv.State(c.n, dt), sv.State(c.n, dt))
                    for c in spec]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            es, gs = [], []
            for (ci, psi, lam), c in zip(objs, spec):
                psi.set_basis(0)
                e1, g1 = ci.adjoint_grad(psi, lam, c.params, W.sum_z(c.n))
                es.append(e1)
                gs.append(g1)
            ts = time.perf_counter() - t0
            out[dt]["sequential_op_by_op_s"] = ts
            out[dt]["speedup_vs_sequential"] = ts / t
            out[dt]["max_abs_err_vs_sequential_grad"] = float(np.max(np.abs(g_b - np.concatenate(gs))))
            out[dt]["max_abs_err_vs_sequential_expval"] = float(np.max(np.abs(e_b - np.array(es))))
            del objs
            torch.cuda.empty_cache()
    return out


def circuit_jobs(n, layers):
    """(basis index of the QFT input, {name: (ops, params)}) of the circuits
    benchmark: HEA (layers of RY+RZ and a CNOT ladder), the QFT of a seeded
    basis state and the universal circuit after an H on every qubit."""
    import numpy as np
    import workloads as W
    x = W.random_basis_index(n, 1004)
    prep = [W.Op("X", (), (q,)) for q in range(n) if (x >> q) & 1]
    return x, {"hea": (W.hea_ops(n, layers), W.uniform_angles(W.hea_n_params(n, layers), 1003)),
               "qft": (prep + W.qft_ops(n), np.zeros(0)),
               "universal": ([W.Op("H", (), (q,)) for q in range(n)] + W.universal_ops(n), np.zeros(0))}


def config3(sv, torch, n, layers, reps, names=("hea", "qft", "universal"), engine_only=False):
    """32-qubit HEA (10 layers RY+RZ, CNOT ladder, from |0..0>), QFT of a
    random basis state and the universal circuit (2 n^2 gates after an H on
    every qubit), forward + sum Z on the fused engine, both dtypes; the same
    circuits as dense 5-qubit blocks on the matrix cores, and the QFT on the
    single-gate kernels with and without fused diagonal runs.  The
    complex64 error is taken against the complex128 GPU result (itself
    checked against the fp64 oracle at 20 qubits by the GPU tests)."""
    import workloads as W
    x, jobs = circuit_jobs(n, layers)
    jobs = {k: v for k, v in jobs.items() if k in names}
    out = {"qubits": n, "hea_layers": layers, "qft_basis_index": x}
    for name, (ops, th) in jobs.items():
        for dt in ("c128", "c64"):
            b = sv.Batch([(n, ops, len(th), "sum_z")], dt, with_grad=False)
            res = {}

            def run():
                res["e"] = b.run(th)[0][0]

            t = _timed(torch, run, reps)
            info = b.info()
            out[f"{name}_{dt}"] = {"s": t, "gates": len(ops), "gates_per_s": len(ops) / t, "passes": info["passes"],
                                   "algorithmic_GBps": info["pass_bytes"] / t / 1e9, "expval_sum_z": res["e"]}
            del b
            torch.cuda.empty_cache()
        out[f"{name}_abs_err_expval_c64_vs_c128"] = abs(out[f"{name}_c64"]["expval_sum_z"] - out[f"{name}_c128"]["expval_sum_z"])
    if engine_only:
        return out
    # the same circuits packed into 5-qubit dense blocks on the matrix cores
    for name, (ops, th) in jobs.items():
        circ = sv.Circuit(n, ops, len(th))
        plan = sv.block_plan(n, ops, 5)
        for dt in ("c128", "c64"):
            st = sv.State(n, dt, basis=0)

            def run():
                st.set_basis(0)
                circ.apply(st, th, dense_block=5)
                st.synchronize()
            t = _timed(torch, run, 1)
            out[f"{name}_{dt}"]["dense_blocks_k5_s"] = t
            out[f"{name}_{dt}"]["dense_blocks_k5"] = plan["dense_blocks"]
            log(f"[bench] {n}-qubit {name} {dt} as {plan['dense_blocks']} dense 5-qubit blocks: {t:.3f} s "
                f"(pass engine {out[f'{name}_{dt}']['s']:.3f} s)")
            del st
            torch.cuda.empty_cache()
    if "qft" not in jobs:
        return out
    # the same QFT on the single-gate kernels, op by op, and with each target's
    # H and controlled-phase run fused into one pass
    qft = sv.Circuit(n, W.qft_ops(n), 0)
    for dt in ("c128", "c64"):
        st = sv.State(n, dt, basis=x)
        r = {}
        for label, fuse in (("op_by_op_s", False), ("fused_diagonal_s", True)):
            def run():
                st.set_basis(x)
                qft.apply(st, [], fuse_diagonal=fuse)
                st.synchronize()
            r[label] = _timed(torch, run, 1)
        r["launches_op_by_op"] = len(W.qft_ops(n))
        r["launches_fused"] = n  # each H with the controlled-phase run after it
        r["speedup"] = r["op_by_op_s"] / r["fused_diagonal_s"]
        out[f"qft_single_gate_kernels_{dt}"] = r
        log(f"[bench] {n}-qubit QFT op by op {dt}: {r['op_by_op_s']:.3f} s, diagonal runs fused "
            f"{r['fused_diagonal_s']:.3f} s")
        del st
        torch.cuda.empty_cache()
    return out


def dense_block(sv, torch, W, n, gen, reps=5):
    """Dense k-qubit blocks (k = 4..6) on the matrix cores at n qubits, both
    dtypes: ms per block, HBM GB/s (2S moved) and achieved TFLOP/s (8 * 2^k
    flops per amplitude) against the dense matrix-core peak of the dtype, for
    targets at the bottom, the top and scattered over the index; beside it,
    the same Kronecker-product block as k one-qubit kernel launches."""
    import numpy as np
    peak = {"c128": 78.6, "c64": 157.3}  # TFLOP/s, dense FP64 / FP32 MFMA
    tdt = {"c128": torch.complex128, "c64": torch.complex64}
    rng = np.random.default_rng(1010)
    out = {}
    for dt in ("c128", "c64"):
        t = torch.randn(1 << n, dtype=tdt[dt], device="cuda", generator=gen)
        t /= torch.linalg.vector_norm(t)
        st = sv.State(n, dt, tensor=t, basis=None)
        S = (1 << n) * (16 if dt == "c128" else 8)
        res = {}
        for k in (4, 5, 6):
            us = [W.haar_unitary(1, rng) for _ in range(k)]
            big = us[0]
            for u in us[1:]:
                big = np.kron(big, u)
            placements = {"low": tuple(range(k - 1, -1, -1)), "high": tuple(range(n - 1, n - 1 - k, -1)),
                          "scattered": tuple(int(q) for q in rng.permutation(n)[:k])}
            rk = {}
            for name, tg in placements.items():
                def run_block():
                    st.apply_dense(tg, big)

                def run_gates():
                    for q, u in zip(tg, us):
                        st.apply("U2", (q,), matrix=u)
                ms = {}
                for label, fn in (("block", run_block), ("one_qubit_gates", run_gates)):
                    fn()
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(reps):
                        fn()
                    e1.record()
                    e1.synchronize()
                    ms[label] = e0.elapsed_time(e1) / reps
                tflops = 8 * (1 << k) * (1 << n) / (ms["block"] * 1e-3) / 1e12
                rk[name] = {"targets": list(tg), "ms": ms["block"], "GBps": 2 * S / (ms["block"] * 1e-3) / 1e9,
                            "frac_of_8TBps": 2 * S / (ms["block"] * 1e-3) / 8e12, "TFLOPs": tflops,
                            "frac_of_mfma_peak": tflops / peak[dt], "one_qubit_gates_ms": ms["one_qubit_gates"]}
            res[f"k{k}"] = rk
            log(f"[bench] dense {dt} k={k}: " + ", ".join(f"{nm} {v['ms']:.2f} ms ({v['TFLOPs']:.1f} TF/s, "
                                                            f"{v['GBps']:.0f} GB/s)" for nm, v in rk.items()))
        out[dt] = res
        del st, t
        torch.cuda.empty_cache()
    return out


def _r(x, nd=4):
    """Round for the headline line (None passes through)."""
    return None if x is None else float(f"{x:.{nd}g}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--qubits", type=int, default=30)
    ap.add_argument("--cpu-qubits", type=int, default=30)
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--skip-c64-sweep", action="store_true", help="skip the secondary complex64 sweep (one step)")
    ap.add_argument("--skip-adjoint", action="store_true")
    ap.add_argument("--adjoint-qubits", type=int, default=24)
    ap.add_argument("--adjoint-layers", type=int, default=8)
    ap.add_argument("--ps-params", type=int, default=48, help="parameters timed with parameter shift")
    ap.add_argument("--full-param-shift", action="store_true")
    ap.add_argument("--skip-fused", action="store_true", help="skip configs 3, 4 (fused) and 5")
    ap.add_argument("--config3-qubits", type=int, default=32)
    ap.add_argument("--no-sequential", action="store_true", help="skip the op-by-op baseline of config 5")
    ap.add_argument("--skip-dense", action="store_true", help="skip the matrix-core dense-block section")
    ap.add_argument("--detail", default=os.path.join(ROOT, "gpurun_out", "bench_detail.json"),
                    help="where the full results go (the stdout line is the headline only)")
    ap.add_argument("--only", default="",
                    help="comma list of sections to run alone (profiling runs): sweep, c64, adjoint, adjoint_fused, "
                         "batch, circuits32, circuits20, dense, cpu")
    ap.add_argument("--circuits", default="hea,qft,universal", help="circuits of the circuits32 section")
    ap.add_argument("--engine-only", action="store_true",
                    help="circuits32: the pass engine only (no dense blocks, no single-gate QFT)")
    args = ap.parse_args()
    only = {x for x in args.only.split(",") if x}
    known = {"sweep", "c64", "adjoint", "adjoint_fused", "batch", "circuits32", "circuits20", "dense", "cpu"}
    if only - known:
        ap.error(f"unknown sections {sorted(only - known)}")

    def want(section, skipped=False):
        return section in only if only else not skipped
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the state-vector path here is built and measured on a single "
              "MI355X (the multi-GPU sharding is a design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2508_13615_amd as sv
    import workloads as W

    torch.cuda.set_device(0)
    n = args.qubits
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1001)
    rng = np.random.default_rng(1002)
    cases = sweep_cases(n, rng, W)
    denses = [dense_of(c, None) for c in cases]
    head = {"metric": METRIC, "value": None, "unit": "gates/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    detail = {}
    if want("sweep"):
        log(f"[bench] {n}-qubit complex128 state ({(1 << n) * 16 / 2**30:.1f} GiB)")
        t = torch.randn(1 << n, dtype=torch.complex128, device="cuda", generator=gen)
        t /= torch.linalg.vector_norm(t)
        state = sv.State(n, "c128", tensor=t, basis=None)
        ceiling = measure_ceiling(sv, torch, state)
        log(f"[bench] {len(cases)} gate cases per step; streaming kernel: in place {ceiling['inplace_GBps']:.0f}, copy "
            f"{ceiling['copy_GBps']:.0f}, read {ceiling['read_GBps']:.0f}, write {ceiling['write_GBps']:.0f} GB/s")

        recs = []
        for w in range(args.warmup):
            run_sweep(sv, torch, state, cases, denses, False, recs)
        log(f"[bench] {args.warmup} warm-up steps done")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            run_sweep(sv, torch, state, cases, denses, True, recs)
            if (k + 1) % 5 == 0 or k + 1 == args.steps:
                log(f"[bench] step {k + 1}/{args.steps} done")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        norm = state.norm2()

        tot, per_class, per_kernel, by_kernel, per_target_ms = summarize_sweep(recs, n, "c128", ceiling["ceiling_GBps"])
        # dominant kernel: the instantiation with the largest total time
        dk, (dt_, db, dc) = max(by_kernel.items(), key=lambda kv: kv[1][0])
        achieved = db / dt_ / 1e9
        roof = {"bound": "hbm", "achieved": _r(achieved, 5), "peak": PEAK_GBPS, "unit": "GB/s",
                "frac": _r(achieved / PEAK_GBPS), "traffic": pmc_traffic(dk), "kernel": dk, "launches": dc,
                "avg_launch_ms": _r(1e3 * dt_ / dc, 5), "algorithmic_bytes_per_launch": db / dc,
                "frac_of_streaming_ceiling": _r(achieved / ceiling["ceiling_GBps"])}
        if roof["traffic"] is not None:
            roof["traffic_over_algorithmic"] = _r(roof["traffic"] / roof["algorithmic_bytes_per_launch"])
        detail.update({"sweep": {"totals": tot, "per_class": per_class, "per_kernel": per_kernel,
                                 "per_target_ms": per_target_ms, "norm_after": norm, "tuned_entries": sv.TUNED_ENTRIES},
                       "ceiling": ceiling})
        head = {
            "metric": METRIC,
            "value": _r(tot["gates_per_s"], 6),
            "unit": "gates/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": _r(1e3 * wall / args.steps, 6),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"single-gate sweep, {n} qubits complex128 (seeded Gaussian state), gate-specific "
                                   f"and general kernels", "qubits": n, "cases_per_step": len(cases),
                       "second_qubits": [0, n // 2, n - 1]},
            "roofline": roof,
            "effective_GBps": _r(tot["effective_GBps"]),
            "effective_frac_of_8TBps": _r(tot["effective_frac_of_8TBps"]),
            "line_GBps": _r(tot["line_GBps"]),
            "general_gates_per_s": _r(tot["general_gates_per_s"]),
            "ceiling_GBps": {k: _r(ceiling[f"{k}_GBps"]) for k in ("inplace", "copy", "read", "write")},
            # per class: [gate-specific, general] as fractions of 8 TB/s
            "classes_frac": {k: [_r(v["specific"]["frac_of_8TBps"], 3), _r(v["general"]["frac_of_8TBps"], 3)]
                             for k, v in per_class.items()},
            "partial_touch_lowest_qubit_ge3_frac": {k: _r(v["specific_lowest_qubit_ge_line_bits"]["frac_of_8TBps"], 3)
                                                    for k, v in per_class.items()
                                                    if "specific_lowest_qubit_ge_line_bits" in v},
        }
        del state, t
        torch.cuda.empty_cache()
    head["detail"] = os.path.relpath(args.detail, ROOT)
    if want("c64", args.skip_c64_sweep):
        log(f"[bench] complex64 sweep, {n} qubits, one step after one warm-up")
        t = torch.randn(1 << n, dtype=torch.complex64, device="cuda", generator=gen)
        t /= torch.linalg.vector_norm(t)
        st64 = sv.State(n, "c64", tensor=t, basis=None)
        r64 = []
        run_sweep(sv, torch, st64, cases, denses, False, r64)
        run_sweep(sv, torch, st64, cases, denses, True, r64)
        tot64, pc64, pk64, _, pt64 = summarize_sweep(r64, n, "c64", None)
        detail["sweep_c64"] = {"totals": tot64, "per_class": pc64, "per_kernel": pk64, "per_target_ms": pt64}
        head["sweep_c64"] = {"gates_per_s": _r(tot64["gates_per_s"]), "frac": _r(tot64["effective_frac_of_8TBps"]),
                             "classes_frac": {k: _r(v["specific"]["frac_of_8TBps"], 3) for k, v in pc64.items()}}
        del st64, t
        torch.cuda.empty_cache()
    if want("adjoint", args.skip_adjoint):
        log(f"[bench] adjoint vs parameter shift at {args.adjoint_qubits} qubits")
        a = adjoint_compare(sv, torch, args.adjoint_qubits, args.adjoint_layers, args.ps_params, args.full_param_shift)
        detail["adjoint"] = a
        head["adjoint"] = {k: _r(a.get(k)) for k in (
            "adjoint_s_c128", "param_shift_s_c128", "speedup_c128", "adjoint_s_c64", "param_shift_s_c64",
            "speedup_c64", "max_abs_err_adjoint_c128_vs_oracle_ps", "max_abs_err_adjoint_c64_vs_oracle_ps",
            "max_abs_err_adjoint_c128_vs_oracle_fd")}
    if want("adjoint_fused", args.skip_fused):
        log("[bench] adjoint workload on the fused engine")
        a = adjoint_fused(sv, torch, args.adjoint_qubits, args.adjoint_layers, 128)
        detail["adjoint_fused"] = a
        head["adjoint_fused"] = {k: _r(a.get(k)) for k in ("adjoint_s_c128", "adjoint_s_c64", "speedup_c128",
                                                            "speedup_c64")}
    if want("batch", args.skip_fused):
        log("[bench] 256 mixed circuits in one graph launch")
        bt = config5(sv, torch, 3, not args.no_sequential)
        detail["batch"] = bt
        head["batch"] = {dt: {"s": _r(bt[dt]["run_s"]), "speedup_vs_sequential": _r(bt[dt].get("speedup_vs_sequential"))}
                         for dt in ("c128", "c64")}
    if want("circuits32", args.skip_fused):
        log(f"[bench] {args.config3_qubits}-qubit circuits")
        names = tuple(x for x in args.circuits.split(",") if x)
        c3 = config3(sv, torch, args.config3_qubits, 10, 3, names, args.engine_only)
        detail["circuits32"] = c3
        head["circuits32_s"] = {f"{nm}_{dt}": _r(c3[f"{nm}_{dt}"]["s"]) for nm in names for dt in ("c128", "c64")}
        if "qft_single_gate_kernels_c128" in c3:
            head["circuits32_s"]["qft_fused_diagonal_c128"] = _r(c3["qft_single_gate_kernels_c128"]["fused_diagonal_s"])
    if want("circuits20", args.skip_fused):
        log("[bench] 20-qubit circuits against the oracle's stored results")
        c20 = circuits20(sv, torch)
        detail["circuits20"] = c20
        head["circuits20_err"] = {k: [_r(v["engine_amp_err"], 2), _r(v["op_by_op_amp_err"], 2)] for k, v in c20.items()}
    if want("dense", args.skip_dense):
        log(f"[bench] dense 4- to 6-qubit blocks on the matrix cores at {n} qubits")
        detail["dense_block"] = dense_block(sv, torch, W, n, gen)
    if want("cpu", args.skip_cpu_baseline):
        log(f"[bench] oracle CPU baseline at {args.cpu_qubits} qubits")
        cb = cpu_baseline(args.cpu_qubits, n)
        cb["host"] = host_info()
        # the same oracle on one host thread (separate process: OpenMP's thread
        # count is fixed when the oracle library loads), on a 24-qubit sample
        import subprocess
        r = subprocess.run([sys.executable, "-c", "import json, bench; print(json.dumps(bench.cpu_baseline(24, %d, 5.0)))" % n],
                           cwd=ROOT, env=dict(os.environ, OMP_NUM_THREADS="1"), capture_output=True, text=True)
        if r.returncode == 0:
            one = json.loads(r.stdout.strip().splitlines()[-1])
            cb["single_thread_gates_per_s"] = _r(one["value"])
        if want("adjoint", args.skip_adjoint) or only:
            cps = cpu_param_shift_estimate(args.adjoint_qubits, args.adjoint_layers)
            cb["oracle_param_shift_24q_s"] = _r(cps["param_shift_s_extrapolated"])
            detail["cpu_param_shift"] = cps
        detail["cpu_baseline"] = cb
        head["cpu_baseline"] = dict(cb, value=_r(cb["value"]))
    os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
    with open(args.detail, "w") as f:
        json.dump(detail, f, indent=1)
    print(json.dumps(head, separators=(",", ":")), flush=True)


if __name__ == "__main__":
    main()
