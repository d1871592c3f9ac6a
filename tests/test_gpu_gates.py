"""GPU parity: libsv's HIP kernels against the oracle, element by element.

Bars: permutation gates (X / CNOT / Toffoli / SWAP) bit-exact in both dtypes;
complex128 amplitudes within 1e-12 max-abs of the fp64 oracle; complex64
amplitudes within 1e-5 max-abs of the fp64 oracle run on the same (rounded)
input.
"""
import itertools
import math
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

sv = pytest.importorskip("paper_2508_13615_amd")

TOL = {"c128": 1e-12, "c64": 1e-5}
NP_DT = {"c128": np.complex128, "c64": np.complex64}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_native_library_is_loaded():
    maps = open("/proc/self/maps").read()
    assert "paper_2508_13615_amd/libsv.so" in maps


def _oracle_apply(psi_in, case):
    """Oracle result for one gate case; permutation gates move elements of the
    state's own dtype, everything else runs in fp64 on the (upcast) input."""
    if case.gate in ("X", "SWAP"):
        out = psi_in.copy()
        return oracle.apply_gate(out, case.gate, case.targets, case.controls)
    out = psi_in.astype(np.complex128)
    return oracle.apply_gate(out, case.gate, case.targets, case.controls, case.params, case.matrix)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_sweep_every_gate_every_index_12q(dtype):
    n = 12
    log(f"sweep n={n} dtype={dtype}")
    psi0 = W.gaussian_state(n, 1001).astype(NP_DT[dtype])
    base = sv.State(n, dtype).load(psi0)
    work = sv.State(n, dtype)
    worst = {}
    for case in W.sweep_cases(n, 1002):
        work.copy_from(base)
        work.apply(case.gate, case.targets, case.controls, case.params, case.matrix)
        got = work.numpy()
        ref = _oracle_apply(psi0, case)
        key = (case.gate, len(case.controls))
        if case.gate in ("X", "SWAP"):
            assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), case[:3]
        else:
            err = float(np.max(np.abs(got.astype(np.complex128) - ref)))
            worst[key] = max(worst.get(key, 0.0), err)
            assert err <= TOL[dtype], (case[:3], err)
    log("worst error per (gate, controls):", {k: f"{v:.2e}" for k, v in sorted(worst.items())})


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_general_kernel_vs_oracle(dtype):
    n = 10
    rng = np.random.default_rng(2001)
    psi0 = W.gaussian_state(n, 2002).astype(NP_DT[dtype])
    base = sv.State(n, dtype).load(psi0)
    work = sv.State(n, dtype)
    for k in (1, 2, 3):
        for _ in range(12):
            qs = tuple(int(q) for q in rng.permutation(n)[:k])
            u = W.haar_unitary(k, rng)
            work.copy_from(base).apply_general(qs, u)
            ref = oracle.apply_matrix(psi0.astype(np.complex128), qs, u)
            err = float(np.max(np.abs(work.numpy().astype(np.complex128) - ref)))
            assert err <= TOL[dtype], (k, qs, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_lds_staged_gate_every_launch_shape(dtype):
    """Every launch shape the tuner may pick for the LDS-staged kernel (block,
    lines staged per thread, non-temporal or not) on gates with a qubit
    below the 1 KiB run: dense 2- and 3-qubit matrices, U4 with and without
    controls below and above the 256-amplitude chunk, and the SWAP move, with
    0 to 2 gate qubits above the chunk, against the oracle (SWAP
    bit-exact).  The launch table is restored after."""
    n = 13
    rng = np.random.default_rng(2010)
    psi0 = W.gaussian_state(n, 2011).astype(NP_DT[dtype])
    base = sv.State(n, dtype).load(psi0)
    work = sv.State(n, dtype)
    ref_in = psi0.astype(np.complex128)
    cases = []
    for qs in [(0, 3), (12, 0), (2, 9), (1, 2, 5), (0, 12, 8), (11, 4, 10)]:
        cases.append(("GENERAL", qs, (), W.haar_unitary(len(qs), rng)))
    cases += [("U4", (12, 1), (), W.haar_unitary(2, rng)), ("U4", (1, 12), (5,), W.haar_unitary(2, rng)),
              ("U4", (0, 4), (9, 11), W.haar_unitary(2, rng)), ("SWAP", (0, 11), (), None),
              ("SWAP", (4, 2), (), None), ("SWAP", (1, 3), (12,), None)]
    hit = set()
    for g, qs, ct, m in cases:
        info = sv.plan_info(n, dtype, g, qs, ct)
        if info["class"] == 6:
            hit.add((len(qs), info["op"] & 15))
    assert {(2, 0), (3, 0), (2, 1)} <= hit, hit
    saved = {t: sv.tune_get(6, dtype, t) for t in range(3)}
    try:
        for block in (64, 128, 256, 512):
            for unroll in (1, 2, 4):
                for nt in (0, 1):
                    for t in range(3):
                        sv.tune_set(6, dtype, t, block, unroll, nt)
                    for g, qs, ct, m in cases:
                        work.copy_from(base)
                        if g == "GENERAL":
                            work.apply_general(qs, m)
                            ref = oracle.apply_matrix(ref_in.copy(), qs, m)
                        elif g == "SWAP":
                            work.apply("SWAP", qs, ct)
                            ref = oracle.apply_gate(psi0.copy(), "SWAP", qs, ct)
                        else:
                            work.apply(g, qs, ct, matrix=m)
                            ref = oracle.apply_gate(ref_in.copy(), g, qs, ct, (), m)
                        got = work.numpy()
                        if g == "SWAP":
                            assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), (block, unroll, nt, qs)
                        else:
                            err = float(np.max(np.abs(got.astype(np.complex128) - ref)))
                            assert err <= TOL[dtype], (block, unroll, nt, g, qs, err)
                log(f"lds {dtype}: block {block} shapes ok")
    finally:
        for t, shp in saved.items():
            sv.tune_set(6, dtype, t, *shp)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_block_orders_agree_and_match_oracle(dtype):
    """Both workgroup walk orders (launch order; one contiguous eighth of the
    grid per XCD) on every gate form at 7 and 12 qubits: the results must be
    bit-identical to each other (each group is still touched once with the
    same arithmetic) and within the bar of the oracle.  Launch shapes of 192
    threads make grids that are not multiples of 8, and the 7-qubit state has
    grids under 8 workgroups.  Settings are restored after."""
    classes = (0, 1, 3, 4, 5, 6)
    saved_order = sv.get_block_order()
    saved = {(kc, t): sv.tune_get(kc, dtype, t) for kc in classes for t in range(3)}
    rng = np.random.default_rng(2020)
    try:
        for n in (7, 12):
            psi0 = W.gaussian_state(n, 2021 + n).astype(NP_DT[dtype])
            base = sv.State(n, dtype).load(psi0)
            work = sv.State(n, dtype)
            # every case at 7 qubits; at 12, every seventh Toffoli
            cases = [(c.gate, c.targets, c.controls, c.params, c.matrix)
                     for i, c in enumerate(W.sweep_cases(n, 2030 + n))
                     if n == 7 or len(c.controls) < 2 or i % 7 == 0]
            for k in (1, 2, 3):
                cases.append(("GENERAL", tuple(int(q) for q in rng.permutation(n)[:k]), (), (),
                              W.haar_unitary(k, rng)))
            for shape in ((64, 1, 1), (192, 2, 0)):
                for kc in classes:
                    for t in range(3):
                        sv.tune_set(kc, dtype, t, *shape)
                outs = {}
                for order in (0, 1):
                    sv.set_block_order(order)
                    res = []
                    for g, tg, ct, p, m in cases:
                        work.copy_from(base)
                        if g == "GENERAL":
                            work.apply_general(tg, m)
                        else:
                            work.apply(g, tg, ct, p, m)
                        res.append(work.numpy())
                    outs[order] = res
                for i, (g, tg, ct, p, m) in enumerate(cases):
                    a, b = outs[0][i], outs[1][i]
                    assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (n, shape, g, tg, ct)
                    if g == "GENERAL":
                        ref = oracle.apply_matrix(psi0.astype(np.complex128), tg, m)
                    else:
                        ref = _oracle_apply(psi0, W.GateCase(g, ct, tg, p, m))
                    err = float(np.max(np.abs(b.astype(np.complex128) - ref.astype(np.complex128))))
                    assert err <= TOL[dtype], (n, shape, g, tg, ct, err)
                log(f"block orders {dtype} n={n} shape={shape}: {len(cases)} cases agree")
    finally:
        sv.set_block_order(saved_order)
        for (kc, t), shp in saved.items():
            sv.tune_set(kc, dtype, t, *shp)


def test_general_kernel_equals_specific_for_permutations():
    # Sec. 3.1 "general approach": CNOT as a 4x4 and Toffoli as an 8x8 dense
    # matrix give the same state as the dedicated move kernels (products with
    # exact 0 and 1 entries are exact for finite non-zero amplitudes).
    n = 9
    psi0 = W.gaussian_state(n, 2003)
    cnot = np.eye(4, dtype=np.complex128)[[0, 1, 3, 2]]
    tof = np.eye(8, dtype=np.complex128)[[0, 1, 2, 3, 4, 5, 7, 6]]
    a = sv.State(n).load(psi0)
    b = sv.State(n).load(psi0)
    for c, t in [(0, 1), (5, 2), (8, 0)]:
        a.apply("X", (t,), (c,))
        b.apply_general((c, t), cnot)
    for c1, c2, t in [(0, 1, 2), (7, 3, 5)]:
        a.apply("X", (t,), (c1, c2))
        b.apply_general((c1, c2, t), tof)
    assert np.array_equal(a.numpy(), b.numpy())


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_flag_inverts_every_gate(dtype):
    n = 7
    rng = np.random.default_rng(2004)
    psi0 = W.gaussian_state(n, 2005).astype(NP_DT[dtype])
    s = sv.State(n, dtype).load(psi0)
    for g in ["X", "Y", "Z", "H", "S", "T", "RX", "RY", "RZ", "PHASE", "U2", "U4", "SWAP"]:
        nt = 2 if g in ("U4", "SWAP") else 1
        qs = [int(q) for q in rng.permutation(n)]
        tg, ct = tuple(qs[:nt]), tuple(qs[nt:nt + int(rng.integers(0, 3))])
        p = (float(rng.uniform(0, 6.28)),)
        m = W.haar_unitary(nt, rng) if g in ("U2", "U4") else None
        s.apply(g, tg, ct, p, m)
        s.apply(g, tg, ct, p, m, adjoint=True)
    err = float(np.max(np.abs(s.numpy().astype(np.complex128) - psi0.astype(np.complex128))))
    assert err <= 10 * TOL[dtype], err


def test_ghz_bit_exact_closed_form():
    n = 16
    s = sv.State(n)
    for op in W.ghz_ops(n):
        s.apply(op.gate, op.targets, op.controls)
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[0] = ref[-1] = math.sqrt(0.5)
    assert np.array_equal(s.numpy(), ref)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_qft_basis_state_closed_form(dtype):
    n = 14
    x = W.random_basis_index(n, 1004)
    s = sv.State(n, dtype, basis=x)
    for op in W.qft_ops(n):
        s.apply(op.gate, op.targets, op.controls, (op.value,))
    y = np.arange(1 << n, dtype=np.int64)
    rev = np.zeros_like(y)
    for b in range(n):
        rev |= ((y >> b) & 1) << (n - 1 - b)
    m = (x * rev) % (1 << n)
    ref = np.exp(2j * np.pi * m / (1 << n)) * 2.0 ** (-n / 2)
    err = float(np.max(np.abs(s.numpy().astype(np.complex128) - ref)))
    assert err <= (1e-12 if dtype == "c128" else 1e-5), err


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_random_circuits_vs_oracle(dtype):
    rng = np.random.default_rng(2006)
    gates = ["X", "Y", "Z", "H", "S", "T", "RX", "RY", "RZ", "PHASE", "U2", "U4", "SWAP"]
    for n in (1, 2, 3, 5, 9, 16):
        psi0 = W.gaussian_state(n, 2007 + n).astype(NP_DT[dtype])
        s = sv.State(n, dtype).load(psi0)
        ref = psi0.astype(np.complex128)
        for _ in range(40):
            g = str(rng.choice(gates))
            nt = 2 if g in ("U4", "SWAP") else 1
            if nt > n:
                continue
            qs = [int(q) for q in rng.permutation(n)]
            nc = int(rng.integers(0, min(3, n - nt) + 1))
            tg, ct = tuple(qs[:nt]), tuple(qs[nt:nt + nc])
            p = (float(rng.uniform(0, 2 * math.pi)),)
            m = W.haar_unitary(nt, rng) if g in ("U2", "U4") else None
            s.apply(g, tg, ct, p, m)
            oracle.apply_gate(ref, g, tg, ct, p, m)
        err = float(np.max(np.abs(s.numpy().astype(np.complex128) - ref)))
        assert err <= 4 * TOL[dtype], (n, err)


def test_edge_cases_tiny_states_and_many_controls():
    # 1-qubit state; a gate whose group count (1) is far below one block; eight controls
    for dtype in ("c128", "c64"):
        s = sv.State(1, dtype)
        s.apply("H", (0,))
        assert np.allclose(s.numpy(), [math.sqrt(0.5), math.sqrt(0.5)], atol=TOL[dtype])
    n = 10
    psi0 = W.gaussian_state(n, 2010)
    s = sv.State(n).load(psi0)
    ctl = tuple(range(1, 9))
    s.apply("X", (0,), ctl)
    ref = oracle.apply_gate(psi0.copy(), "X", (0,), ctl)
    assert np.array_equal(s.numpy(), ref)
    u = W.haar_unitary(1, np.random.default_rng(1))
    s.apply("U2", (9,), ctl, (), u)
    oracle.apply_gate(ref, "U2", (9,), ctl, (), u)
    assert np.max(np.abs(s.numpy() - ref)) <= TOL["c128"]
    s.apply("I", (3,))
    assert np.max(np.abs(s.numpy() - ref)) <= TOL["c128"]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_norm_and_pauli_expectations(dtype):
    n = 11
    rng = np.random.default_rng(2011)
    psi0 = W.gaussian_state(n, 2012).astype(NP_DT[dtype])
    ref_state = psi0.astype(np.complex128)
    s = sv.State(n, dtype).load(psi0)
    assert abs(s.norm2() - oracle.norm2(ref_state)) <= (1e-13 if dtype == "c128" else 1e-6)
    for _ in range(30):
        k = int(rng.integers(1, n + 1))
        qs = tuple(int(q) for q in rng.permutation(n)[:k])
        ps = "".join(rng.choice(list("IXYZ"), size=k))
        e = s.expval_pauli(ps, qs)
        r = oracle.expval_pauli(ref_state, ps, qs).real
        assert abs(e - r) <= 1e-13, (ps, qs, e, r)  # fp64 accumulation in both dtypes
    # repeated calls are bit-identical (fixed-order reduction)
    assert s.expval_pauli("XYZ", (0, 5, 9)) == s.expval_pauli("XYZ", (0, 5, 9))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_observable_sums(dtype):
    n = 12
    rng = np.random.default_rng(2013)
    psi0 = W.gaussian_state(n, 2014).astype(NP_DT[dtype])
    ref_state = psi0.astype(np.complex128)
    s = sv.State(n, dtype).load(psi0)
    mixed = [(float(rng.normal()), "".join(rng.choice(list("XYZ"), size=3)),
              tuple(int(q) for q in rng.permutation(n)[:3])) for _ in range(12)]
    mixed += [(0.7, "ZZ", (1, 4)), (-1.3, "Z", (7,))]
    many_diag = [(float(rng.normal()), "Z" * 2, (i, (i + 3) % n)) for i in range(n)] * 4  # > 32 diagonal terms
    for terms in (W.sum_z(n), W.sum_zz(n), mixed, many_diag, [(2.5, "ZZ", (q, q + 1)) for q in range(n - 1)]):
        e = s.expval(terms)
        r = oracle.expval_obs(ref_state, terms)
        assert abs(e - r) <= 1e-12 * max(1, len(terms)), (e, r)
    assert s.expval([]) == 0.0


def test_expval_dev_output():
    import torch
    n = 9
    s = sv.State(n).load(W.gaussian_state(n, 2015))
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.expval_dev(W.sum_zz(n), out)
    torch.cuda.synchronize()
    assert out.item() == s.expval(W.sum_zz(n))


def test_full_size_sampled_parity_30q():
    """30-qubit complex128 state (16 GiB) in the benchmark's launch shapes:
    sampled groups are read before and after each gate and compared with the
    oracle applied to the same groups."""
    import torch
    n = 30
    log("full-size parity: allocating 30-qubit complex128 state")
    g = torch.Generator(device="cuda")
    g.manual_seed(1001)
    t = torch.randn(1 << n, dtype=torch.complex128, device="cuda", generator=g)
    t /= torch.linalg.vector_norm(t)
    s = sv.State(n, "c128", tensor=t, basis=None)
    rng = np.random.default_rng(3001)
    cases = [("X", (0,), ()), ("X", (29,), (15,)), ("H", (0,), ()), ("H", (17,), ()), ("RY", (29,), ()),
             ("Z", (3,), ()), ("RZ", (12,), ()), ("PHASE", (29,), (0,)), ("SWAP", (2, 28), ()),
             ("X", (15,), (0, 29)), ("U2", (6,), ()), ("U4", (29, 1), ())]
    for gate, tg, ct in cases:
        log("  case", gate, tg, ct)
        p = (float(rng.uniform(0, 2 * math.pi)),)
        m = W.haar_unitary(len(tg), rng) if gate in ("U2", "U4") else None
        qs = list(ct) + list(tg)
        # sample 512 groups: random indices with the gate's qubits cleared, controls set
        free = rng.integers(0, 1 << n, size=512, dtype=np.int64)
        for q in qs:
            free &= ~(1 << q)
        for q in ct:
            free |= 1 << q
        members = []
        for r in range(1 << len(tg)):
            off = 0
            for j, q in enumerate(tg):
                if (r >> (len(tg) - 1 - j)) & 1:
                    off |= 1 << q
            members.append(free | off)
        idx = torch.from_numpy(np.stack(members, axis=1).reshape(-1)).cuda()
        before = t[idx].cpu().numpy().reshape(512, -1)
        s.apply(gate, tg, ct, p, m)
        after = t[idx].cpu().numpy().reshape(512, -1)
        u = oracle.gate_matrix(gate, p, m)
        for row in range(512):
            mini = before[row].copy()
            k = len(tg)
            # oracle on a k-qubit mini-state: member r has first target as MSB
            if gate in ("X", "SWAP"):
                ref = oracle.apply_gate(mini, gate, tuple(range(k - 1, -1, -1)), ())
                assert np.array_equal(after[row], ref), (gate, tg, ct, row)
            else:
                ref = oracle.apply_matrix(mini, tuple(range(k - 1, -1, -1)), u)
                assert np.max(np.abs(after[row] - ref)) <= 1e-12, (gate, tg, ct, row)
    del s, t
    torch.cuda.empty_cache()


def test_single_gates_on_32_qubits_sampled():
    """32-qubit complex64 state (32 GiB): launches whose work-item count
    exceeds 2^32 for a naive grid (pairs, element-wise, LDS-staged and
    general kernels) run, checked on 256 sampled groups per gate."""
    import torch
    n = 32
    log("32-qubit single gates: allocating complex64 state")
    g = torch.Generator(device="cuda")
    g.manual_seed(1032)
    t = torch.randn(1 << n, dtype=torch.complex64, device="cuda", generator=g)
    t /= torch.linalg.vector_norm(t)
    s = sv.State(n, "c64", tensor=t, basis=None)
    rng = np.random.default_rng(3032)
    cases = [("H", (0,), ()), ("H", (31,), ()), ("RZ", (12,), ()), ("U4", (31, 1), ()), ("SWAP", (2, 30), ()),
             ("X", (5,), (0,)), ("GENERAL", (2, 1, 0), ())]
    for gate, tg, ct in cases:
        log("  case", gate, tg, ct)
        p = (float(rng.uniform(0, 2 * math.pi)),)
        k = len(tg)
        m = W.haar_unitary(k, rng) if gate in ("U4", "GENERAL") else None
        free = rng.integers(0, 1 << n, size=256, dtype=np.int64)
        for q in list(ct) + list(tg):
            free &= ~(1 << q)
        for q in ct:
            free |= 1 << q
        members = []
        for r in range(1 << k):
            off = 0
            for j, q in enumerate(tg):
                if (r >> (k - 1 - j)) & 1:
                    off |= 1 << q
            members.append(free | off)
        idx = torch.from_numpy(np.stack(members, axis=1).reshape(-1)).cuda()
        before = t[idx].cpu().numpy().astype(np.complex128).reshape(256, -1)
        if gate == "GENERAL":
            s.apply_general(tg, m)
            u = m
        else:
            s.apply(gate, tg, ct, p, m)
            u = oracle.gate_matrix(gate, p, m)
        s.synchronize()
        after = t[idx].cpu().numpy().astype(np.complex128).reshape(256, -1)
        for row in range(256):
            ref = oracle.apply_matrix(before[row].copy(), tuple(range(k - 1, -1, -1)), u)
            assert np.max(np.abs(after[row] - ref)) <= 1e-5, (gate, tg, ct, row)
    del s, t
    torch.cuda.empty_cache()


@pytest.mark.parametrize("n,dtype,tol", [(33, "c128", 1e-12), (34, "c64", 1e-5)])
def test_largest_states_sampled(n, dtype, tol):
    """The largest states one MI355X holds for each dtype (128 GiB: 33 qubits
    complex128, 34 qubits complex64): every kernel form once, at targets
    that put members 2^32 and more apart, checked on 256 sampled groups per
    gate against the oracle's dense apply, then the norm (a unitary keeps
    it) through the two-stage reduction."""
    import torch
    log(f"{n}-qubit {dtype}: allocating {((1 << n) * (16 if dtype == 'c128' else 8)) >> 30} GiB")
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    g = torch.Generator(device="cuda")
    g.manual_seed(1033 + n)
    t = torch.randn(1 << n, dtype=tdt, device="cuda", generator=g)
    t /= torch.linalg.vector_norm(t)
    s = sv.State(n, dtype, tensor=t, basis=None)
    rng = np.random.default_rng(3033 + n)
    top = n - 1
    cases = [("H", (0,), ()), ("RY", (top,), ()), ("RZ", (top - 1,), (2,)), ("U4", (top, 1), ()),
             ("SWAP", (3, top), ()), ("X", (top,), (0, 17)), ("Z", (top,), (top - 2,)), ("U2", (5,), (top,)),
             ("GENERAL", (top, 2, 0), ()), ("DENSE", (top, top - 1, 3, 0), ())]
    for gate, tg, ct in cases:
        log("  case", gate, tg, ct)
        p = (float(rng.uniform(0, 2 * math.pi)),)
        k = len(tg)
        m = W.haar_unitary(k, rng) if gate in ("U4", "U2", "GENERAL", "DENSE") else None
        free = rng.integers(0, 1 << n, size=256, dtype=np.int64)
        for q in list(ct) + list(tg):
            free &= ~(1 << q)
        for q in ct:
            free |= 1 << q
        members = []
        for r in range(1 << k):
            off = 0
            for j, q in enumerate(tg):
                if (r >> (k - 1 - j)) & 1:
                    off |= 1 << q
            members.append(free | off)
        idx = torch.from_numpy(np.stack(members, axis=1).reshape(-1)).cuda()
        before = t[idx].cpu().numpy().astype(np.complex128).reshape(256, -1)
        if gate == "GENERAL":
            s.apply_general(tg, m)
            u = m
        elif gate == "DENSE":
            s.apply_dense(tg, m)
            u = m
        else:
            s.apply(gate, tg, ct, p, m)
            u = oracle.gate_matrix(gate, p, m)
        s.synchronize()
        after = t[idx].cpu().numpy().astype(np.complex128).reshape(256, -1)
        if gate in ("X", "SWAP"):
            # moves: the sampled members are permuted bit for bit
            perm = [1, 0] if gate == "X" else [0, 2, 1, 3]
            assert np.array_equal(after, before[:, perm]), (gate, tg, ct)
            continue
        for row in range(256):
            ref = oracle.apply_matrix(before[row].copy(), tuple(range(k - 1, -1, -1)), u)
            assert np.max(np.abs(after[row] - ref)) <= tol, (gate, tg, ct, row)
    nrm = s.norm2()
    log(f"  norm^2 after the gates: {nrm!r}")
    assert abs(nrm - 1.0) <= (1e-11 if dtype == "c128" else 1e-4)
    del s, t
    torch.cuda.empty_cache()
