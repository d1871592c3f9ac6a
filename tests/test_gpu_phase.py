"""Runs of diagonal gates as one pass (sv_apply_phases, sv_circuit_apply_fused)
against the fp64 oracle: explicit phase terms against the oracle's
controlled phases; circuits mixing diagonal and other gates, fused against
the oracle and against the op-by-op path; the QFT of a basis state against
its closed form, at 14 qubits and on sampled amplitudes at 32."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

sv = pytest.importorskip("paper_2508_13615_amd")
pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


def _rev(y, n):
    return int(format(y, f"0{n}b")[::-1], 2)


def _input(n, dtype, seed):
    psi = W.gaussian_state(n, seed)
    return psi.astype(np.complex64).astype(np.complex128) if dtype == "c64" else psi


def _oracle_phases(psi, masks, angles):
    # each term is a phase on the amplitudes holding all its bits: the
    # controlled PHASE gate with one of the bits as target (mask 0: global)
    for m, a in zip(masks, angles):
        bits = [q for q in range(64) if (m >> q) & 1]
        if not bits:
            psi = psi * np.exp(1j * a)
        else:
            psi = oracle.apply_gate(psi, "PHASE", (bits[0],), tuple(bits[1:]), (a,))
    return psi


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_phase_terms_vs_oracle(dtype):
    n = 12
    rng = np.random.default_rng(8000)
    psi0 = _input(n, dtype, 8001)
    for n_terms in (1, 2, 7, 31, 64):
        for common in (0, 1 << 5):
            masks = []
            for _ in range(n_terms):
                m = common
                for q in rng.choice(n, size=int(rng.integers(0, 4)), replace=False):
                    m |= 1 << int(q)
                masks.append(m)
            angles = rng.uniform(-2 * math.pi, 2 * math.pi, size=n_terms)
            s = sv.State(n, dtype, basis=None).load(psi0).apply_phases(masks, angles)
            ref = _oracle_phases(psi0.copy(), masks, angles)
            err = float(np.max(np.abs(s.numpy().astype(np.complex128) - ref)))
            print(f"phases {dtype} terms={n_terms} common={common}: {err:.2e}", flush=True)
            assert err <= 4 * TOL[dtype], (n_terms, common, err)


def test_phase_terms_exact_at_quarter_turns():
    # Z, S and CZ-type terms (multiples of pi/2) give exact phases: the result
    # equals the oracle's element-wise products exactly, up to signed zeros
    n = 10
    psi0 = W.gaussian_state(n, 8100)
    masks = [1 << 3, (1 << 3) | (1 << 7), 1 << 0, (1 << 2) | (1 << 9)]
    angles = [math.pi, math.pi / 2, -math.pi / 2, math.pi]
    got = sv.State(n, "c128", basis=None).load(psi0).apply_phases(masks, angles).numpy()
    idx = np.arange(1 << n)
    k = np.zeros(1 << n, dtype=np.int64)  # quarter turns per amplitude
    for m, a in zip(masks, angles):
        k += np.where((idx & m) == m, int(round(a / (math.pi / 2))), 0)
    unit = np.array([1, 1j, -1, -1j])[k % 4]
    assert np.array_equal(got, psi0 * unit)


def _mixed_ops(n, rng, count):
    ops, npar = [], 0
    diag1 = ["Z", "S", "T"]
    for _ in range(count):
        r = rng.random()
        q = [int(v) for v in rng.permutation(n)[:3]]
        if r < 0.15:
            ops.append(W.Op("H", (), (q[0],)))
        elif r < 0.25:
            ops.append(W.Op("X", (q[1],), (q[0],)))
        elif r < 0.35:
            ops.append(W.Op("RY", (), (q[0],), npar, 0.0))
            npar += 1
        elif r < 0.55:
            ctl = tuple(q[1:1 + int(rng.integers(0, 3))])
            ops.append(W.Op("RZ", ctl, (q[0],), npar, 0.0))
            npar += 1
        elif r < 0.75:
            ctl = tuple(q[1:1 + int(rng.integers(0, 3))])
            ops.append(W.Op("PHASE", ctl, (q[0],), -1, float(rng.uniform(-3, 3))))
        else:
            ctl = tuple(q[1:1 + int(rng.integers(0, 2))])
            ops.append(W.Op(diag1[int(rng.integers(0, 3))], ctl, (q[0],)))
    return ops, npar


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fused_circuit_vs_oracle_and_op_by_op(dtype):
    n = 12
    rng = np.random.default_rng(8200)
    for trial in range(4):
        ops, npar = _mixed_ops(n, rng, 120)
        th = rng.uniform(0, 2 * math.pi, size=max(1, npar))[:npar]
        psi0 = _input(n, dtype, 8210 + trial)
        circ = sv.Circuit(n, ops, npar)
        a = circ.apply(sv.State(n, dtype, basis=None).load(psi0), th, fuse_diagonal=True).numpy()
        b = circ.apply(sv.State(n, dtype, basis=None).load(psi0), th).numpy()
        ref = oracle.run_circuit(psi0.copy(), ops, th)
        err = float(np.max(np.abs(a.astype(np.complex128) - ref)))
        print(f"fused circuit {dtype} trial {trial}: {err:.2e}", flush=True)
        assert err <= 10 * TOL[dtype], (trial, err)
        assert float(np.max(np.abs(a.astype(np.complex128) - b.astype(np.complex128)))) <= 10 * TOL[dtype]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fused_same_qubit_products_vs_oracle(dtype):
    """Runs of 1 to 4 uncontrolled one-target gates (X, Y, H, RX, RY, U2) on
    one qubit, composed into one 2x2 by the fused path, alone, followed by a
    diagonal run (the product shares its pass) and between controlled gates,
    against the oracle and the op-by-op path."""
    n = 11
    rng = np.random.default_rng(8250)
    kinds = ["X", "Y", "H", "RX", "RY", "U2"]
    for trial in range(4):
        ops, npar = [], 0
        for _ in range(40):
            q = int(rng.integers(0, n))
            for _ in range(int(rng.integers(1, 5))):
                g = kinds[int(rng.integers(0, len(kinds)))]
                if g in ("RX", "RY"):
                    ops.append(W.Op(g, (), (q,), npar, 0.0))
                    npar += 1
                elif g == "U2":
                    ops.append(W.Op("U2", (), (q,), -1, 0.0, W.haar_unitary(1, rng)))
                else:
                    ops.append(W.Op(g, (), (q,)))
            r = rng.random()
            other = int((q + 1 + rng.integers(0, n - 1)) % n)
            if r < 0.4:
                for _ in range(int(rng.integers(1, 4))):
                    c = int(rng.integers(0, n))
                    ops.append(W.Op("PHASE", (c,) if c != q else (), (q,), -1, float(rng.uniform(-3, 3))))
            elif r < 0.7:
                ops.append(W.Op("X", (q,), (other,)))
        th = rng.uniform(0, 2 * math.pi, size=npar)
        psi0 = _input(n, dtype, 8260 + trial)
        circ = sv.Circuit(n, ops, npar)
        a = circ.apply(sv.State(n, dtype, basis=None).load(psi0), th, fuse_diagonal=True).numpy()
        b = circ.apply(sv.State(n, dtype, basis=None).load(psi0), th).numpy()
        ref = oracle.run_circuit(psi0.copy(), ops, th)
        err = float(np.max(np.abs(a.astype(np.complex128) - ref)))
        print(f"same-qubit products {dtype} trial {trial}: {len(ops)} ops, {err:.2e}", flush=True)
        assert err <= 10 * TOL[dtype], (trial, err)
        assert float(np.max(np.abs(a.astype(np.complex128) - b.astype(np.complex128)))) <= 10 * TOL[dtype]


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-13), ("c64", 2e-7)])
def test_fused_qft_closed_form(dtype, tol):
    n = 14
    x = W.random_basis_index(n, 8300)
    st = sv.State(n, dtype, basis=x)
    sv.Circuit(n, W.qft_ops(n), 0).apply(st, [], fuse_diagonal=True)
    got = st.numpy().astype(np.complex128)
    y = np.arange(1 << n)
    want = np.array([math.pow(2.0, -n / 2) * np.exp(2j * math.pi * ((x * _rev(int(v), n)) % (1 << n)) / (1 << n))
                     for v in y])
    assert float(np.max(np.abs(got - want))) <= tol


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-13), ("c64", 2e-9)])
def test_fused_qft32_closed_form_sampled(dtype, tol):
    """The 32-qubit QFT op by op with its controlled-phase runs fused (the
    benchmark's form), against the closed form on 4096 sampled amplitudes."""
    import torch
    n = 32
    x = W.random_basis_index(n, 1004)
    print(f"fused qft32 {dtype}: allocating", flush=True)
    st = sv.State(n, dtype, basis=x)
    sv.Circuit(n, W.qft_ops(n), 0).apply(st, [], fuse_diagonal=True)
    idx = np.unique(np.random.default_rng(7).integers(0, 1 << n, size=4096, dtype=np.int64))
    got = st.tensor[torch.as_tensor(idx, device="cuda")].cpu().numpy().astype(np.complex128)
    want = np.array([math.pow(2.0, -n / 2) * np.exp(2j * math.pi * ((x * _rev(int(v), n)) % (1 << n)) / (1 << n))
                     for v in idx])
    err = float(np.max(np.abs(got - want)))
    print(f"fused qft32 {dtype}: max sampled error {err:.2e}", flush=True)
    assert err <= tol, err
    del st
    torch.cuda.empty_cache()
