"""Pins of the oracle against facts that do not come from the oracle itself.

Each test below would fail on a plausible slip in the oracle: a transposed
matrix index, a dropped or mis-signed term, a control read as a 0-control or
ignored, a wrong rotation sign or half-angle, a Y gate or a Pauli Y inside an
expectation with the wrong sign, an expectation that forgets the conjugate.
Nothing here takes its reference from the oracle's own gate table: the
brute-force routes use the Pauli matrices written out in tests/bruteforce.py.  Routes used: Kronecker-product and
tensor-contraction embeddings (tests/bruteforce.py), closed forms (GHZ, QFT of
a basis state and of an arbitrary state via numpy.fft), gate identities,
analytic expectation values and derivatives, and hand-derived fixtures
under tests/golden/.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W
from bruteforce import (P1, PAULI, full_operator_tensordot, kron_controlled_single, kron_factors,
                        kron_pauli, kron_single, tensordot_apply)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-13


def rand_state(n, seed):
    return W.gaussian_state(n, seed)


ONE_Q = ["X", "Y", "Z", "H", "S", "T", "RX", "RY", "RZ", "PHASE", "U2"]


def _params(g, rng):
    if g in ("RX", "RY", "RZ", "PHASE"):
        return (float(rng.uniform(0, 2 * math.pi)),)
    return ()


# ---------------------------------------------------------------------------
# brute force: every gate, every qubit index / ordered pair / triple
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 3, 5])
def test_single_qubit_vs_kron(n):
    rng = np.random.default_rng(10 + n)
    psi = rand_state(n, 20 + n)
    for g in ONE_Q:
        for t in range(n):
            p = _params(g, rng)
            m = W.haar_unitary(1, rng) if g == "U2" else None
            u = oracle.gate_matrix(g, p, m)
            ref = kron_single(n, t, u) @ psi
            got = oracle.apply_gate(psi.copy(), g, (t,), (), p, m)
            assert np.max(np.abs(got - ref)) < TOL, (g, t)


@pytest.mark.parametrize("n", [2, 4])
def test_controlled_single_vs_kron(n):
    rng = np.random.default_rng(30 + n)
    psi = rand_state(n, 40 + n)
    for g in ONE_Q:
        for c, t in itertools.permutations(range(n), 2):
            p = _params(g, rng)
            m = W.haar_unitary(1, rng) if g == "U2" else None
            u = oracle.gate_matrix(g, p, m)
            ref = kron_controlled_single(n, (c,), t, u) @ psi
            got = oracle.apply_gate(psi.copy(), g, (t,), (c,), p, m)
            assert np.max(np.abs(got - ref)) < TOL, (g, c, t)


def test_toffoli_every_triple_vs_kron():
    n = 4
    psi = rand_state(n, 50)
    X = PAULI["X"]
    for a, b, t in itertools.permutations(range(n), 3):
        ref = kron_controlled_single(n, (a, b), t, X) @ psi
        got = oracle.apply_gate(psi.copy(), "X", (t,), (a, b))
        assert np.array_equal(got, ref), (a, b, t)


def test_y_gate_vs_independent_pauli_matrix():
    # The Y gate against the Pauli Y written out in tests/bruteforce.py (not
    # the oracle's gate table), uncontrolled and with one or two controls.
    n = 4
    psi = rand_state(n, 52)
    Y = PAULI["Y"]
    for t in range(n):
        got = oracle.apply_gate(psi.copy(), "Y", (t,))
        assert np.max(np.abs(got - kron_single(n, t, Y) @ psi)) < TOL, t
    for c, t in itertools.permutations(range(n), 2):
        got = oracle.apply_gate(psi.copy(), "Y", (t,), (c,))
        assert np.max(np.abs(got - kron_controlled_single(n, (c,), t, Y) @ psi)) < TOL, (c, t)
    for a, b, t in itertools.permutations(range(n), 3):
        got = oracle.apply_gate(psi.copy(), "Y", (t,), (a, b))
        assert np.max(np.abs(got - kron_controlled_single(n, (a, b), t, Y) @ psi)) < TOL, (a, b, t)


def test_y_gate_identities_and_basis_action():
    # Y = i X Z through the oracle's X move and Z; Y^2 = I; RY(pi) = -i Y and
    # RX(pi) = -i X; Y|0> = i|1>, Y|1> = -i|0> exactly.
    n = 3
    psi = rand_state(n, 53)
    for t in range(n):
        y = oracle.apply_gate(psi.copy(), "Y", (t,))
        ixz = 1j * oracle.apply_gate(oracle.apply_gate(psi.copy(), "Z", (t,)), "X", (t,))
        assert np.max(np.abs(y - ixz)) < TOL
        yy = oracle.apply_gate(y.copy(), "Y", (t,))
        assert np.max(np.abs(yy - psi)) < TOL
        ry = oracle.apply_gate(psi.copy(), "RY", (t,), (), (math.pi,))
        assert np.max(np.abs(ry - (-1j) * y)) < TOL
        rx = oracle.apply_gate(psi.copy(), "RX", (t,), (), (math.pi,))
        assert np.max(np.abs(rx - (-1j) * oracle.apply_gate(psi.copy(), "X", (t,)))) < TOL
    e0 = oracle.apply_gate(oracle.basis_state(1, 0), "Y", (0,))
    assert np.array_equal(e0, np.array([0, 1j]))
    e1 = oracle.apply_gate(oracle.basis_state(1, 1), "Y", (0,))
    assert np.array_equal(e1, np.array([-1j, 0]))


def _swap_operator(n, a, b):
    """SWAP of qubits a and b as (I + XX + YY + ZZ) / 2, from Kronecker
    factors of the written-out Pauli matrices (entries are exact 0 and 1)."""
    terms = [kron_factors(n, {})] + [kron_factors(n, {a: PAULI[p], b: PAULI[p]}) for p in "XYZ"]
    return sum(terms) / 2


def test_swap_operator_route_is_a_permutation():
    # the route itself: a 0/1 permutation matrix that exchanges the two bits
    n = 3
    for a, b in itertools.permutations(range(n), 2):
        op = _swap_operator(n, a, b)
        for x in range(1 << n):
            ba, bb = (x >> a) & 1, (x >> b) & 1
            y = x & ~((1 << a) | (1 << b)) | (bb << a) | (ba << b)
            col = np.zeros(1 << n)
            col[y] = 1
            assert np.array_equal(op[:, x], col)


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_controlled_swap_every_triple_vs_kron(dtype):
    # Fredkin on every ordered (control, a, b) at n = 4, and with two controls
    # on every ordered 4-tuple: I - Pi + Pi SWAP_ab, Pi the projector onto
    # all controls in |1>; bit-exact (the operator has 0/1 entries).
    n = 4
    psi = rand_state(n, 54)
    for c, a, b in itertools.permutations(range(n), 3):
        pi = kron_factors(n, {c: P1})
        op = np.eye(1 << n) - pi + pi @ _swap_operator(n, a, b)
        ref = (op @ psi).astype(dtype)
        got = oracle.move_swap(psi.astype(dtype), a, b, (c,))
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), (c, a, b)
    for c1, c2, a, b in itertools.permutations(range(n), 4):
        pi = kron_factors(n, {c1: P1, c2: P1})
        op = np.eye(1 << n) - pi + pi @ _swap_operator(n, a, b)
        got = oracle.move_swap(psi.copy(), a, b, (c1, c2))
        assert np.array_equal(got, op @ psi), (c1, c2, a, b)


def test_controlled_swap_hand_fixture():
    # 3 qubits, control 2, swap (1, 0): only |101> <-> |110> trade places
    # (indices 5 and 6); every other amplitude stays.  With the control at 0
    # everywhere the move is the identity.
    psi = np.arange(1, 9, dtype=np.float64) + 1j * np.arange(11, 19, dtype=np.float64)
    got = oracle.move_swap(psi.copy(), 1, 0, (2,))
    ref = psi.copy()
    ref[5], ref[6] = psi[6], psi[5]
    assert np.array_equal(got, ref)
    off = psi.copy()
    off[4:] = 0
    assert np.array_equal(oracle.move_swap(off.copy(), 1, 0, (2,)), off)
    # uncontrolled: |01x> <-> |10x> style exchange of bits 1 and 0 everywhere
    got = oracle.move_swap(psi.copy(), 1, 0)
    ref = psi.copy()
    ref[1], ref[2], ref[5], ref[6] = psi[2], psi[1], psi[6], psi[5]
    assert np.array_equal(got, ref)


def test_cnot_textbook_matrix():
    # CNOT(control=1, target=0) on 2 qubits; index = 2*b1 + b0 and the textbook
    # matrix with the control as the most significant bit.
    cnot = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 0, 1], [0, 0, 1, 0]], dtype=np.complex128)
    psi = rand_state(2, 51)
    got = oracle.apply_gate(psi.copy(), "X", (0,), (1,))
    assert np.array_equal(got, cnot @ psi)
    # and the same matrix given densely on (control, target) = (1, 0)
    got2 = oracle.apply_matrix(psi.copy(), (1, 0), cnot)
    assert np.max(np.abs(got2 - cnot @ psi)) < TOL


@pytest.mark.parametrize("n", [3, 5])
def test_two_qubit_dense_every_ordered_pair_vs_tensordot(n):
    rng = np.random.default_rng(60 + n)
    psi = rand_state(n, 61 + n)
    for a, b in itertools.permutations(range(n), 2):
        u = W.haar_unitary(2, rng)
        ref = tensordot_apply(psi, (a, b), u)
        got = oracle.apply_gate(psi.copy(), "U4", (a, b), (), (), u)
        assert np.max(np.abs(got - ref)) < TOL, (a, b)
        sw = oracle.apply_gate(psi.copy(), "SWAP", (a, b))
        ref_sw = tensordot_apply(psi, (a, b), oracle.gate_matrix("SWAP"))
        assert np.array_equal(sw, ref_sw), (a, b)


def test_adjacent_two_qubit_vs_kron():
    n = 4
    rng = np.random.default_rng(70)
    psi = rand_state(n, 71)
    for t in range(n - 1):
        u = W.haar_unitary(2, rng)
        # first-listed target t+1 is the matrix MSB, matching the kron order
        ref = np.kron(np.kron(np.eye(1 << (n - 2 - t)), u), np.eye(1 << t)) @ psi
        got = oracle.apply_matrix(psi.copy(), (t + 1, t), u)
        assert np.max(np.abs(got - ref)) < TOL


def test_three_qubit_dense_vs_tensordot_and_operator():
    n = 5
    rng = np.random.default_rng(80)
    psi = rand_state(n, 81)
    for tg in [(0, 1, 2), (4, 0, 2), (3, 1, 4), (2, 4, 0)]:
        u = W.haar_unitary(3, rng)
        ref = tensordot_apply(psi, tg, u)
        got = oracle.apply_matrix(psi.copy(), tg, u)
        assert np.max(np.abs(got - ref)) < TOL
    # controlled two-qubit unitary: full operator via contraction of basis vectors
    u = W.haar_unitary(2, rng)
    full = full_operator_tensordot(n, (3, 1), u, (0, 4))
    got = oracle.apply_matrix(psi.copy(), (3, 1), u, (0, 4))
    assert np.max(np.abs(got - full @ psi)) < TOL


def test_routes_agree_with_each_other():
    # the two brute-force routes pin each other as well
    n = 4
    rng = np.random.default_rng(90)
    for t in range(n):
        u = W.haar_unitary(1, rng)
        assert np.max(np.abs(kron_single(n, t, u) - full_operator_tensordot(n, (t,), u))) < 1e-15


# ---------------------------------------------------------------------------
# permutation gates: bit-exact, both precisions
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_permutation_identities_bit_exact(dtype):
    n = 6
    psi = rand_state(n, 100).astype(dtype)
    for t in range(n):
        a = oracle.move_x(oracle.move_x(psi.copy(), t), t)
        assert np.array_equal(a.view(np.uint8), psi.view(np.uint8))
    for c, t in itertools.permutations(range(n), 2):
        a = oracle.move_x(oracle.move_x(psi.copy(), t, (c,)), t, (c,))
        assert np.array_equal(a.view(np.uint8), psi.view(np.uint8))
        s1 = oracle.move_swap(psi.copy(), c, t)
        s3 = psi.copy()
        oracle.move_x(s3, t, (c,))
        oracle.move_x(s3, c, (t,))
        oracle.move_x(s3, t, (c,))
        assert np.array_equal(s1.view(np.uint8), s3.view(np.uint8))
        s2 = oracle.move_swap(s1.copy(), t, c)
        assert np.array_equal(s2.view(np.uint8), psi.view(np.uint8))


def test_move_path_equals_dense_path_bit_for_bit():
    # 1*a + 0*b == a exactly for finite non-zero a, b: the dense definition of
    # X / CNOT / SWAP / Toffoli reproduces the move path bit for bit.
    n = 5
    psi = rand_state(n, 101)
    X = oracle.gate_matrix("X")
    for t in range(n):
        assert np.array_equal(oracle.move_x(psi.copy(), t), oracle.apply_matrix(psi.copy(), (t,), X))
    for a, b in itertools.permutations(range(n), 2):
        assert np.array_equal(oracle.move_x(psi.copy(), b, (a,)),
                              oracle.apply_matrix(psi.copy(), (b,), X, (a,)))
        assert np.array_equal(oracle.move_swap(psi.copy(), a, b),
                              oracle.apply_matrix(psi.copy(), (a, b), oracle.gate_matrix("SWAP")))


def test_control_zero_is_identity_bit_exact():
    n = 5
    rng = np.random.default_rng(102)
    psi = rand_state(n, 103)
    psi[(np.arange(psi.size) >> 3) & 1 == 1] = 0  # control qubit 3 is |0> everywhere
    for g in ONE_Q:
        p = _params(g, rng)
        m = W.haar_unitary(1, rng) if g == "U2" else None
        got = oracle.apply_gate(psi.copy(), g, (1,), (3,), p, m)
        assert np.array_equal(got, psi), g


# ---------------------------------------------------------------------------
# gate identities
# ---------------------------------------------------------------------------
def _apply_seq(psi, seq):
    psi = psi.copy()
    for g, t, c, p in seq:
        oracle.apply_gate(psi, g, t, c, p)
    return psi


def test_gate_identities():
    n = 4
    psi = rand_state(n, 110)
    for t in range(n):
        assert np.max(np.abs(_apply_seq(psi, [("H", (t,), (), ()), ("H", (t,), (), ())]) - psi)) < TOL
        hxh = _apply_seq(psi, [("H", (t,), (), ()), ("X", (t,), (), ()), ("H", (t,), (), ())])
        assert np.max(np.abs(hxh - _apply_seq(psi, [("Z", (t,), (), ())]))) < TOL
        hzh = _apply_seq(psi, [("H", (t,), (), ()), ("Z", (t,), (), ()), ("H", (t,), (), ())])
        assert np.max(np.abs(hzh - _apply_seq(psi, [("X", (t,), (), ())]))) < TOL
        a, b = 0.37, 2.91
        rz2 = _apply_seq(psi, [("RZ", (t,), (), (a,)), ("RZ", (t,), (), (b,))])
        assert np.max(np.abs(rz2 - _apply_seq(psi, [("RZ", (t,), (), (a + b,))]))) < TOL
        assert np.max(np.abs(_apply_seq(psi, [("RY", (t,), (), (2 * math.pi,))]) + psi)) < TOL
        assert np.max(np.abs(_apply_seq(psi, [("RY", (t,), (), (4 * math.pi,))]) - psi)) < TOL
        ss = _apply_seq(psi, [("S", (t,), (), ()), ("S", (t,), (), ())])
        assert np.max(np.abs(ss - _apply_seq(psi, [("Z", (t,), (), ())]))) < TOL
        tt = _apply_seq(psi, [("T", (t,), (), ()), ("T", (t,), (), ())])
        assert np.max(np.abs(tt - _apply_seq(psi, [("S", (t,), (), ())]))) < TOL
        # RX(th) = H RZ(th) H, RZ(th) = e^{-i th/2} PHASE(th)
        th = 1.234
        rx = _apply_seq(psi, [("RX", (t,), (), (th,))])
        hrzh = _apply_seq(psi, [("H", (t,), (), ()), ("RZ", (t,), (), (th,)), ("H", (t,), (), ())])
        assert np.max(np.abs(rx - hrzh)) < TOL
        rz = _apply_seq(psi, [("RZ", (t,), (), (th,))])
        ph = _apply_seq(psi, [("PHASE", (t,), (), (th,))]) * complex(math.cos(th / 2), -math.sin(th / 2))
        assert np.max(np.abs(rz - ph)) < TOL
    for c, t in itertools.permutations(range(n), 2):
        cp = _apply_seq(psi, [("PHASE", (t,), (c,), (math.pi,))])
        cz = _apply_seq(psi, [("Z", (t,), (c,), ())])
        assert np.max(np.abs(cp - cz)) < TOL
        hch = _apply_seq(psi, [("H", (t,), (), ()), ("X", (t,), (c,), ()), ("H", (t,), (), ())])
        assert np.max(np.abs(hch - cz)) < TOL
        # CZ and CP are symmetric in their two qubits
        assert np.max(np.abs(_apply_seq(psi, [("Z", (c,), (t,), ())]) - cz)) < TOL


def test_haar_unitarity_and_adjoint_roundtrip():
    n = 4
    rng = np.random.default_rng(120)
    psi = rand_state(n, 121)
    for k in (1, 2, 3):
        u = W.haar_unitary(k, rng)
        assert np.max(np.abs(u.conj().T @ u - np.eye(1 << k))) < 1e-14
        tg = tuple(range(k))[::-1]
        a = oracle.apply_matrix(psi.copy(), tg, u)
        b = oracle.apply_matrix(a, tg, np.ascontiguousarray(u.conj().T))
        assert np.max(np.abs(b - psi)) < TOL


def test_norm_preserved_random_circuits():
    rng = np.random.default_rng(130)
    n = 7
    psi = rand_state(n, 131)
    for _ in range(60):
        g = rng.choice(ONE_Q + ["U4", "SWAP"])
        qs = [int(q) for q in rng.permutation(n)]
        nt = 2 if g in ("U4", "SWAP") else 1
        nc = int(rng.integers(0, 3))
        tg, ct = tuple(qs[:nt]), tuple(qs[nt:nt + nc])
        m = W.haar_unitary(2, rng) if g == "U4" else (W.haar_unitary(1, rng) if g == "U2" else None)
        oracle.apply_gate(psi, g, tg, ct, _params(g, rng), m)
    assert abs(oracle.norm2(psi) - 1.0) < 1e-13


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 5, 10])
def test_ghz_bit_exact(n):
    psi = oracle.run_circuit(oracle.zero_state(n), W.ghz_ops(n))
    ref = np.zeros(1 << n, dtype=np.complex128)
    ref[0] = ref[-1] = math.sqrt(0.5)  # fl(2^(-1/2)): H entries times exact 1s and 0s
    assert np.array_equal(psi, ref)


@pytest.mark.parametrize("n", [1, 4, 9])
def test_hadamard_wall_uniform(n):
    psi = oracle.zero_state(n)
    for q in range(n):
        oracle.apply_gate(psi, "H", (q,))
    assert np.max(np.abs(psi - 2.0 ** (-n / 2))) < 1e-15


def _rev(y, n):
    return int(format(y, f"0{n}b")[::-1], 2)


@pytest.mark.parametrize("n", [1, 2, 3, 6, 10])
def test_qft_basis_state_closed_form(n):
    # <y|QFT_noswap|x> = 2^{-n/2} exp(2 pi i x rev_n(y) / 2^n); the phase
    # numerator is taken mod 2^n in integers.
    rng = np.random.default_rng(140 + n)
    for x in sorted({0, (1 << n) - 1, int(rng.integers(0, 1 << n))}):
        psi = oracle.run_circuit(oracle.basis_state(n, x), W.qft_ops(n))
        ys = np.arange(1 << n)
        m = np.array([(x * _rev(int(y), n)) % (1 << n) for y in ys], dtype=np.float64)
        ref = np.exp(2j * math.pi * m / (1 << n)) * 2.0 ** (-n / 2)
        assert np.max(np.abs(psi - ref)) < 1e-12, x


@pytest.mark.parametrize("n", [3, 8])
def test_qft_arbitrary_state_vs_numpy_fft(n):
    psi0 = rand_state(n, 150 + n)
    psi = oracle.run_circuit(psi0.copy(), W.qft_ops(n))
    f = np.sqrt(1 << n) * np.fft.ifft(psi0)
    ref = f[[_rev(y, n) for y in range(1 << n)]]
    assert np.max(np.abs(psi - ref)) < 1e-12


def test_golden_qft2_hand_derived():
    # tests/golden/qft2_noswap.txt: the 4x4 matrix of the two-qubit QFT circuit
    # (Sec. 3.2: Hadamards and controlled phase gates), derived by hand.
    rows = []
    with open(os.path.join(GOLDEN, "qft2_noswap.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([complex(tok.replace("i", "j")) for tok in line.split()])
    ref = np.array(rows, dtype=np.complex128) / 2.0
    cols = []
    for x in range(4):
        cols.append(oracle.run_circuit(oracle.basis_state(2, x), W.qft_ops(2)))
    assert np.max(np.abs(np.stack(cols, axis=1) - ref)) < 1e-15


# ---------------------------------------------------------------------------
# expectation values
# ---------------------------------------------------------------------------
def test_expval_basis_states():
    n = 6
    for x in [0, 1, 37, 63]:
        psi = oracle.basis_state(n, x)
        for q in range(n):
            assert oracle.expval_pauli(psi, "Z", (q,)).real == 1 - 2 * ((x >> q) & 1)
        sz = oracle.expval_obs(psi, W.sum_z(n))
        assert sz == n - 2 * bin(x).count("1")
        szz = oracle.expval_obs(psi, W.sum_zz(n))
        assert szz == (n - 1) - 2 * bin((x ^ (x >> 1)) & ((1 << (n - 1)) - 1)).count("1")


def test_expval_single_qubit_analytic():
    for th in [0.0, 0.3, 1.7, 3.9, 5.5]:
        psi = oracle.apply_gate(oracle.zero_state(1), "RY", (0,), (), (th,))
        assert abs(oracle.expval_pauli(psi, "Z", (0,)).real - math.cos(th)) < 1e-15
        assert abs(oracle.expval_pauli(psi, "X", (0,)).real - math.sin(th)) < 1e-15
        psi = oracle.apply_gate(oracle.zero_state(1), "RX", (0,), (), (th,))
        assert abs(oracle.expval_pauli(psi, "Y", (0,)).real + math.sin(th)) < 1e-15
        assert abs(oracle.expval_pauli(psi, "Z", (0,)).real - math.cos(th)) < 1e-15


def test_expval_vs_kron_pauli():
    n = 5
    rng = np.random.default_rng(160)
    psi = rand_state(n, 161)
    for _ in range(40):
        k = int(rng.integers(1, n + 1))
        qs = tuple(int(q) for q in rng.permutation(n)[:k])
        ps = "".join(rng.choice(list("IXYZ"), size=k))
        ref = np.vdot(psi, kron_pauli(n, ps, qs) @ psi)
        got = oracle.expval_pauli(psi, ps, qs)
        assert abs(got - ref) < 1e-14, (ps, qs)


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------
def test_gradient_single_qubit_analytic():
    ops = [W.Op("RY", (), (0,), 0)]
    for th in [0.2, 1.1, 2.5, 4.0]:
        g = oracle.param_shift_grad(1, ops, [th], [(1.0, "Z", (0,))])
        assert abs(g[0] + math.sin(th)) < 1e-14
        f = oracle.fd_grad(1, ops, [th], [(1.0, "Z", (0,))])
        assert abs(f[0] + math.sin(th)) < 1e-9


def test_gradient_two_qubit_closed_form():
    # RY(a) on 0, RY(b) on 1, CNOT 0->1, O = Z_1  =>  E = cos a cos b
    ops = [W.Op("RY", (), (0,), 0), W.Op("RY", (), (1,), 1), W.Op("X", (0,), (1,))]
    a, b = 0.7, 2.2
    e = oracle.energy(2, ops, [a, b], [(1.0, "Z", (1,))])
    assert abs(e - math.cos(a) * math.cos(b)) < 1e-15
    g = oracle.param_shift_grad(2, ops, [a, b], [(1.0, "Z", (1,))])
    assert abs(g[0] + math.sin(a) * math.cos(b)) < 1e-14
    assert abs(g[1] + math.cos(a) * math.sin(b)) < 1e-14


def test_gradient_phase_and_controlled_phase_closed_form():
    # H on 0 and 1, PHASE(a) on 0, controlled PHASE(b) 0->1, H on 0, O = Z_0:
    # closed form by hand: E = (cos a + cos(a+b)) / 2
    ops = [W.Op("H", (), (0,)), W.Op("H", (), (1,)), W.Op("PHASE", (), (0,), 0),
           W.Op("PHASE", (0,), (1,), 1), W.Op("H", (), (0,))]
    a, b = 0.9, 1.6
    obs = [(1.0, "Z", (0,))]
    e = oracle.energy(2, ops, [a, b], obs)
    assert abs(e - 0.5 * (math.cos(a) + math.cos(a + b))) < 1e-14
    g = oracle.param_shift_grad(2, ops, [a, b], obs)
    assert abs(g[0] + 0.5 * (math.sin(a) + math.sin(a + b))) < 1e-14
    assert abs(g[1] + 0.5 * math.sin(a + b)) < 1e-14


def test_param_shift_vs_fd_hea():
    n, L = 4, 2
    ops = W.hea_ops(n, L)
    th = W.uniform_angles(W.hea_n_params(n, L), 170)
    obs = W.sum_zz(n)
    g = oracle.param_shift_grad(n, ops, th, obs)
    f = oracle.fd_grad(n, ops, th, obs)
    assert np.max(np.abs(g - f)) < 1e-8
    assert np.max(np.abs(g)) > 1e-2


def test_param_shift_rejects_controlled_rotation():
    ops = [W.Op("RY", (0,), (1,), 0)]
    with pytest.raises(ValueError):
        oracle.param_shift_grad(2, ops, [0.1], [(1.0, "Z", (1,))])


# ---------------------------------------------------------------------------
# workload structure pins (Sec. 3.2 counts)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [3, 6, 10])
def test_universal_circuit_gate_counts(n):
    ops = W.universal_ops(n)
    assert len(ops) == 2 * n * n
    assert sum(1 for o in ops if o.gate == "X") == n * (n - 1)
    assert sum(1 for o in ops if o.gate == "RZ") == n * (n + 1)


def test_qft_and_hea_gate_counts():
    assert len(W.qft_ops(32)) == 32 + 32 * 31 // 2
    ops = W.hea_ops(32, 10)
    assert len(ops) == 10 * (2 * 32 + 31)
    assert W.hea_n_params(24, 8) == 384


# ---------------------------------------------------------------------------
# planted mistakes: the pins above must catch them
# ---------------------------------------------------------------------------
def test_planted_transpose_is_caught():
    n = 3
    rng = np.random.default_rng(180)
    psi = rand_state(n, 181)
    u = W.haar_unitary(2, rng)
    wrong = oracle.apply_matrix(psi.copy(), (2, 0), np.ascontiguousarray(u.T))
    assert np.max(np.abs(wrong - tensordot_apply(psi, (2, 0), u))) > 1e-3
    swapped_order = oracle.apply_matrix(psi.copy(), (0, 2), u)
    assert np.max(np.abs(swapped_order - tensordot_apply(psi, (2, 0), u))) > 1e-3


def test_planted_sign_is_caught():
    psi = oracle.apply_gate(oracle.zero_state(1), "RX", (0,), (), (0.8,))
    wrong_y = np.vdot(psi, (-PAULI["Y"]) @ psi).real
    assert abs(wrong_y + math.sin(0.8)) > 0.5
    wrong_rz = oracle.apply_matrix(W.gaussian_state(2, 3), (1,), oracle.gate_matrix("RZ", (-0.8,)))
    good_rz = kron_single(2, 1, np.diag([np.exp(-0.4j), np.exp(0.4j)])) @ W.gaussian_state(2, 3)
    assert np.max(np.abs(wrong_rz - good_rz)) > 1e-2


def test_planted_y_sign_and_ignored_control_are_caught():
    # a Y gate of the wrong sign, and a controlled SWAP that ignores its
    # control, both differ from the independent routes used by the pins
    n = 3
    psi = rand_state(n, 182)
    wrong_y = oracle.apply_matrix(psi.copy(), (1,), np.ascontiguousarray(-PAULI["Y"]))
    assert np.max(np.abs(wrong_y - kron_single(n, 1, PAULI["Y"]) @ psi)) > 1e-2
    ignored = oracle.move_swap(psi.copy(), 1, 0)
    pi = kron_factors(n, {2: P1})
    op = np.eye(1 << n) - pi + pi @ _swap_operator(n, 1, 0)
    assert not np.array_equal(ignored, op @ psi)


def test_golden_oracle_regression_hea6():
    # tests/golden/oracle_hea6.txt was written by tests/golden/make_golden.py,
    # which calls only the oracle; it locks the oracle's arithmetic in place.
    rows = {}
    e_ref = None
    with open(os.path.join(GOLDEN, "oracle_hea6.txt")) as f:
        for line in f:
            if line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "energy":
                e_ref = float(tok[1])
            else:
                rows[int(tok[0])] = complex(float(tok[1]), float(tok[2]))
    n, L = 6, 2
    th = W.uniform_angles(W.hea_n_params(n, L), 1003)
    psi = oracle.run_circuit(oracle.zero_state(n), W.hea_ops(n, L), th)
    ref = np.array([rows[x] for x in range(1 << n)])
    assert np.max(np.abs(psi - ref)) < 1e-15
    assert abs(oracle.expval_obs(psi, W.sum_zz(n)) - e_ref) < 1e-15


def test_dense_four_to_six_qubit_blocks_vs_tensordot():
    # the oracle's dense path at the block sizes of the matrix-core kernel
    # (k = 4..6): against numpy's tensor contraction, for target orders that
    # are ascending, descending and scattered
    n = 8
    rng = np.random.default_rng(140)
    psi = rand_state(n, 141)
    for tg in [(0, 1, 2, 3), (7, 5, 3, 1), (6, 0, 4, 2, 7), (3, 4, 5, 6, 7), (5, 1, 7, 0, 3, 6), (0, 1, 2, 3, 4, 5)]:
        u = W.haar_unitary(len(tg), rng)
        got = oracle.apply_matrix(psi.copy(), tg, u)
        assert np.max(np.abs(got - tensordot_apply(psi, tg, u))) < TOL, tg


def test_dense_block_of_kron_product_equals_one_qubit_gates():
    # a 4-qubit Kronecker product u0 (x) u1 (x) u2 (x) u3 on targets (a, b, c, d)
    # (first factor on the first-listed target, the matrix MSB) equals the
    # four one-qubit gates applied one by one
    n = 7
    rng = np.random.default_rng(150)
    psi = rand_state(n, 151)
    tg = (5, 0, 3, 6)
    us = [W.haar_unitary(1, rng) for _ in tg]
    big = np.kron(np.kron(np.kron(us[0], us[1]), us[2]), us[3])
    got = oracle.apply_matrix(psi.copy(), tg, big)
    ref = psi.copy()
    for t, u in zip(tg, us):
        ref = oracle.apply_matrix(ref, (t,), u)
    assert np.max(np.abs(got - ref)) < TOL


def test_dense_six_qubit_adjoint_roundtrip():
    n = 9
    rng = np.random.default_rng(160)
    psi = rand_state(n, 161)
    tg = (8, 2, 5, 0, 7, 3)
    u = W.haar_unitary(6, rng)
    a = oracle.apply_matrix(psi.copy(), tg, u)
    b = oracle.apply_matrix(a, tg, np.ascontiguousarray(u.conj().T))
    assert abs(oracle.norm2(a) - 1.0) < 1e-13
    assert np.max(np.abs(b - psi)) < TOL
