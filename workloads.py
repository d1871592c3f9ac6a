"""Seeded synthetic inputs shared by the oracle-side and GPU-side tests and benches.

This module holds no arithmetic of the simulation method itself: it only draws
random states, angles and unitaries and writes down circuit structures (which
gate acts on which qubits, with which parameter slot). Both the CPU oracle and
the HIP library receive these inputs and compute independently.

Conventions (shared input format, nothing more):
  * qubit q is bit q (weight 2**q) of the amplitude index (Sec. 2 numbers qubits
    from zero, with the first L qubits local under a block partition, i.e. the
    low index bits);
  * an ``Op`` names a gate, its control qubits (1-controls), its target qubits,
    a parameter slot ``pidx`` (-1 = fixed angle ``value``) and, for the matrix
    gates U2/U4/GENERAL, a row-major complex matrix whose row/column index puts
    the first-listed target in the most significant bit.
"""
from __future__ import annotations

import math
from typing import List, NamedTuple, Optional, Sequence, Tuple

import numpy as np


class Op(NamedTuple):
    gate: str
    controls: Tuple[int, ...] = ()
    targets: Tuple[int, ...] = ()
    pidx: int = -1
    value: float = 0.0
    matrix: Optional[np.ndarray] = None


# A Pauli-sum observable is a list of (coefficient, pauli-letters, qubits).
Term = Tuple[float, str, Tuple[int, ...]]

ONE_QUBIT_FIXED = ("I", "X", "Y", "Z", "H", "S", "T")
ONE_QUBIT_ROT = ("RX", "RY", "RZ", "PHASE")
PERMUTATION = ("X", "SWAP")


# --------------------------------------------------------------------------
# random inputs
# --------------------------------------------------------------------------
def gaussian_state(n: int, seed: int) -> np.ndarray:
    """i.i.d. complex Gaussian amplitudes (Re, Im ~ N(0,1)), normalised in fp64.
    The real parts are drawn first, then the imaginary parts, straight into
    the result (a 30-qubit state peaks near 2.5x its own 16 GiB)."""
    rng = np.random.default_rng(seed)
    psi = np.empty(1 << n, dtype=np.complex128)
    psi.real = rng.standard_normal(1 << n)
    psi.imag = rng.standard_normal(1 << n)
    re, im = psi.real, psi.imag
    psi /= math.sqrt(float(np.sum(re * re + im * im)))
    return psi


def haar_unitary(k: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random U(2**k): QR of a complex Ginibre matrix with the phases of
    R's diagonal moved into Q (Mezzadri 2007)."""
    d = 1 << k
    z = (rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d))) / math.sqrt(2.0)
    q, r = np.linalg.qr(z)
    ph = np.diag(r) / np.abs(np.diag(r))
    return (q * ph[None, :]).astype(np.complex128)


def uniform_angles(count: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, size=count)


def random_basis_index(n: int, seed: int) -> int:
    return int(np.random.default_rng(seed).integers(0, 1 << n))


# --------------------------------------------------------------------------
# circuits (structure only)
# --------------------------------------------------------------------------
def hea_ops(n: int, layers: int) -> List[Op]:
    """Hardware-efficient ansatz: per layer RY then RZ on every qubit, then a
    CNOT ladder q -> q+1.  Parameter slot of RY on (layer l, qubit q) is
    2*(l*n+q), of the RZ right after it 2*(l*n+q)+1."""
    ops: List[Op] = []
    for l in range(layers):
        for q in range(n):
            ops.append(Op("RY", (), (q,), 2 * (l * n + q)))
            ops.append(Op("RZ", (), (q,), 2 * (l * n + q) + 1))
        for q in range(n - 1):
            ops.append(Op("X", (q,), (q + 1,)))
    return ops


def hea_n_params(n: int, layers: int) -> int:
    return 2 * n * layers


def qft_ops(n: int) -> List[Op]:
    """QFT as Hadamards and controlled phase gates, no final swaps: for
    j = n-1 .. 0, H on j, then for c = j-1 .. 0 a controlled phase of angle
    pi / 2**(j-c) with control c and target j."""
    ops: List[Op] = []
    for j in range(n - 1, -1, -1):
        ops.append(Op("H", (), (j,)))
        for c in range(j - 1, -1, -1):
            ops.append(Op("PHASE", (c,), (j,), -1, math.pi / float(1 << (j - c))))
    return ops


def ghz_ops(n: int) -> List[Op]:
    ops = [Op("H", (), (0,))]
    ops += [Op("X", (q,), (q + 1,)) for q in range(n - 1)]
    return ops


def universal_ops(n: int) -> List[Op]:
    """One reading of the universal circuit (2 n^2 gates: n(n-1) CNOTs and
    n(n+1) Z-rotations R_k by pi/2^k): for each target t, R on t, then for each
    other qubit c a CNOT c->t followed by R on t.  The figure that fixes the
    structure is not available, so only the gate counts are pinned."""
    ops: List[Op] = []
    for t in range(n):
        k = 1
        ops.append(Op("RZ", (), (t,), -1, math.pi / float(1 << k)))
        for c in range(n):
            if c == t:
                continue
            k += 1
            ops.append(Op("X", (c,), (t,)))
            ops.append(Op("RZ", (), (t,), -1, math.pi / float(1 << min(k, 60))))
        ops.append(Op("RZ", (), (t,), -1, math.pi / float(1 << min(k + 1, 60))))
    return ops


def sum_z(n: int) -> List[Term]:
    return [(1.0, "Z", (q,)) for q in range(n)]


def sum_zz(n: int) -> List[Term]:
    return [(1.0, "ZZ", (q, q + 1)) for q in range(n - 1)]


# --------------------------------------------------------------------------
# gate sweeps (single-gate parity and bench cases)
# --------------------------------------------------------------------------
class GateCase(NamedTuple):
    gate: str
    controls: Tuple[int, ...]
    targets: Tuple[int, ...]
    params: Tuple[float, ...]
    matrix: Optional[np.ndarray]


def sweep_cases(n: int, seed: int = 1002, extras: bool = True) -> List[GateCase]:
    """Every gate class on every valid qubit index: one-qubit gates on each t,
    two-qubit gates on every ordered pair, Toffoli on every ordered triple."""
    rng = np.random.default_rng(seed)
    cases: List[GateCase] = []
    one = ["H", "X", "Z", "RZ", "RY", "U2"] + (["RX", "S", "T", "PHASE", "Y"] if extras else [])
    for g in one:
        for t in range(n):
            p: Tuple[float, ...] = ()
            m = None
            if g in ONE_QUBIT_ROT:
                p = (float(rng.uniform(0, 2 * math.pi)),)
            if g == "U2":
                m = haar_unitary(1, rng)
            cases.append(GateCase(g, (), (t,), p, m))
    pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
    for g in ["CNOT", "SWAP", "U4"] + (["CZ", "CP", "CU2"] if extras else []):
        for a, b in pairs:
            if g == "CNOT":
                cases.append(GateCase("X", (a,), (b,), (), None))
            elif g == "SWAP":
                cases.append(GateCase("SWAP", (), (a, b), (), None))
            elif g == "U4":
                cases.append(GateCase("U4", (), (a, b), (), haar_unitary(2, rng)))
            elif g == "CZ":
                cases.append(GateCase("Z", (a,), (b,), (), None))
            elif g == "CP":
                cases.append(GateCase("PHASE", (a,), (b,), (float(rng.uniform(0, 2 * math.pi)),), None))
            elif g == "CU2":
                cases.append(GateCase("U2", (a,), (b,), (), haar_unitary(1, rng)))
    for a in range(n):
        for b in range(n):
            for t in range(n):
                if len({a, b, t}) == 3:
                    cases.append(GateCase("X", (a, b), (t,), (), None))
    return cases


def second_qubit_choices(t: int, n: int) -> List[int]:
    """Controls (or second qubits) for the large single-gate sweep: indices 0,
    n//2 and n-1, minus the target itself."""
    return [c for c in (0, n // 2, n - 1) if c != t]


# --------------------------------------------------------------------------
# batched mixed-size workload
# --------------------------------------------------------------------------
class BatchCircuit(NamedTuple):
    n: int
    layers: int
    params: np.ndarray


def batch_spec(count: int = 256, seed: int = 1006, qmin: int = 14, qmax: int = 22,
               lmin: int = 4, lmax: int = 12) -> List[BatchCircuit]:
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.integers(qmin, qmax + 1))
        layers = int(rng.integers(lmin, lmax + 1))
        out.append(BatchCircuit(n, layers, rng.uniform(0, 2 * math.pi, size=hea_n_params(n, layers))))
    return out
