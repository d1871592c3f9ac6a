"""Independent routes to the full 2^N x 2^N action of a gate, used to pin the oracle.

Two routes that do not share the oracle's index-loop structure:
  * Kronecker products of per-qubit factors (textbook tensor-product embedding;
    with qubit q = bit q, the leftmost Kronecker factor is the most significant
    bit, i.e. qubit N-1);
  * tensor contraction: the state reshaped to N axes of size 2 (axis i holds
    bit N-1-i), the gate contracted with numpy.tensordot on the target axes.
"""
from __future__ import annotations

from functools import reduce
from typing import Dict, Sequence

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
P0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
P1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
PAULI = {
    "I": I2,
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def kron_factors(n: int, factors: Dict[int, np.ndarray]) -> np.ndarray:
    """Full operator that is factors[q] on qubit q and identity elsewhere."""
    mats = [factors.get(q, I2) for q in range(n - 1, -1, -1)]
    return reduce(np.kron, mats)


def kron_single(n: int, t: int, u: np.ndarray) -> np.ndarray:
    return np.kron(np.kron(np.eye(1 << (n - 1 - t)), u), np.eye(1 << t))


def kron_controlled_single(n: int, controls: Sequence[int], t: int, u: np.ndarray) -> np.ndarray:
    """Controlled-U = I - Pi + Pi (x) U, with Pi the projector onto all
    controls in |1>, built from per-qubit Kronecker factors."""
    pi = kron_factors(n, {c: P1 for c in controls})
    fac = {c: P1 for c in controls}
    fac[t] = u
    piu = kron_factors(n, fac)
    return np.eye(1 << n, dtype=np.complex128) - pi + piu


def kron_pauli(n: int, paulis: str, qubits: Sequence[int]) -> np.ndarray:
    return kron_factors(n, {q: PAULI[p] for p, q in zip(paulis, qubits)})


def tensordot_apply(psi: np.ndarray, targets: Sequence[int], u: np.ndarray,
                    controls: Sequence[int] = ()) -> np.ndarray:
    """Apply u on `targets` (first target = most significant matrix bit) by
    tensor contraction; controls restrict the result to indices whose control
    bits are 1 (elsewhere the state is unchanged)."""
    n = int(psi.size).bit_length() - 1
    k = len(targets)
    st = psi.reshape([2] * n)
    ut = u.reshape([2] * (2 * k))
    axes = [n - 1 - t for t in targets]
    out = np.tensordot(ut, st, axes=(list(range(k, 2 * k)), axes))
    out = np.moveaxis(out, list(range(k)), axes).reshape(-1)
    if controls:
        idx = np.arange(psi.size)
        sel = np.ones(psi.size, dtype=bool)
        for c in controls:
            sel &= ((idx >> c) & 1) == 1
        out = np.where(sel, out, psi)
    return out


def full_operator_tensordot(n: int, targets: Sequence[int], u: np.ndarray,
                            controls: Sequence[int] = ()) -> np.ndarray:
    eye = np.eye(1 << n, dtype=np.complex128)
    return np.stack([tensordot_apply(eye[:, j].copy(), targets, u, controls) for j in range(1 << n)], axis=1)
