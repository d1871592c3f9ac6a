"""Writes tests/golden/oracle_circuits20.txt by calling only the oracle.

Reference results of the two 20-qubit circuits the complex64 error is
reported on:
  * hea: hardware-efficient ansatz (RY then RZ on every qubit, CNOT ladder
    q -> q+1), 10 layers, angles workloads.uniform_angles(400, 1003), from
    |0...0>;
  * qft: the QFT circuit (Hadamards and controlled phases, no swaps) on the
    basis state |x>, x = workloads.random_basis_index(20, 1004).
For each: the energy of sum_i Z_i and the amplitudes at 1024 indices drawn by
numpy.random.default_rng(1008).choice(2**20, 1024, replace=False), sorted.
A few seconds on the host.  Regenerate only when the oracle's arithmetic is
deliberately changed (and say why in the commit message).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "oracle_circuits20.txt")
N = 20


def sample_indices():
    return sorted(int(i) for i in np.random.default_rng(1008).choice(1 << N, 1024, replace=False))


def circuits():
    x = W.random_basis_index(N, 1004)
    return {"hea": (W.hea_ops(N, 10), W.uniform_angles(W.hea_n_params(N, 10), 1003), oracle.zero_state(N)),
            "qft": (W.qft_ops(N), np.zeros(0), oracle.basis_state(N, x))}


def main():
    idx = sample_indices()
    lines = ["# written by tests/golden/make_golden_circuits20.py (oracle only): 20-qubit HEA (10 layers, "
             "angles uniform_angles(400, 1003), from |0>) and QFT of |random_basis_index(20, 1004)>",
             "# rows: 'energy name E' (sum Z_i) | 'amp name index re im'"]
    for name, (ops, th, psi) in circuits().items():
        oracle.run_circuit(psi, ops, th)
        lines.append(f"energy {name} {oracle.expval_obs(psi, W.sum_z(N))!r}")
        lines += [f"amp {name} {i} {float(psi[i].real)!r} {float(psi[i].imag)!r}" for i in idx]
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
