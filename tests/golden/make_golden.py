"""Writes tests/golden/oracle_hea6.txt by calling only the oracle.

Fixture: hardware-efficient ansatz on 6 qubits, 2 layers, angles from
workloads.uniform_angles(24, 1003); energy of sum_i Z_i Z_{i+1} and the full
final state.  Regenerate only when the oracle's arithmetic is deliberately
changed (and say why in the commit message).
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    n, L = 6, 2
    th = W.uniform_angles(W.hea_n_params(n, L), 1003)
    psi = oracle.run_circuit(oracle.zero_state(n), W.hea_ops(n, L), th)
    e = oracle.expval_obs(psi, W.sum_zz(n))
    with open(os.path.join(HERE, "oracle_hea6.txt"), "w") as f:
        f.write("# written by tests/golden/make_golden.py (oracle only): HEA n=6 L=2, "
                "angles uniform_angles(24, 1003), observable sum Z_i Z_{i+1}\n")
        f.write(f"energy {float(e)!r}\n")
        for x, a in enumerate(psi):
            f.write(f"{x} {float(a.real)!r} {float(a.imag)!r}\n")


if __name__ == "__main__":
    main()
