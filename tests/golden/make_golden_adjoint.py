"""Writes tests/golden/oracle_adjoint_hea.txt by calling only the oracle.

Reference gradients for the adjoint-differentiation workload: the
hardware-efficient ansatz (per layer RY then RZ on every qubit, then a CNOT
ladder q -> q+1) from |0...0>, 8 layers, angles workloads.uniform_angles(
2 * n * 8, 1005), observable sum_i Z_i Z_{i+1}.  The oracle has no adjoint
method of its own; its gradients are the two-term parameter-shift rule (exact
for exp(-i th P / 2)) and central differences with h = 1e-6.

  * n = 24 (384 parameters): the energy, and on 16 parameter indices drawn by
    numpy.random.default_rng(1007).choice(384, 16, replace=False) the
    parameter-shift and the central-difference gradient;
  * n = 12 and n = 16: the energy and the parameter-shift gradient of every
    parameter.

About 20 minutes on 8 host threads.  Regenerate only when the oracle's
arithmetic is deliberately changed (and say why in the commit message).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "oracle_adjoint_hea.txt")
LAYERS = 8
SEED_ANGLES = 1005
SEED_SAMPLE = 1007
SAMPLE = 16
FD_H = 1e-6


def sample_indices(npar):
    return sorted(int(j) for j in np.random.default_rng(SEED_SAMPLE).choice(npar, SAMPLE, replace=False))


def main():
    lines = ["# written by tests/golden/make_golden_adjoint.py (oracle only): HEA, 8 layers, angles "
             "uniform_angles(2*n*8, 1005), observable sum Z_i Z_{i+1}",
             "# rows: 'energy n E' | 'ps n j dE/dth_j' (parameter shift) | 'fd n j dE/dth_j' (central, h=1e-6)"]
    for n in (12, 16, 24):
        t0 = time.time()
        ops = W.hea_ops(n, LAYERS)
        npar = W.hea_n_params(n, LAYERS)
        th = W.uniform_angles(npar, SEED_ANGLES)
        obs = W.sum_zz(n)
        lines.append(f"energy {n} {oracle.energy(n, ops, th, obs)!r}")
        which = list(range(npar)) if n < 24 else sample_indices(npar)
        g = oracle.param_shift_grad(n, ops, th, obs, which=which)
        lines += [f"ps {n} {j} {float(g[j])!r}" for j in which]
        if n == 24:
            f = oracle.fd_grad(n, ops, th, obs, h=FD_H, which=which)
            lines += [f"fd {n} {j} {float(f[j])!r}" for j in which]
        print(f"n={n}: {len(which)} parameters in {time.time() - t0:.0f} s", flush=True)
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
