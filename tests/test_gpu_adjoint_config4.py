"""The adjoint gradient of the 24-qubit workload against the oracle.

Workload: hardware-efficient ansatz from |0...0>, 8 layers of RY then RZ on
every qubit followed by a CNOT ladder, angles uniform_angles(2 n 8, 1005),
observable sum_i Z_i Z_{i+1}.  The oracle's gradients are stored in
tests/golden/oracle_adjoint_hea.txt (written by make_golden_adjoint.py, which
calls only the oracle: a 24-qubit oracle gradient takes about 25 minutes on 8
host threads, too long for a test):
  * n = 24, 384 parameters: parameter shift and central differences
    (h = 1e-6) on 16 seeded parameter indices;
  * n = 12 and 16: parameter shift on every parameter.
Both GPU forms are checked: the op-by-op adjoint sweep (sv_adjoint_grad) and
the fused pass engine (sv_batch_run with the gradient).

Bars: complex128 within 1e-10 of the parameter shift and 1e-7 of the central
differences (their own rounding at 24 qubits is about 3e-8); complex64
within 1e-4 of the fp64 parameter shift; energies within 1e-12 per term
(complex128) and 1e-5 per term (complex64).
"""
import os
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

sv = pytest.importorskip("paper_2508_13615_amd")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_adjoint_hea.txt")
LAYERS = 8
TOL_PS = {"c128": 1e-10, "c64": 1e-4}
TOL_E = {"c128": 1e-12, "c64": 1e-5}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def golden(n):
    e, ps, fd = None, {}, {}
    with open(GOLDEN) as f:
        for line in f:
            tok = line.split()
            if not tok or tok[0].startswith("#") or int(tok[1]) != n:
                continue
            if tok[0] == "energy":
                e = float(tok[2])
            else:
                (ps if tok[0] == "ps" else fd)[int(tok[2])] = float(tok[3])
    return e, ps, fd


def gpu_grads(n, dtype):
    """(E, grad) from the op-by-op adjoint sweep and from the fused engine."""
    ops = W.hea_ops(n, LAYERS)
    npar = W.hea_n_params(n, LAYERS)
    th = W.uniform_angles(npar, 1005)
    obs = W.sum_zz(n)
    circ = sv.Circuit(n, ops, npar)
    e1, g1 = circ.adjoint_grad(sv.State(n, dtype), sv.State(n, dtype), th, obs)
    b = sv.Batch([(n, ops, npar, "sum_zz")], dtype, with_grad=True)
    e2, g2 = b.run(th)
    return {"op_by_op": (e1, g1), "fused": (float(e2[0]), g2)}


def test_golden_reference_shape():
    # 16 sampled indices at 24 qubits (both routes), every index at 12 and 16
    e, ps, fd = golden(24)
    assert e is not None and len(ps) == 16 and sorted(ps) == sorted(fd)
    for n in (12, 16):
        e, ps, fd = golden(n)
        assert e is not None and sorted(ps) == list(range(W.hea_n_params(n, LAYERS))) and not fd


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [12, 16])
def test_adjoint_all_parameters_vs_oracle(n, dtype):
    e_ref, ps, _ = golden(n)
    g_ref = np.array([ps[j] for j in range(len(ps))])
    for form, (e, g) in gpu_grads(n, dtype).items():
        err = float(np.max(np.abs(g - g_ref)))
        log(f"n={n} {dtype} {form}: max|g - g_ps| = {err:.2e}, |E - E_ref| = {abs(e - e_ref):.2e}")
        assert err <= TOL_PS[dtype], form
        assert abs(e - e_ref) <= TOL_E[dtype] * (n - 1), form


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_adjoint_24q_sampled_vs_oracle_param_shift_and_fd(dtype):
    n = 24
    e_ref, ps, fd = golden(n)
    js = sorted(ps)
    g_ps = np.array([ps[j] for j in js])
    g_fd = np.array([fd[j] for j in js])
    for form, (e, g) in gpu_grads(n, dtype).items():
        err_ps = float(np.max(np.abs(g[js] - g_ps)))
        err_fd = float(np.max(np.abs(g[js] - g_fd)))
        log(f"n=24 {dtype} {form}: max|g - g_ps| = {err_ps:.2e}, max|g - g_fd| = {err_fd:.2e}, "
            f"|E - E_ref| = {abs(e - e_ref):.2e}")
        assert err_ps <= TOL_PS[dtype], form
        if dtype == "c128":
            assert err_fd <= 1e-7, form
        assert abs(e - e_ref) <= TOL_E[dtype] * (n - 1), form
