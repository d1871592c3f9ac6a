"""GPU adjoint differentiation against the oracle's parameter-shift and
central-difference gradients (the oracle has no adjoint of its own).

Bars: complex128 adjoint vs oracle parameter shift <= 1e-10 max-abs, vs central
differences (h = 1e-6) <= 1e-7; complex64 adjoint vs the fp64 reference
<= 1e-4 max-abs.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

sv = pytest.importorskip("paper_2508_13615_amd")


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-10), ("c64", 1e-4)])
@pytest.mark.parametrize("n,layers,obs_name", [(6, 2, "zz"), (8, 3, "z"), (5, 2, "mixed")])
def test_adjoint_hea_vs_param_shift(dtype, tol, n, layers, obs_name):
    ops = W.hea_ops(n, layers)
    npar = W.hea_n_params(n, layers)
    th = W.uniform_angles(npar, 1005 + n)
    if obs_name == "zz":
        obs = W.sum_zz(n)
    elif obs_name == "z":
        obs = W.sum_z(n)
    else:
        obs = [(0.5, "XX", (0, 1)), (-0.8, "YZ", (2, 4)), (1.1, "Z", (3,)), (0.3, "XYZ", (0, 2, 4))]
    circ = sv.Circuit(n, ops, npar)
    psi = sv.State(n, dtype)
    lam = sv.State(n, dtype)
    e, g = circ.adjoint_grad(psi, lam, th, obs)
    e_ref = oracle.energy(n, ops, th, obs)
    g_ref = oracle.param_shift_grad(n, ops, th, obs)
    assert abs(e - e_ref) <= tol, (e, e_ref)
    err = float(np.max(np.abs(g - g_ref)))
    print(f"adjoint n={n} L={layers} {obs_name} {dtype}: max|g - g_ps| = {err:.2e}", flush=True)
    assert err <= tol
    # the reverse sweep un-applies every gate: psi is back at |0...0>
    back = psi.numpy().astype(np.complex128)
    assert abs(back[0] - 1.0) <= 100 * tol and np.max(np.abs(back[1:])) <= 100 * tol


def test_adjoint_phase_controlled_and_rx_vs_fd():
    n = 5
    ops = [W.Op("H", (), (q,)) for q in range(n)]
    ops += [W.Op("RX", (), (0,), 0), W.Op("PHASE", (), (1,), 1), W.Op("RY", (0,), (2,), 2),
            W.Op("PHASE", (2,), (3,), 3), W.Op("RZ", (1, 3), (4,), 4), W.Op("X", (4,), (0,)),
            W.Op("RY", (), (3,), 0), W.Op("U2", (), (2,), -1, 0.0, W.haar_unitary(1, np.random.default_rng(5))),
            W.Op("RX", (4,), (1,), 5), W.Op("SWAP", (), (0, 3)), W.Op("T", (), (2,)), W.Op("S", (), (1,))]
    th = W.uniform_angles(6, 4001)
    obs = [(0.9, "ZZ", (0, 1)), (0.4, "X", (2,)), (-0.7, "YY", (3, 4)), (0.2, "Z", (4,))]
    circ = sv.Circuit(n, ops, 6)
    psi, lam = sv.State(n), sv.State(n)
    e, g = circ.adjoint_grad(psi, lam, th, obs)
    assert abs(e - oracle.energy(n, ops, th, obs)) <= 1e-12
    f = oracle.fd_grad(n, ops, th, obs, h=1e-6)
    assert np.max(np.abs(g - f)) <= 1e-7, (g, f)
    assert np.max(np.abs(g)) > 1e-3  # parameter 0 is shared by two ops: its gradient is their sum


def test_adjoint_analytic_single_qubit():
    for th in (0.3, 1.9, 4.4):
        circ = sv.Circuit(1, [W.Op("RY", (), (0,), 0)], 1)
        e, g = circ.adjoint_grad(sv.State(1), sv.State(1), [th], [(1.0, "Z", (0,))])
        assert abs(e - math.cos(th)) <= 1e-15 and abs(g[0] + math.sin(th)) <= 1e-15


def test_autograd_function():
    import torch
    n, layers = 6, 2
    ops = W.hea_ops(n, layers)
    npar = W.hea_n_params(n, layers)
    th = W.uniform_angles(npar, 4002)
    circ = sv.Circuit(n, ops, npar)
    psi, lam = sv.State(n), sv.State(n)
    params = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    loss = 3.0 * sv.AdjointExpval.apply(params, circ, psi, lam, W.sum_zz(n))
    loss.backward()
    g_ref = oracle.param_shift_grad(n, ops, th, W.sum_zz(n))
    assert np.max(np.abs(params.grad.numpy() - 3.0 * g_ref)) <= 3e-10


def test_autograd_function_forward_only_when_no_gradient_is_needed():
    # under no_grad (or for parameters without requires_grad) only the forward
    # pass runs: lam is never written, and E matches the oracle
    import torch
    n, layers = 6, 2
    ops = W.hea_ops(n, layers)
    npar = W.hea_n_params(n, layers)
    th = W.uniform_angles(npar, 4003)
    circ = sv.Circuit(n, ops, npar)
    psi, lam = sv.State(n), sv.State(n)
    lam.set_basis(5)
    params = torch.tensor(th, dtype=torch.float64, requires_grad=True)
    with torch.no_grad():
        e = sv.AdjointExpval.apply(params, circ, psi, lam, W.sum_zz(n))
    assert not e.requires_grad
    assert abs(float(e) - oracle.energy(n, ops, th, W.sum_zz(n))) <= 1e-12
    lam_host = lam.numpy()
    assert lam_host[5] == 1 and np.count_nonzero(lam_host) == 1  # untouched
    e2 = sv.AdjointExpval.apply(torch.tensor(th), circ, psi, lam, W.sum_zz(n))
    assert float(e2) == float(e)


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-10), ("c64", 1e-4)])
def test_autograd_function_engine_form_keeps_parameters_on_device(dtype, tol):
    # a one-circuit Batch: params, E and the gradient stay in device memory
    import torch
    n, layers = 8, 3
    ops = W.hea_ops(n, layers)
    npar = W.hea_n_params(n, layers)
    th = W.uniform_angles(npar, 4004)
    b = sv.Batch([(n, ops, npar, "sum_zz")], dtype, with_grad=True)
    params = torch.tensor(th, dtype=torch.float64, device="cuda", requires_grad=True)
    loss = -2.0 * sv.AdjointExpval.apply(params, b)
    assert loss.device.type == "cuda"
    loss.backward()
    g_ref = oracle.param_shift_grad(n, ops, th, W.sum_zz(n))
    e_ref = oracle.energy(n, ops, th, W.sum_zz(n))
    assert abs(float(loss.detach()) + 2.0 * e_ref) <= 2 * tol * (n - 1)
    assert params.grad.device.type == "cuda"
    assert np.max(np.abs(params.grad.cpu().numpy() + 2.0 * g_ref)) <= 2 * tol
    # forward only: a batch without the sweep, and no gradient asked for
    f = sv.Batch([(n, ops, npar, "sum_zz")], dtype, with_grad=False)
    with torch.no_grad():
        e = sv.AdjointExpval.apply(params, f)
    assert abs(float(e) - e_ref) <= tol * (n - 1)
    with pytest.raises(ValueError):
        sv.AdjointExpval.apply(params, f)  # a gradient is needed, the batch has no sweep
