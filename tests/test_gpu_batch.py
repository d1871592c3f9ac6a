"""The fused pass engine (sv_batch_*) against the oracle and the op-by-op path.

Small tile sizes force many passes and many tiles per pass, so scheduling,
tile addressing and the cross-workgroup dependencies are exercised on states
the oracle handles in milliseconds.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

sv = pytest.importorskip("paper_2508_13615_amd")

TOL = {"c128": 1e-12, "c64": 1e-5}
GATES = ["X", "Y", "Z", "H", "S", "T", "RX", "RY", "RZ", "PHASE", "U2", "U4", "SWAP"]


def random_circuit(n, n_ops, rng, max_q, n_params):
    ops = []
    for _ in range(n_ops):
        g = str(rng.choice(GATES))
        nt = 2 if g in ("U4", "SWAP") else 1
        if nt > n:
            continue
        qs = [int(q) for q in rng.permutation(n)]
        nc = int(rng.integers(0, max(0, min(2, n - nt, max_q - nt)) + 1))
        m = W.haar_unitary(nt, rng) if g in ("U2", "U4") else None
        pidx = int(rng.integers(0, n_params)) if g in ("RX", "RY", "RZ", "PHASE") and n_params else -1
        val = float(rng.uniform(0, 2 * math.pi))
        ops.append(W.Op(g, tuple(qs[nt:nt + nc]), tuple(qs[:nt]), pidx, val, m))
    return ops


def obs_terms(kind, n):
    return W.sum_z(n) if kind == "sum_z" else W.sum_zz(n)


@pytest.mark.parametrize("apt", [16, 8])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("tile", [4, 5, 0])
def test_batch_forward_states_and_energies(dtype, tile, apt):
    # 3 qubits is below a register tile (LDS-sweep form); the others are register-tiled
    rng = np.random.default_rng(5000 + tile)
    circs, params = [], []
    for n in (3, 5, 8, 10):
        npar = 6
        ops = random_circuit(n, 40, rng, tile if tile else 12, npar)
        th = rng.uniform(0, 2 * math.pi, size=npar)
        circs.append((n, ops, npar, "sum_z" if n % 2 else "sum_zz"))
        params.append(th)
    b = sv.Batch(circs, dtype, tile_qubits=tile, amps_per_thread=apt, with_grad=False)
    e, g = b.run(np.concatenate(params))
    assert g is None
    info = b.info()
    assert info["passes"] >= len(circs)
    for i, (n, ops, npar, obs) in enumerate(circs):
        ref = oracle.run_circuit(oracle.zero_state(n), ops, params[i])
        got = b.state(i).astype(np.complex128)
        err = float(np.max(np.abs(got - ref)))
        assert err <= 4 * TOL[dtype], (i, n, err)
        e_ref = oracle.expval_obs(ref, obs_terms(obs, n))
        assert abs(e[i] - e_ref) <= 4 * TOL[dtype] * n, (i, e[i], e_ref)


def two_branch_circuit(n, rng, reps):
    """Runs of one-target gates on a target t in which some gates are
    controlled by one other qubit c: the forward passes fuse each run into one
    2x2 chosen by bit c.  Four patterns: rotation, CNOT, rotation; CNOT then
    uncontrolled gates; controlled diagonal and phase gates inside a run;
    controlled U2 and Z between uncontrolled gates.  Each parameterised gate
    has a parameter of its own (the two-term shift rule needs that); returns
    (ops, number of parameters)."""
    ops = []
    n_params = 0
    for _ in range(reps):
        t, c = (int(x) for x in rng.permutation(n)[:2])
        p = n_params
        v = float(rng.uniform(0, 2 * math.pi))
        pat = int(rng.integers(0, 4))
        if pat == 0:
            ops += [W.Op("U2", (), (t,), -1, 0.0, W.haar_unitary(1, rng)), W.Op("X", (c,), (t,)),
                    W.Op("RY", (), (t,), p, v)]
            n_params += 1
        elif pat == 1:
            ops += [W.Op("X", (c,), (t,)), W.Op("RZ", (), (t,), p, v), W.Op("H", (), (t,))]
            n_params += 1
        elif pat == 2:
            ops += [W.Op("RX", (), (t,), p, v), W.Op("RZ", (c,), (t,), -1, v / 3),
                    W.Op("PHASE", (c,), (t,), -1, v / 5), W.Op("Y", (), (t,))]
            n_params += 1
        else:
            ops += [W.Op("H", (), (t,)), W.Op("U2", (c,), (t,), -1, 0.0, W.haar_unitary(1, rng)),
                    W.Op("S", (), (t,)), W.Op("Z", (c,), (t,))]
    return ops, n_params


@pytest.mark.parametrize("apt", [16, 8])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("tile", [4, 5, 0])
def test_two_branch_fusion_states_and_energies(dtype, tile, apt):
    # 3 qubits runs the LDS-sweep form; the others put selectors on lane and
    # register bits across the layouts
    rng = np.random.default_rng(5100 + tile)
    circs, params, n_gates = [], [], 0
    for n in (3, 6, 10):
        ops, npar = two_branch_circuit(n, rng, 30)
        n_gates += len(ops)
        circs.append((n, ops, npar, "sum_zz"))
        params.append(rng.uniform(0, 2 * math.pi, size=npar))
    b = sv.Batch(circs, dtype, tile_qubits=tile, amps_per_thread=apt, with_grad=False)
    e, _ = b.run(np.concatenate(params))
    assert b.info()["fused_ops"] < n_gates // 2  # runs of 3-4 gates became one op each
    for i, (n, ops, npar, obs) in enumerate(circs):
        ref = oracle.run_circuit(oracle.zero_state(n), ops, params[i])
        got = b.state(i).astype(np.complex128)
        err = float(np.max(np.abs(got - ref)))
        assert err <= 4 * TOL[dtype], (i, n, err)
        e_ref = oracle.expval_obs(ref, obs_terms(obs, n))
        assert abs(e[i] - e_ref) <= 4 * TOL[dtype] * n, (i, e[i], e_ref)


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-10), ("c64", 1e-4)])
def test_two_branch_fusion_gradients_vs_oracle(dtype, tol):
    # with the adjoint: forward passes fused, reverse passes gate by gate
    rng = np.random.default_rng(5200)
    n = 9
    ops, npar = two_branch_circuit(n, rng, 25)
    th = rng.uniform(0, 2 * math.pi, size=npar)
    b = sv.Batch([(n, ops, npar, "sum_z")], dtype, tile_qubits=6, with_grad=True)
    e, g = b.run(th)
    g_ref = oracle.param_shift_grad(n, ops, th, W.sum_z(n))
    assert abs(e[0] - oracle.energy(n, ops, th, W.sum_z(n))) <= tol * n
    assert float(np.max(np.abs(g - g_ref))) <= tol


@pytest.mark.parametrize("apt", [16, 8])
@pytest.mark.parametrize("dtype,tol", [("c128", 1e-10), ("c64", 1e-4)])
def test_batch_gradients_vs_oracle(dtype, tol, apt):
    rng = np.random.default_rng(5101)
    circs, params, refs = [], [], []
    for n, L in ((4, 2), (6, 2), (9, 1)):
        ops = W.hea_ops(n, L)
        npar = W.hea_n_params(n, L)
        th = rng.uniform(0, 2 * math.pi, size=npar)
        obs = "sum_zz" if n != 4 else "sum_z"
        circs.append((n, ops, npar, obs))
        params.append(th)
        refs.append((oracle.energy(n, ops, th, obs_terms(obs, n)),
                     oracle.param_shift_grad(n, ops, th, obs_terms(obs, n))))
    # a circuit with controlled rotations, PHASE and shared parameters: central differences
    n = 5
    ops = [W.Op("H", (), (q,)) for q in range(n)]
    ops += [W.Op("RX", (), (0,), 0), W.Op("PHASE", (), (1,), 1), W.Op("RY", (0,), (2,), 2),
            W.Op("PHASE", (2,), (3,), 3), W.Op("RZ", (1, 3), (4,), 4), W.Op("X", (4,), (0,)),
            W.Op("RY", (), (3,), 0), W.Op("SWAP", (), (0, 3)), W.Op("RX", (4,), (1,), 5), W.Op("T", (), (2,))]
    th = rng.uniform(0, 2 * math.pi, size=6)
    circs.append((n, ops, 6, "sum_zz"))
    params.append(th)
    refs.append((oracle.energy(n, ops, th, W.sum_zz(n)), oracle.fd_grad(n, ops, th, W.sum_zz(n))))
    for tile in (4, 0):
        b = sv.Batch(circs, dtype, tile_qubits=tile, amps_per_thread=apt, with_grad=True)
        e, g = b.run(np.concatenate(params))
        off = 0
        for i, (n, ops, npar, obs) in enumerate(circs):
            e_ref, g_ref = refs[i]
            gt = tol if i < 3 else max(tol, 1e-7)
            assert abs(e[i] - e_ref) <= tol, (tile, i, e[i], e_ref)
            assert np.max(np.abs(g[off:off + npar] - g_ref)) <= gt, (tile, i, g[off:off + npar], g_ref)
            off += npar


def test_batch_graph_replays_equal_eager():
    rng = np.random.default_rng(5202)
    circs = []
    for n, L in ((6, 3), (8, 2), (11, 2)):
        circs.append((n, W.hea_ops(n, L), W.hea_n_params(n, L), "sum_z"))
    total = sum(c[2] for c in circs)
    bg = sv.Batch(circs, "c128", tile_qubits=5, use_graph=True, with_grad=True)
    be = sv.Batch(circs, "c128", tile_qubits=5, use_graph=False, with_grad=True)
    for rep in range(3):
        th = rng.uniform(0, 2 * math.pi, size=total)
        eg, gg = bg.run(th)
        # eager work between replays
        s = sv.State(7).set_basis(3)
        s.apply("H", (2,))
        ee, ge = be.run(th)
        assert np.array_equal(eg, ee), rep
        assert np.array_equal(gg, ge), rep


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-10), ("c64", 1e-4)])
def test_batch_matches_op_by_op_adjoint_mixed_sizes(dtype, tol):
    # config-5 shaped, scaled down: qubit counts and layer counts drawn per circuit
    spec = W.batch_spec(count=10, seed=5303, qmin=6, qmax=14, lmin=2, lmax=5)
    circs = [(c.n, W.hea_ops(c.n, c.layers), len(c.params), "sum_z") for c in spec]
    b = sv.Batch(circs, dtype, with_grad=True)
    e, g = b.run(np.concatenate([c.params for c in spec]))
    off = 0
    for i, c in enumerate(spec):
        circ = sv.Circuit(c.n, W.hea_ops(c.n, c.layers), len(c.params))
        e1, g1 = circ.adjoint_grad(sv.State(c.n, "c128"), sv.State(c.n, "c128"), c.params, W.sum_z(c.n))
        assert abs(e[i] - e1) <= tol, (i, e[i], e1)
        assert np.max(np.abs(g[off:off + len(c.params)] - g1)) <= tol, i
        off += len(c.params)


def test_batch_large_circuit_multi_tile():
    # one 20-qubit circuit with the default tile: many tiles and passes
    n, L = 20, 3
    ops = W.hea_ops(n, L)
    th = W.uniform_angles(W.hea_n_params(n, L), 5404)
    b = sv.Batch([(n, ops, len(th), "sum_zz")], "c128", with_grad=True)
    e, g = b.run(th)
    circ = sv.Circuit(n, ops, len(th))
    e1, g1 = circ.adjoint_grad(sv.State(n), sv.State(n), th, W.sum_zz(n))
    assert abs(e[0] - e1) <= 1e-11
    assert np.max(np.abs(g - g1)) <= 1e-10
    assert abs(e[0] - oracle.energy(n, ops, th, W.sum_zz(n))) <= 1e-11
    info = b.info()
    assert info["max_passes"] < len(ops) / 4  # fusion: far fewer passes than gates


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-10), ("c64", 1e-4)])
def test_every_tunable_engine_shape_vs_oracle(dtype, tol):
    """Every tile shape the autotuner may pick, for each stage mix: the
    forward state against the fp64 oracle, and with the adjoint, energy and
    gradient against the op-by-op adjoint kernels."""
    from paper_2508_13615_amd.autotune import ENGINE_SHAPES
    n, L = 16, 3
    ops = W.hea_ops(n, L)
    th = W.uniform_angles(W.hea_n_params(n, L), 5405)
    ref = oracle.run_circuit(oracle.zero_state(n), ops, th)
    e1, g1 = sv.Circuit(n, ops, len(th)).adjoint_grad(sv.State(n), sv.State(n), th, W.sum_zz(n))
    for grad in (False, True):
        for tq, apt in ENGINE_SHAPES[(dtype, grad)]:
            print(f"shape {dtype} grad={grad} tile {tq} x {apt}", flush=True)
            b = sv.Batch([(n, ops, len(th), "sum_zz")], dtype, tile_qubits=tq, amps_per_thread=apt, with_grad=grad)
            e, g = b.run(th)
            assert b.info()["threads"] == max(64, 2 ** tq // apt)
            if grad:
                assert abs(e[0] - e1) <= tol * n and np.max(np.abs(g - g1)) <= tol, (tq, apt)
            else:
                err = float(np.max(np.abs(b.state(0).astype(np.complex128) - ref)))
                assert err <= (1e-12 if dtype == "c128" else 1e-5), (tq, apt, err)


def phase_run_circuit(n, rng):
    """QFT-shaped circuit whose controlled phases each carry a parameter of
    their own, with RZ and H between targets and a few doubly controlled
    phases (three-qubit masks, applied as per-mask chains): the forward passes
    multiply the phases on one target (and one lane bit besides) into a
    factor per lane, the reverse passes differentiate each of them.  Returns
    (ops, number of parameters)."""
    ops, np_ = [], 0
    for j in range(n - 1, -1, -1):
        ops.append(W.Op("H", (), (j,)))
        for c in range(j - 1, -1, -1):
            ops.append(W.Op("PHASE", (c,), (j,), np_, float(rng.uniform(0, 2 * math.pi))))
            np_ += 1
        if j >= 2:
            ops.append(W.Op("T", (j - 1, j - 2), (j,)))
        ops.append(W.Op("RZ", (), (j,), np_, float(rng.uniform(0, 2 * math.pi))))
        np_ += 1
    return ops, np_


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-10), ("c64", 1e-4)])
@pytest.mark.parametrize("tile", [4, 6, 0])
def test_phase_run_gradients_vs_oracle(dtype, tol, tile):
    rng = np.random.default_rng(5600 + tile)
    n = 9
    ops, npar = phase_run_circuit(n, rng)
    th = rng.uniform(0, 2 * math.pi, size=npar)
    ref = oracle.run_circuit(oracle.zero_state(n), ops, th)
    b = sv.Batch([(n, ops, npar, "sum_zz")], dtype, tile_qubits=tile, with_grad=False)
    b.run(th)
    err = float(np.max(np.abs(b.state(0).astype(np.complex128) - ref)))
    assert err <= 4 * TOL[dtype], err
    b = sv.Batch([(n, ops, npar, "sum_zz")], dtype, tile_qubits=tile, with_grad=True)
    e, g = b.run(th)
    g_ref = oracle.param_shift_grad(n, ops, th, W.sum_zz(n))
    assert abs(e[0] - oracle.expval_obs(ref, W.sum_zz(n))) <= tol * n
    assert float(np.max(np.abs(g - g_ref))) <= tol


def rotation_pairs_circuit(n, rng, reps):
    """Pairs of parameterised rotations on one target with the same controls
    (none, one or two), the reverse passes' fusable form, between H layers and
    CNOTs; every rotation has a parameter of its own.  Returns (ops, number of
    parameters)."""
    ops = [W.Op("H", (), (q,)) for q in range(n)]
    np_ = 0
    for _ in range(reps):
        qs = [int(q) for q in rng.permutation(n)]
        t, ctl = qs[0], tuple(qs[1:1 + int(rng.integers(0, 3))])
        g1, g2 = (str(x) for x in rng.choice(["RX", "RY", "RZ"], size=2))
        ops.append(W.Op(g1, ctl, (t,), np_, 0.0))
        ops.append(W.Op(g2, ctl, (t,), np_ + 1, 0.0))
        np_ += 2
        ops.append(W.Op("X", (qs[-1],), (qs[-2],)))
    return ops, np_


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-7), ("c64", 1e-4)])
@pytest.mark.parametrize("tile", [4, 6, 0])
def test_reverse_pair_gradients_vs_oracle(dtype, tol, tile):
    # controlled rotations: central differences (the two-term shift rule does not hold for them)
    rng = np.random.default_rng(5700 + tile)
    n = 8
    ops, npar = rotation_pairs_circuit(n, rng, 14)
    th = rng.uniform(0, 2 * math.pi, size=npar)
    b = sv.Batch([(n, ops, npar, "sum_zz")], dtype, tile_qubits=tile, with_grad=True)
    e, g = b.run(th)
    g_ref = oracle.fd_grad(n, ops, th, W.sum_zz(n), h=1e-6)
    e_tol = (1e-10 if dtype == "c128" else 1e-4) * n
    assert abs(e[0] - oracle.energy(n, ops, th, W.sum_zz(n))) <= e_tol
    assert float(np.max(np.abs(g - g_ref))) <= tol


def test_config3_circuits_at_20_qubits_vs_oracle():
    """HEA (10 layers) and QFT of a random basis state at 20 qubits on the
    fused engine: complex128 within 1e-12, complex64 within 1e-5 of the fp64
    oracle per amplitude (the complex64 error is printed)."""
    n = 20
    x = W.random_basis_index(n, 1004)
    prep = [W.Op("X", (), (q,)) for q in range(n) if (x >> q) & 1]
    th = W.uniform_angles(W.hea_n_params(n, 10), 1003)
    for name, ops, p in (("hea", W.hea_ops(n, 10), th), ("qft", prep + W.qft_ops(n), np.zeros(0))):
        ref = oracle.run_circuit(oracle.zero_state(n), ops, p)
        for dtype, tol in (("c128", 1e-12), ("c64", 1e-5)):
            b = sv.Batch([(n, ops, len(p), "sum_z")], dtype, with_grad=False)
            e, _ = b.run(p)
            err = float(np.max(np.abs(b.state(0).astype(np.complex128) - ref)))
            print(f"{name} n={n} {dtype}: max |psi - psi_oracle| = {err:.2e}, passes {b.info()['passes']}", flush=True)
            assert err <= tol, (name, dtype, err)
            assert abs(e[0] - oracle.expval_obs(ref, W.sum_z(n))) <= tol * n


def far_control_runs(n, rng, reps):
    """Runs of one-target gates on a target t whose controls are qubits far
    from it (at or above n - 4, outside a tile of the low qubits), mixed with
    uncontrolled gates: with a small tile the forward passes fuse each run into
    one 2x2 per tile, chosen by the tile's values of those qubits.  CNOTs with
    one or two far controls, controlled rotations and phases, uncontrolled
    rotations, H and U2; each parameterised gate has a parameter of its own.
    Returns (ops, number of parameters)."""
    ops = []
    n_params = 0
    far = list(range(n - 4, n))
    for _ in range(reps):
        t = int(rng.integers(0, n - 4))
        for _ in range(int(rng.integers(3, 9))):
            k = int(rng.integers(0, 7))
            ctl = tuple(int(x) for x in rng.choice(far, size=1 + (k == 1), replace=False))
            v = float(rng.uniform(0, 2 * math.pi))
            if k <= 1:
                ops.append(W.Op("X", ctl, (t,)))
            elif k == 2:
                ops.append(W.Op("RY", ctl, (t,), -1, v))
            elif k == 3:
                ops.append(W.Op("PHASE" if v < math.pi else "RZ", ctl, (t,), -1, v))
            elif k == 4:
                ops.append(W.Op("RZ", (), (t,), n_params, v))
                n_params += 1
            elif k == 5:
                ops.append(W.Op("H", (), (t,)))
            else:
                ops.append(W.Op("U2", (), (t,), -1, 0.0, W.haar_unitary(1, rng)))
    return ops, n_params


@pytest.mark.parametrize("apt", [16, 8])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("tile", [3, 4, 6])
def test_tile_selected_fusion_states_and_energies(dtype, tile, apt):
    # tile 3 with 16 amplitudes per thread runs the LDS-sweep form
    rng = np.random.default_rng(5400 + tile)
    circs, params, n_gates = [], [], 0
    for n in (8, 11):
        ops, npar = far_control_runs(n, rng, 12)
        n_gates += len(ops)
        circs.append((n, ops, npar, "sum_zz"))
        params.append(rng.uniform(0, 2 * math.pi, size=npar))
    b = sv.Batch(circs, dtype, tile_qubits=tile, amps_per_thread=apt, with_grad=False)
    e, _ = b.run(np.concatenate(params))
    assert b.info()["fused_ops"] < n_gates // 2  # runs of 3-8 gates became one op each
    for i, (n, ops, npar, obs) in enumerate(circs):
        ref = oracle.run_circuit(oracle.zero_state(n), ops, params[i])
        got = b.state(i).astype(np.complex128)
        err = float(np.max(np.abs(got - ref)))
        assert err <= 4 * TOL[dtype], (i, n, err)
        e_ref = oracle.expval_obs(ref, obs_terms(obs, n))
        assert abs(e[i] - e_ref) <= 4 * TOL[dtype] * n, (i, e[i], e_ref)


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-10), ("c64", 1e-4)])
def test_tile_selected_fusion_gradients_vs_oracle(dtype, tol):
    # with the adjoint: forward passes fused per tile, reverse passes gate by gate
    rng = np.random.default_rng(5500)
    n = 10
    ops, npar = far_control_runs(n, rng, 10)
    th = rng.uniform(0, 2 * math.pi, size=npar)
    b = sv.Batch([(n, ops, npar, "sum_z")], dtype, tile_qubits=5, with_grad=True)
    e, g = b.run(th)
    g_ref = oracle.param_shift_grad(n, ops, th, W.sum_z(n))
    assert abs(e[0] - oracle.energy(n, ops, th, W.sum_z(n))) <= tol * n
    assert float(np.max(np.abs(g - g_ref))) <= tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_universal_circuit_fused_and_op_by_op_vs_oracle(dtype):
    """The universal circuit (2 n^2 gates: CNOTs and Z rotations) after an H on
    every qubit, at 10 qubits: fused engine and op-by-op kernels against the
    oracle on the same op list (its gate order is one reading of the paper;
    the comparison pins the kernels, not that reading)."""
    n = 10
    ops = [W.Op("H", (), (q,)) for q in range(n)] + W.universal_ops(n)
    ref = oracle.run_circuit(oracle.zero_state(n), ops, np.zeros(0))
    b = sv.Batch([(n, ops, 0, "sum_zz")], dtype, with_grad=False)
    e, _ = b.run([])
    err = float(np.max(np.abs(b.state(0).astype(np.complex128) - ref)))
    assert err <= 4 * TOL[dtype], err
    assert abs(e[0] - oracle.expval_obs(ref, W.sum_zz(n))) <= 4 * TOL[dtype] * n
    st = sv.State(n, dtype)
    sv.Circuit(n, ops, 0).apply(st)
    err2 = float(np.max(np.abs(st.numpy().astype(np.complex128) - ref)))
    assert err2 <= 4 * TOL[dtype], err2


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-10), ("c64", 1e-4)])
def test_batch_tiny_and_empty_circuits_with_gradients_device_io(dtype, tol):
    """1- and 2-qubit circuits (tiles below a register tile: the LDS-sweep
    form), a circuit with no ops, and a larger one in the same batch; inputs
    and outputs in device memory (run_device)."""
    import torch
    rng = np.random.default_rng(5505)
    circs = [(1, [W.Op("RY", (), (0,), 0), W.Op("RZ", (), (0,), 1)], 2, "sum_z"),
             (2, [W.Op("RX", (), (1,), 0), W.Op("X", (1,), (0,)), W.Op("PHASE", (0,), (1,), 1)], 2, "sum_zz"),
             (3, [], 0, "sum_z"),
             (8, W.hea_ops(8, 2), W.hea_n_params(8, 2), "sum_zz")]
    params = [rng.uniform(0, 2 * math.pi, size=c[2]) for c in circs]
    b = sv.Batch(circs, dtype, with_grad=True)
    p = torch.as_tensor(np.concatenate(params), device="cuda", dtype=torch.float64)
    e = torch.zeros(len(circs), device="cuda", dtype=torch.float64)
    g = torch.zeros(max(1, sum(c[2] for c in circs)), device="cuda", dtype=torch.float64)
    b.run_device(p, e, g)
    e, g = e.cpu().numpy(), g.cpu().numpy()
    off = 0
    for i, (n, ops, npar, obs) in enumerate(circs):
        terms = obs_terms(obs, n)
        e_ref = oracle.energy(n, ops, params[i], terms)
        assert abs(e[i] - e_ref) <= tol, (i, e[i], e_ref)
        if npar:
            g_ref = oracle.fd_grad(n, ops, params[i], terms)
            assert np.max(np.abs(g[off:off + npar] - g_ref)) <= max(tol, 1e-7), (i, g[off:off + npar], g_ref)
        off += npar
    assert e[2] == 3.0  # |000>: sum Z = 3 exactly
