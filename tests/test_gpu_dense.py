"""Dense 4- to 6-qubit blocks on the matrix cores (sv_apply_dense) against
the fp64 oracle: every block size in both dtypes, target orders ascending,
descending, scattered and at the top of the index; states smaller than one
16-group block; repeated calls that reuse the staging buffers; a 30-qubit
complex128 state checked on sampled groups.  Circuits packed into dense
blocks (sv_circuit_apply_blocks): random circuits of every gate kind against
the oracle, the QFT against its closed form, and the 32-qubit HEA against the
fused pass engine on sampled amplitudes."""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

sv = pytest.importorskip("paper_2508_13615_amd")
pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-5}


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _target_sets(k, n, rng):
    yield tuple(range(k))                       # lowest qubits, ascending
    yield tuple(range(k - 1, -1, -1))           # lowest, descending
    yield tuple(range(n - 1, n - 1 - k, -1))    # highest
    yield tuple(int(q) for q in rng.permutation(n)[:k])  # scattered
    yield (n - 1,) + tuple(range(k - 1))        # top and bottom together


def _input(n, dtype, seed):
    psi = W.gaussian_state(n, seed)
    # complex64 runs start from the complex64 rounding of the same state; the
    # oracle gets that rounded state in fp64
    return psi.astype(np.complex64).astype(np.complex128) if dtype == "c64" else psi


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [4, 5, 6])
def test_dense_block_vs_oracle(dtype, k):
    n = 12
    rng = np.random.default_rng(7000 + k)
    psi0 = _input(n, dtype, 7100 + k)
    for tg in _target_sets(k, n, rng):
        log(f"dense {dtype} k={k} targets {tg}")
        u = W.haar_unitary(k, rng)
        s = sv.State(n, dtype, basis=None).load(psi0)
        s.apply_dense(tg, u)
        got = s.numpy().astype(np.complex128)
        ref = oracle.apply_matrix(psi0.copy(), tg, u)
        err = float(np.max(np.abs(got - ref)))
        assert err <= TOL[dtype], (tg, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_dense_block_states_smaller_than_one_block(dtype):
    # 2^(n-k) groups < 16: the only 16-row block is partial (n = k: one group)
    rng = np.random.default_rng(7200)
    for k in (4, 5, 6):
        for n in (k, k + 1, k + 3):
            tg = tuple(int(q) for q in rng.permutation(n)[:k])
            log(f"dense {dtype} n={n} k={k} targets {tg}")
            psi0 = _input(n, dtype, 7300 + 10 * n + k)
            u = W.haar_unitary(k, rng)
            s = sv.State(n, dtype, basis=None).load(psi0)
            s.apply_dense(tg, u)
            err = float(np.max(np.abs(s.numpy().astype(np.complex128) - oracle.apply_matrix(psi0.copy(), tg, u))))
            assert err <= TOL[dtype], (n, k, tg, err)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_dense_blocks_back_to_back_and_mixed_with_gates(dtype):
    # several dense blocks of different sizes queued without a sync in
    # between, and gate-specific kernels between them, against the oracle
    # applying the same sequence
    n = 13
    rng = np.random.default_rng(7400)
    psi0 = _input(n, dtype, 7401)
    s = sv.State(n, dtype, basis=None).load(psi0)
    ref = psi0.copy()
    for step, k in enumerate((6, 4, 5, 6, 4)):
        tg = tuple(int(q) for q in rng.permutation(n)[:k])
        u = W.haar_unitary(k, rng)
        s.apply_dense(tg, u)
        ref = oracle.apply_matrix(ref, tg, u)
        s.apply("H", (step,))
        ref = oracle.apply_gate(ref, "H", (step,))
    err = float(np.max(np.abs(s.numpy().astype(np.complex128) - ref)))
    assert err <= 5 * TOL[dtype], err


def test_dense_kron_product_equals_one_qubit_kernels():
    # a dense block that is a Kronecker product of one-qubit gates gives the
    # state the one-qubit kernels give
    n = 14
    rng = np.random.default_rng(7500)
    psi0 = W.gaussian_state(n, 7501)
    tg = (13, 0, 7, 3, 10)
    us = [W.haar_unitary(1, rng) for _ in tg]
    big = us[0]
    for u in us[1:]:
        big = np.kron(big, u)
    a = sv.State(n, "c128", basis=None).load(psi0).apply_dense(tg, big).numpy()
    b = sv.State(n, "c128", basis=None).load(psi0)
    for t, u in zip(tg, us):
        b.apply("U2", (t,), matrix=u)
    assert np.max(np.abs(a - b.numpy())) <= 1e-12


def test_dense_full_size_sampled_30q():
    """30-qubit complex128 state (16 GiB): 512 sampled groups read before and
    after each block and compared with the oracle applied to each group."""
    import torch
    n = 30
    log("dense full size: allocating 30-qubit complex128 state")
    g = torch.Generator(device="cuda")
    g.manual_seed(7601)
    t = torch.randn(1 << n, dtype=torch.complex128, device="cuda", generator=g)
    t /= torch.linalg.vector_norm(t)
    s = sv.State(n, "c128", tensor=t, basis=None)
    rng = np.random.default_rng(7602)
    for tg in [(0, 1, 2, 3), (29, 3, 17, 0, 24, 9), (28, 27, 26, 25, 24), (5, 29, 11, 2)]:
        k = len(tg)
        log(f"  dense k={k} targets {tg}")
        u = W.haar_unitary(k, rng)
        free = rng.integers(0, 1 << n, size=512, dtype=np.int64)
        for q in tg:
            free &= ~(1 << q)
        members = []
        for r in range(1 << k):
            off = 0
            for j, q in enumerate(tg):
                if (r >> (k - 1 - j)) & 1:
                    off |= 1 << q
            members.append(free | off)
        idx = torch.from_numpy(np.stack(members, axis=1).reshape(-1)).cuda()
        before = t[idx].cpu().numpy().reshape(512, -1)
        s.apply_dense(tg, u)
        s.synchronize()
        after = t[idx].cpu().numpy().reshape(512, -1)
        for row in range(512):
            ref = oracle.apply_matrix(before[row].copy(), tuple(range(k - 1, -1, -1)), u)
            assert np.max(np.abs(after[row] - ref)) <= 1e-12, (tg, row)
    del s, t
    torch.cuda.empty_cache()


def _mixed_circuit(n, rng, count):
    ops, npar = [], 0
    for _ in range(count):
        q = [int(v) for v in rng.permutation(n)[:4]]
        r = rng.random()
        if r < 0.12:
            ops.append(W.Op("H", (), (q[0],)))
        elif r < 0.24:
            ops.append(W.Op("X", (q[1],), (q[0],)))
        elif r < 0.30:
            ops.append(W.Op("X", (q[1], q[2]), (q[0],)))  # Toffoli
        elif r < 0.40:
            ops.append(W.Op("RY", (), (q[0],), npar, 0.0))
            npar += 1
        elif r < 0.50:
            ops.append(W.Op("RZ", (q[1],), (q[0],), npar, 0.0))
            npar += 1
        elif r < 0.58:
            ops.append(W.Op("RX", (), (q[0],), npar, 0.0))
            npar += 1
        elif r < 0.66:
            ops.append(W.Op("PHASE", (q[1],), (q[0],), -1, float(rng.uniform(-3, 3))))
        elif r < 0.72:
            ops.append(W.Op("SWAP", (), (q[0], q[1])))
        elif r < 0.80:
            ops.append(W.Op("U4", (), (q[0], q[1]), -1, 0.0, W.haar_unitary(2, rng)))
        elif r < 0.88:
            ops.append(W.Op("U2", (q[2],), (q[0],), -1, 0.0, W.haar_unitary(1, rng)))
        else:
            ops.append(W.Op(["Y", "Z", "S", "T"][int(rng.integers(0, 4))], (), (q[0],)))
    return ops, npar


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_circuit_dense_blocks_vs_oracle(dtype):
    # random circuits of every gate kind, packed into 4-, 5- and 6-qubit
    # blocks, against the oracle; the block count is the host plan's
    n = 12
    rng = np.random.default_rng(7700)
    for trial, k in enumerate((4, 5, 6, 5)):
        ops, npar = _mixed_circuit(n, rng, 150)
        th = rng.uniform(0, 2 * np.pi, size=npar)
        psi0 = _input(n, dtype, 7710 + trial)
        circ = sv.Circuit(n, ops, npar)
        a = circ.apply(sv.State(n, dtype, basis=None).load(psi0), th, dense_block=k).numpy().astype(np.complex128)
        nb = circ.last_dense_blocks
        ref = oracle.run_circuit(psi0.copy(), ops, th)
        err = float(np.max(np.abs(a - ref)))
        log(f"blocks {dtype} k={k}: {nb} dense blocks for {len(ops)} ops, error {err:.2e}")
        assert nb == sv.block_plan(n, ops, k)["dense_blocks"]
        assert err <= 10 * TOL[dtype], (k, err)


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-13), ("c64", 2e-7)])
def test_qft_dense_blocks_closed_form(dtype, tol):
    import math
    n = 14
    x = W.random_basis_index(n, 7800)
    st = sv.State(n, dtype, basis=x)
    sv.Circuit(n, W.qft_ops(n), 0).apply(st, [], dense_block=5)
    got = st.numpy().astype(np.complex128)

    def rev(y):
        return int(format(y, f"0{n}b")[::-1], 2)
    want = np.array([math.pow(2.0, -n / 2) * np.exp(2j * math.pi * ((x * rev(v)) % (1 << n)) / (1 << n))
                     for v in range(1 << n)])
    assert float(np.max(np.abs(got - want))) <= tol


def test_hea32_dense_blocks_vs_engine_sampled():
    """The 32-qubit, 10-layer HEA (complex128, 64 GiB) as 5-qubit blocks on
    the matrix cores against the fused pass engine (an independent path, each
    pinned to the oracle at small sizes) on 4096 sampled amplitudes."""
    import torch
    n, L = 32, 10
    ops = W.hea_ops(n, L)
    th = W.uniform_angles(W.hea_n_params(n, L), 1003)
    idx = torch.as_tensor(np.unique(np.random.default_rng(7900).integers(0, 1 << n, size=4096, dtype=np.int64)),
                          device="cuda")
    log("hea32: fused engine")
    b = sv.Batch([(n, ops, len(th), "sum_z")], "c128", with_grad=False)
    b.run(th)
    ref = b.state_tensor(0)[idx].cpu().numpy()
    del b
    torch.cuda.empty_cache()
    log("hea32: dense blocks")
    st = sv.State(n, "c128", basis=0)
    sv.Circuit(n, ops, len(th)).apply(st, th, dense_block=5)
    got = st.tensor[idx].cpu().numpy()
    err = float(np.max(np.abs(got - ref)))
    log(f"hea32 blocks vs engine: max sampled difference {err:.2e}")
    assert err <= 1e-12, err
    del st
    torch.cuda.empty_cache()
