"""The fused engine at the benchmark's full size (32 qubits: 64 GiB complex128,
32 GiB complex64), in the benchmark's launch configuration (default tile,
default register width), checked on sampled amplitudes through properties
that hold at any size:

- QFT of a basis state x: every amplitude equals 2^{-n/2} exp(2 pi i x rev(y) / 2^n)
  (closed form of the circuit without swaps);
- the universal circuit after an H on every qubit: CNOTs permute and Z
  rotations rotate phases, so every amplitude keeps magnitude 2^{-n/2};
- the 10-layer HEA: the fused engine and the op-by-op single-gate kernels
  (two independent code paths, each pinned to the oracle at small sizes)
  agree on sampled amplitudes and on the energy, and the norm stays 1.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

sv = pytest.importorskip("paper_2508_13615_amd")

N = 32
SAMPLES = 4096


def _rev(y, n):
    return int(format(y, f"0{n}b")[::-1], 2)


def _sample_idx(seed):
    rng = np.random.default_rng(seed)
    return np.unique(rng.integers(0, 1 << N, size=SAMPLES, dtype=np.int64))


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-13), ("c64", 2e-9)])
def test_qft32_closed_form_sampled(dtype, tol):
    x = W.random_basis_index(N, 1004)
    prep = [W.Op("X", (), (q,)) for q in range(N) if (x >> q) & 1]
    b = sv.Batch([(N, prep + W.qft_ops(N), 0, "sum_z")], dtype, with_grad=False)
    e, _ = b.run([])
    idx = _sample_idx(7)
    got = b.state_tensor(0)[torch.as_tensor(idx, device="cuda")].cpu().numpy().astype(np.complex128)
    want = np.array([math.pow(2.0, -N / 2) * np.exp(2j * math.pi * ((x * _rev(int(y), N)) % (1 << N)) / (1 << N))
                     for y in idx])
    err = float(np.max(np.abs(got - want)))
    print(f"qft32 {dtype}: max sampled error {err:.2e} (amplitudes {2.0 ** (-N / 2):.2e}), E = {e[0]:.3e}", flush=True)
    assert err <= tol, err
    # uniform magnitudes: sum Z_i = 0 in exact arithmetic; bar 1e-12 (c128) or
    # 1e-5 (c64) per term, the expectation tolerances of the parity tests
    assert abs(e[0]) <= (1e-5 if dtype == "c64" else 1e-12) * N, e[0]
    del b
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-15), ("c64", 2e-10)])
def test_universal32_magnitudes_sampled(dtype, tol):
    ops = [W.Op("H", (), (q,)) for q in range(N)] + W.universal_ops(N)
    b = sv.Batch([(N, ops, 0, "sum_z")], dtype, with_grad=False)
    b.run([])
    idx = _sample_idx(8)
    got = b.state_tensor(0)[torch.as_tensor(idx, device="cuda")].cpu().numpy().astype(np.complex128)
    err = float(np.max(np.abs(np.abs(got) - 2.0 ** (-N / 2))))
    print(f"universal32 {dtype}: max | |amp| - 2^-16 | = {err:.2e}", flush=True)
    assert err <= tol, err
    del b
    torch.cuda.empty_cache()


def test_hea32_fused_equals_op_by_op_sampled():
    ops = W.hea_ops(N, 10)
    th = W.uniform_angles(W.hea_n_params(N, 10), 1003)
    b = sv.Batch([(N, ops, len(th), "sum_z")], "c128", with_grad=False)
    e_fused = b.run(th)[0][0]
    idx = torch.as_tensor(_sample_idx(9), device="cuda")
    fused = b.state_tensor(0)
    f_norm = float(torch.linalg.vector_norm(fused).item())
    f_samp = fused[idx].cpu().numpy()
    del fused, b
    torch.cuda.empty_cache()
    st = sv.State(N, "c128")
    sv.Circuit(N, ops, len(th)).apply(st, th)
    o_samp = st.tensor[idx].cpu().numpy()
    e_op = st.expval(W.sum_z(N))
    err = float(np.max(np.abs(f_samp - o_samp)))
    scale = float(np.max(np.abs(o_samp)))
    print(f"hea32: fused vs op-by-op max sampled error {err:.2e} (max |amp| {scale:.2e}); "
          f"E {e_fused:.12f} vs {e_op:.12f}; fused norm {f_norm:.15f}", flush=True)
    assert err <= 1e-12 * max(1.0, scale * 1e4)
    assert abs(e_fused - e_op) <= 1e-10
    assert abs(f_norm - 1.0) <= 1e-12
    del st
    torch.cuda.empty_cache()
