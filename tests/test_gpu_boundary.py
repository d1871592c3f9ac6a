"""GPU tests of the boundary's owning and failure paths, the device-output
measurement, the batch's ordering against the caller's stream and the
streaming kernel that measures the HBM ceiling.  Every call goes through the
C ABI (ctypes) or its thin binding.

Bars: complex128 amplitudes within 1e-12 of the fp64 oracle; expectations
within 1e-12 per term; moves and copies bit-exact.
"""
import ctypes
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

sv = pytest.importorskip("paper_2508_13615_amd")
torch = pytest.importorskip("torch")
from paper_2508_13615_amd import _lib  # noqa: E402

lib = sv.lib
OK, ARG, QUBIT, OOM, HIP, UNSUP, HANDLE = range(7)


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ints(*q):
    return (ctypes.c_int * max(1, len(q)))(*q)


@pytest.mark.parametrize("dtype,code,tol", [("c128", 2, 1e-12), ("c64", 1, 1e-5)])
def test_owned_state_from_sv_alloc_vs_oracle(dtype, code, tol):
    # sv_alloc owns its memory and starts at |0...0>; gates on it match the oracle
    n = 11
    log(f"sv_alloc n={n} {dtype}")
    h = ctypes.c_void_p()
    assert lib.sv_alloc(n, code, None, ctypes.byref(h)) == OK
    try:
        nq, dt, ptr = ctypes.c_int(), ctypes.c_int(), ctypes.c_void_p()
        assert lib.sv_get_info(h, ctypes.byref(nq), ctypes.byref(dt), ctypes.byref(ptr)) == OK
        assert (nq.value, dt.value) == (n, code) and ptr.value
        npdt = np.complex128 if dtype == "c128" else np.complex64
        host = np.empty(1 << n, dtype=npdt)
        assert lib.sv_copy_to_host(h, host.ctypes.data_as(ctypes.c_void_p), host.nbytes) == OK
        assert host[0] == 1 and not np.any(host[1:])
        rng = np.random.default_rng(31)
        ref = oracle.zero_state(n)
        for gate, tg, ct in [("H", (0,), ()), ("H", (7,), ()), ("X", (3,), (0,)), ("RY", (9,), ()),
                             ("RZ", (3,), (7,)), ("SWAP", (10, 4), ()), ("PHASE", (9,), (0,)), ("U2", (5,), (3,))]:
            p = (ctypes.c_double * 1)(float(rng.uniform(0, 6.28)))
            m = W.haar_unitary(1, rng) if gate == "U2" else None
            mf = None
            if m is not None:
                mf = np.ascontiguousarray(m).view(np.float64).copy()
            rc = lib.sv_apply_controlled(h, _lib.GATES[gate], ints(*ct), len(ct), ints(*tg), len(tg), p,
                                         mf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if mf is not None else None, 0)
            assert rc == OK, lib.sv_last_error()
            oracle.apply_gate(ref, gate, tg, ct, (p[0],), m)
        assert lib.sv_copy_to_host(h, host.ctypes.data_as(ctypes.c_void_p), host.nbytes) == OK
        err = float(np.max(np.abs(host.astype(np.complex128) - ref)))
        log(f"  max err {err:.2e}")
        assert err <= tol
        out = ctypes.c_double()
        assert lib.sv_norm2(h, ctypes.byref(out)) == OK
        assert abs(out.value - 1.0) <= 10 * tol
    finally:
        assert lib.sv_free(h) == OK
    # the handle is gone, the memory released
    assert lib.sv_set_basis(h, 0) == HANDLE


def test_alloc_beyond_hbm_reports_oom_and_leaves_runtime_usable():
    # 36 qubits of complex128 is 1 TiB, beyond one MI355X's 288 GB
    h = ctypes.c_void_p()
    assert lib.sv_alloc(36, 2, None, ctypes.byref(h)) == OOM
    assert b"allocation" in lib.sv_last_error()
    assert lib.sv_alloc(4, 2, None, ctypes.byref(h)) == OK
    out = ctypes.c_double()
    assert lib.sv_norm2(h, ctypes.byref(out)) == OK and out.value == 1.0
    assert lib.sv_free(h) == OK


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 1e-5)])
def test_expval_pauli_dev_matches_host_and_oracle(dtype, tol):
    n = 10
    psi = W.gaussian_state(n, 77)
    psi_in = psi.astype(np.complex128 if dtype == "c128" else np.complex64)
    st = sv.State(n, dtype).load(psi_in)
    rng = np.random.default_rng(78)
    out = torch.zeros(40, dtype=torch.float64, device="cuda")
    strings = []
    for i in range(40):
        k = int(rng.integers(1, n + 1))
        qs = tuple(int(q) for q in rng.permutation(n)[:k])
        ps = "".join(rng.choice(list("IXYZ"), size=k))
        strings.append((ps, qs))
        st.expval_pauli_dev(ps, qs, out[i:i + 1])
    got = out.cpu().numpy()
    for i, (ps, qs) in enumerate(strings):
        host = st.expval_pauli(ps, qs)
        assert got[i] == host, (ps, qs)  # same kernels, same fixed order
        ref = oracle.expval_pauli(psi_in.astype(np.complex128), ps, qs).real
        assert abs(got[i] - ref) <= tol, (ps, qs, got[i], ref)


def test_expval_pauli_dev_is_ordered_between_gates():
    # queued on the state's stream: each value sees exactly the gates before it
    n = 8
    st = sv.State(n, "c128")
    out = torch.full((4,), 7.0, dtype=torch.float64, device="cuda")
    st.expval_pauli_dev("Z", (3,), out[0:1])   # |0>: +1
    st.apply("X", (3,))
    st.expval_pauli_dev("Z", (3,), out[1:2])   # |1> on qubit 3: -1
    st.apply("H", (5,))
    st.expval_pauli_dev("X", (5,), out[2:3])   # |+>: +1
    st.expval_pauli_dev("ZZ", (3, 5), out[3:4])  # -1 * 0
    got = out.cpu().tolist()
    assert got[0] == 1.0 and got[1] == -1.0 and got[3] == 0.0
    assert abs(got[2] - 1.0) <= 1e-15  # 2 fl(2^-1/2)^2


def test_stream_bench_kernels_move_exact_bytes():
    # copy reproduces the source bit for bit, the in-place form negates its
    # buffer, write leaves zeros, read changes nothing; a ragged length (not a
    # multiple of a workgroup tile)
    for nvec in (1 << 20, 1000003, 37):
        src = torch.randn(2 * nvec, dtype=torch.float64, device="cuda")
        keep = src.clone()
        dst = torch.full_like(src, 3.0)
        for block, unroll in ((256, 4), (512, 8), (64, 1)):
            dst.fill_(3.0)
            sv.stream_bench(0, dst, src, nvec * 16, block, unroll)
            torch.cuda.synchronize()
            assert torch.equal(dst, src)
            sv.stream_bench(3, dst, None, nvec * 16, block, unroll)
            torch.cuda.synchronize()
            assert torch.equal(dst, -src)
            sv.stream_bench(1, None, src, nvec * 16, block, unroll)
            sv.stream_bench(2, dst, None, nvec * 16, block, unroll)
            torch.cuda.synchronize()
            assert torch.equal(src, keep)
            assert not torch.any(dst)


def test_batch_run_device_waits_for_the_callers_stream():
    # parameters are written on a side stream behind a long spin; the batch,
    # ordered against that stream, must see them (not the zeros before)
    import math
    n, L = 8, 3
    ops = W.hea_ops(n, L)
    npar = W.hea_n_params(n, L)
    th = W.uniform_angles(npar, 91)
    b = sv.Batch([(n, ops, npar, "sum_zz")], "c128", with_grad=True)
    e_ref, g_ref = b.run(th)
    side = torch.cuda.Stream()
    params = torch.zeros(npar, dtype=torch.float64, device="cuda")
    exp = torch.zeros(1, dtype=torch.float64, device="cuda")
    grads = torch.zeros(npar, dtype=torch.float64, device="cuda")
    host = torch.from_numpy(th).pin_memory()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        torch.cuda._sleep(50_000_000)  # about 20 ms of spinning on the side stream
        params.copy_(host, non_blocking=True)
        exp.fill_(math.nan)
        b.run_device(params, exp, grads)
        got_e = exp.clone()
        got_g = grads.clone()
    torch.cuda.synchronize()
    assert float(got_e[0]) == float(e_ref[0])
    assert np.array_equal(got_g.cpu().numpy(), g_ref)
