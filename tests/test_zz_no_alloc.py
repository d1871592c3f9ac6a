"""The allocation-free expectation entry point (sv_expval_obs_dev_noalloc)
against the allocating one (sv_expval_obs_dev), through the C ABI.

Both run the same kernels in the same order, so the values must agree bit for
bit; each is also checked against the fp64 oracle (1e-12 per term for
complex128, 1e-5 per term for complex64 widened to fp64).  Two calls in a
row, the second on a smaller state with fewer terms, so the second reuses the
static array the first filled.
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

lib = sv.lib
OK, ARG = 0, 1


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _obs(n, rng, n_diag, n_off):
    terms = []
    for _ in range(n_diag):
        k = int(rng.integers(1, n + 1))
        qs = tuple(int(q) for q in rng.permutation(n)[:k])
        terms.append((float(rng.normal()), "Z" * k, qs))
    for _ in range(n_off):
        k = int(rng.integers(1, n + 1))
        qs = tuple(int(q) for q in rng.permutation(n)[:k])
        letters = "".join(rng.choice(list("XYZ"), size=k))
        if set(letters) == {"Z"}:
            letters = "X" + letters[1:]
        terms.append((float(rng.normal()), letters, qs))
    return terms


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 1e-5)])
def test_noalloc_expval_equals_allocating_one_twice(dtype, tol):
    rng = np.random.default_rng(501)
    npdt = np.complex128 if dtype == "c128" else np.complex64
    # first call: 14 qubits, 70 diagonal terms (3 passes) + 20 off-diagonal;
    # second call: 9 qubits, 5 diagonal + 3 off-diagonal, then the closed form
    for n, nd, no in ((14, 70, 20), (9, 5, 3), (9, 0, 0)):
        log(f"noalloc n={n} diag={nd} off={no} {dtype}")
        psi = W.gaussian_state(n, 600 + n).astype(npdt)
        st = sv.State(n, dtype).load(psi)
        terms = _obs(n, rng, nd, no) if nd or no else W.sum_zz(n)
        obs = sv.Observable(terms)
        out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
        rc = lib.sv_expval_obs_dev_noalloc(st.handle, ctypes.byref(obs.c), ctypes.c_void_p(out.data_ptr()))
        assert rc == OK, lib.sv_last_error()
        rc = lib.sv_expval_obs_dev(st.handle, ctypes.byref(obs.c), ctypes.c_void_p(out.data_ptr() + 8))
        assert rc == OK, lib.sv_last_error()
        a, b = out.cpu().tolist()
        assert a == b, (a, b)
        ref = oracle.expval_obs(psi.astype(np.complex128), terms)
        assert abs(a - ref) <= tol * max(1, len(terms)), (a, ref)


def test_noalloc_rejects_more_passes_than_it_holds():
    n = 6
    st = sv.State(n, "c128")
    rng = np.random.default_rng(502)
    obs = sv.Observable(_obs(n, rng, 0, 65))  # 65 off-diagonal terms = 65 passes
    out = torch.full((1,), 5.0, dtype=torch.float64, device="cuda")
    assert lib.sv_expval_obs_dev_noalloc(st.handle, ctypes.byref(obs.c), ctypes.c_void_p(out.data_ptr())) == ARG
    assert b"passes" in lib.sv_last_error()
    torch.cuda.synchronize()
    assert out.item() == 5.0  # nothing launched
    obs = sv.Observable(_obs(n, rng, 0, 64))  # exactly the limit
    assert lib.sv_expval_obs_dev_noalloc(st.handle, ctypes.byref(obs.c), ctypes.c_void_p(out.data_ptr())) == OK
    ref = torch.zeros(1, dtype=torch.float64, device="cuda")
    st.expval_dev(obs, ref)
    assert out.item() == ref.item()
