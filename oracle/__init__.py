"""The oracle: a plain, slow, obviously correct CPU simulator in fp64.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package.  It shares no code with the
HIP library (``paper_2508_13615_amd``) and neither imports the other; the two
meet only through the seeded inputs of ``workloads.py``.

Method (Kang & Ryu, arXiv 2508.13615):
  * Sec. 2: a state is 2^N complex amplitudes; a gate is its small logic matrix
    applied to each group of amplitudes that differ only in the gate's qubits;
    a control bit only selects where the gate acts.  The dense product (the
    "general approach" of Sec. 3.1) is the plain definition that the
    gate-specific kernels must reproduce, so the oracle applies every
    non-permutation gate densely (``sv_oracle.c: oracle_apply_matrix``).
  * Permutation gates (X and SWAP, any controls) are applied by explicit
    element moves so that bit-exact comparison is meaningful in complex64 and
    complex128 alike.
  * Expectation values follow their definition <psi|P|psi>.
  * Gradients (the project's adjoint differentiation is checked against
    these): the two-term parameter-shift rule, exact for gates exp(-i th G)
    whose generator G has two eigenvalues one unit apart in th-units
    (RX/RY/RZ/PHASE, controlled PHASE), and central finite differences.

Gate definitions (the paper names the gates but not their conventions; the
readings are: rotations are exp(-i th P / 2), PHASE(phi) = diag(1, e^{i phi}),
the first-listed target is the most significant bit of a matrix index).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv_oracle.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (fp64, no fast-math, no FP contraction)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O3", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB_PATH + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.c_void_p
        lib.oracle_apply_matrix.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, ip, ctypes.c_int, dp]
        lib.oracle_move_x.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int, ctypes.c_int]
        lib.oracle_move_swap.argtypes = [dp, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int]
        lib.oracle_inner.argtypes = [dp, dp, ctypes.c_int, dp]
        lib.oracle_expval_pauli.argtypes = [dp, ctypes.c_int, ctypes.c_char_p, ip, ctypes.c_int, dp]
        for f in ("oracle_apply_matrix", "oracle_move_x", "oracle_move_swap", "oracle_inner",
                  "oracle_expval_pauli", "oracle_version", "oracle_num_threads"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _ints(seq: Sequence[int]):
    arr = (ctypes.c_int * max(1, len(seq)))(*[int(q) for q in seq])
    return arr


def _n_of(psi: np.ndarray) -> int:
    n = int(psi.size).bit_length() - 1
    if psi.ndim != 1 or (1 << n) != psi.size:
        raise ValueError("state length must be a power of two")
    return n


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


# ---------------------------------------------------------------------------
# gate definitions
# ---------------------------------------------------------------------------
_R2 = math.sqrt(0.5)  # correctly rounded 2^(-1/2), the H entry


def gate_matrix(name: str, params: Sequence[float] = (), matrix=None) -> np.ndarray:
    """Logic matrix of a named gate (targets only; controls are separate)."""
    if name == "I":
        return np.eye(2, dtype=np.complex128)
    if name == "X":
        return np.array([[0, 1], [1, 0]], dtype=np.complex128)
    if name == "Y":
        return np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    if name == "Z":
        return np.array([[1, 0], [0, -1]], dtype=np.complex128)
    if name == "H":
        return np.array([[_R2, _R2], [_R2, -_R2]], dtype=np.complex128)
    if name == "S":
        return np.array([[1, 0], [0, 1j]], dtype=np.complex128)
    if name == "T":
        return np.array([[1, 0], [0, complex(math.cos(math.pi / 4), math.sin(math.pi / 4))]],
                        dtype=np.complex128)
    if name in ("RX", "RY", "RZ", "PHASE"):
        th = float(params[0])
        c, s = math.cos(th / 2.0), math.sin(th / 2.0)
        if name == "RX":
            return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
        if name == "RY":
            return np.array([[c, -s], [s, c]], dtype=np.complex128)
        if name == "RZ":
            return np.array([[complex(c, -s), 0], [0, complex(c, s)]], dtype=np.complex128)
        return np.array([[1, 0], [0, complex(math.cos(th), math.sin(th))]], dtype=np.complex128)
    if name == "SWAP":
        m = np.zeros((4, 4), dtype=np.complex128)
        m[0, 0] = m[3, 3] = m[1, 2] = m[2, 1] = 1
        return m
    if name in ("U2", "U4", "GENERAL"):
        return np.ascontiguousarray(np.asarray(matrix, dtype=np.complex128))
    raise ValueError(f"unknown gate {name}")


def n_targets(name: str, matrix=None) -> int:
    if name == "SWAP" or name == "U4":
        return 2
    if name == "GENERAL":
        return int(np.asarray(matrix).shape[0]).bit_length() - 1
    return 1


# ---------------------------------------------------------------------------
# state operations
# ---------------------------------------------------------------------------
def num_threads() -> int:
    """OpenMP threads the oracle's group loops use."""
    return int(_load().oracle_num_threads())


def zero_state(n: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    return psi


def basis_state(n: int, x: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[x] = 1.0
    return psi


def apply_matrix(psi: np.ndarray, targets: Sequence[int], U: np.ndarray,
                 controls: Sequence[int] = ()) -> np.ndarray:
    """Dense definition, in place (psi must be contiguous complex128)."""
    assert psi.dtype == np.complex128 and psi.flags.c_contiguous
    U = np.ascontiguousarray(U, dtype=np.complex128)
    k = len(targets)
    if U.shape != (1 << k, 1 << k):
        raise ValueError("matrix shape does not match the number of targets")
    rc = _load().oracle_apply_matrix(psi.ctypes.data, _n_of(psi), _ints(controls), len(controls),
                                     _ints(targets), k, U.ctypes.data)
    _check(rc, "apply_matrix")
    return psi


def move_x(psi: np.ndarray, t: int, controls: Sequence[int] = ()) -> np.ndarray:
    assert psi.dtype in (np.complex128, np.complex64) and psi.flags.c_contiguous
    rc = _load().oracle_move_x(psi.ctypes.data, psi.itemsize, _n_of(psi), _ints(controls),
                               len(controls), int(t))
    _check(rc, "move_x")
    return psi


def move_swap(psi: np.ndarray, a: int, b: int, controls: Sequence[int] = ()) -> np.ndarray:
    assert psi.dtype in (np.complex128, np.complex64) and psi.flags.c_contiguous
    rc = _load().oracle_move_swap(psi.ctypes.data, psi.itemsize, _n_of(psi), _ints(controls),
                                  len(controls), int(a), int(b))
    _check(rc, "move_swap")
    return psi


def apply_gate(psi: np.ndarray, name: str, targets: Sequence[int], controls: Sequence[int] = (),
               params: Sequence[float] = (), matrix=None) -> np.ndarray:
    """Apply one gate in place: X and SWAP as moves, all else by the dense
    definition.  complex64 states are accepted for the move gates only."""
    if name == "X":
        return move_x(psi, targets[0], controls)
    if name == "SWAP":
        return move_swap(psi, targets[0], targets[1], controls)
    return apply_matrix(psi, targets, gate_matrix(name, params, matrix), controls)


def op_params(op, params) -> Tuple[float, ...]:
    if op.gate in ("RX", "RY", "RZ", "PHASE"):
        return (float(params[op.pidx]) if op.pidx >= 0 else float(op.value),)
    return ()


def run_circuit(psi: np.ndarray, ops: Iterable, params: Optional[Sequence[float]] = None) -> np.ndarray:
    for op in ops:
        apply_gate(psi, op.gate, op.targets, op.controls, op_params(op, params), op.matrix)
    return psi


def inner(phi: np.ndarray, chi: np.ndarray) -> complex:
    out = (ctypes.c_double * 2)()
    rc = _load().oracle_inner(phi.ctypes.data, chi.ctypes.data, _n_of(phi), out)
    _check(rc, "inner")
    return complex(out[0], out[1])


def norm2(psi: np.ndarray) -> float:
    return inner(psi, psi).real


def expval_pauli(psi: np.ndarray, paulis: str, qubits: Sequence[int]) -> complex:
    out = (ctypes.c_double * 2)()
    rc = _load().oracle_expval_pauli(psi.ctypes.data, _n_of(psi), paulis.encode(), _ints(qubits),
                                     len(qubits), out)
    _check(rc, "expval_pauli")
    return complex(out[0], out[1])


def expval_obs(psi: np.ndarray, terms) -> float:
    """sum_k c_k <psi|P_k|psi> over a Pauli-sum observable, terms in order."""
    e = 0.0
    for coeff, paulis, qubits in terms:
        e = e + float(coeff) * expval_pauli(psi, paulis, qubits).real
    return e


def energy(n: int, ops, params, terms, init: Optional[np.ndarray] = None) -> float:
    psi = zero_state(n) if init is None else np.array(init, dtype=np.complex128, copy=True)
    run_circuit(psi, ops, params)
    return expval_obs(psi, terms)


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------
_SHIFT_OK = ("RX", "RY", "RZ", "PHASE")


def param_shift_grad(n: int, ops, params, terms, which: Optional[Sequence[int]] = None,
                     init: Optional[np.ndarray] = None) -> np.ndarray:
    """dE/dth_j = [E(th_j + pi/2) - E(th_j - pi/2)] / 2, for every slot j.

    Exact for exp(-i th P/2) (RX/RY/RZ) and for PHASE / controlled PHASE
    (generator with eigenvalues {0, 1}); controlled Pauli rotations have three
    generator eigenvalues, so the two-term rule does not hold for them and they
    are rejected here (use ``fd_grad``)."""
    params = np.asarray(params, dtype=np.float64)
    for op in ops:
        if op.pidx >= 0 and (op.gate not in _SHIFT_OK or (op.controls and op.gate != "PHASE")):
            raise ValueError(f"two-term parameter shift does not apply to {op.gate} with controls")
    idx = range(len(params)) if which is None else which
    g = np.zeros(len(params))
    for j in idx:
        p = params.copy()
        p[j] = params[j] + math.pi / 2
        ep = energy(n, ops, p, terms, init)
        p[j] = params[j] - math.pi / 2
        em = energy(n, ops, p, terms, init)
        g[j] = (ep - em) / 2.0
    return g


def fd_grad(n: int, ops, params, terms, h: float = 1e-6, which: Optional[Sequence[int]] = None,
            init: Optional[np.ndarray] = None) -> np.ndarray:
    """Central finite differences [E(th+h) - E(th-h)] / (2h)."""
    params = np.asarray(params, dtype=np.float64)
    idx = range(len(params)) if which is None else which
    g = np.zeros(len(params))
    for j in idx:
        p = params.copy()
        p[j] = params[j] + h
        ep = energy(n, ops, p, terms, init)
        p[j] = params[j] - h
        em = energy(n, ops, p, terms, init)
        g[j] = (ep - em) / (2.0 * h)
    return g
