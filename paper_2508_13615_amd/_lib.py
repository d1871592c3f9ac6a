"""ctypes declarations of libsv's C ABI (include/sv.h).  Marshalling only.

torch is imported before the library is loaded so that libsv's dependency on
libamdhip64.so.7 resolves to the HIP runtime torch has already mapped: one
runtime per process, so torch streams and allocations are valid in libsv.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede loading libsv, see above)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsv.so")

SV_C64, SV_C128 = 1, 2
STATUS = {0: "SV_OK", 1: "SV_ERR_ARG", 2: "SV_ERR_QUBIT", 3: "SV_ERR_OOM", 4: "SV_ERR_HIP",
          5: "SV_ERR_UNSUPPORTED", 6: "SV_ERR_HANDLE"}
GATES = {"I": 0, "X": 1, "Y": 2, "Z": 3, "H": 4, "S": 5, "T": 6, "RX": 7, "RY": 8, "RZ": 9,
         "PHASE": 10, "SWAP": 11, "U2": 12, "U4": 13}
OP_MAX_QUBITS = 10

# Every symbol include/sv.h declares (the CPU test checks the library exports them).
EXPORTS = [
    "sv_alloc", "sv_wrap", "sv_free", "sv_set_stream", "sv_get_info", "sv_state_bytes", "sv_set_basis",
    "sv_copy_to_host", "sv_copy_from_host", "sv_copy_state", "sv_synchronize", "sv_apply_gate",
    "sv_apply_controlled", "sv_apply_general", "sv_apply_dense", "sv_apply_phases", "sv_norm2", "sv_expval_pauli",
    "sv_expval_obs", "sv_expval_obs_dev", "sv_expval_obs_dev_noalloc", "sv_expval_pauli_dev", "sv_circuit_create", "sv_circuit_free", "sv_circuit_apply",
    "sv_circuit_apply_fused", "sv_circuit_apply_blocks", "sv_block_plan", "sv_adjoint_grad",
    "sv_batch_create", "sv_batch_plan", "sv_batch_run", "sv_batch_info", "sv_batch_state", "sv_batch_copy_state",
    "sv_batch_free", "sv_batch_set_stream",
    "sv_tune_set", "sv_tune_get", "sv_tune_engine_set", "sv_tune_engine_get", "sv_set_block_order",
    "sv_get_block_order", "sv_plan_info", "sv_last_error", "sv_status_string", "sv_version", "sv_stream_bench",
]


class SvObs(ctypes.Structure):
    _fields_ = [("n_terms", ctypes.c_int), ("coeffs", ctypes.POINTER(ctypes.c_double)),
                ("xmask", ctypes.POINTER(ctypes.c_uint64)), ("zmask", ctypes.POINTER(ctypes.c_uint64))]


class SvOp(ctypes.Structure):
    _fields_ = [("gate", ctypes.c_int32), ("n_controls", ctypes.c_int32), ("n_targets", ctypes.c_int32),
                ("param_index", ctypes.c_int32), ("qubits", ctypes.c_int32 * OP_MAX_QUBITS),
                ("value", ctypes.c_double), ("matrix", ctypes.POINTER(ctypes.c_double))]


class SvBatchCircuit(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_ops", ctypes.c_int32), ("ops", ctypes.POINTER(SvOp)),
                ("n_params", ctypes.c_int32), ("obs_kind", ctypes.c_int32)]


class SvBatchOpts(ctypes.Structure):
    _fields_ = [("tile_qubits", ctypes.c_int32), ("amps_per_thread", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("with_grad", ctypes.c_int32)]


class SvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                          "(the HIP library is required; there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d, u64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_uint64
    ip, dp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    sig = {
        "sv_alloc": [i, i, vp, ctypes.POINTER(vp)],
        "sv_wrap": [vp, i, i, vp, ctypes.POINTER(vp)],
        "sv_free": [vp],
        "sv_set_stream": [vp, vp],
        "sv_get_info": [vp, ip, ip, ctypes.POINTER(vp)],
        "sv_set_basis": [vp, u64],
        "sv_copy_to_host": [vp, vp, ctypes.c_size_t],
        "sv_copy_from_host": [vp, vp, ctypes.c_size_t],
        "sv_copy_state": [vp, vp],
        "sv_synchronize": [vp],
        "sv_apply_gate": [vp, i, ip, i, dp, dp, i],
        "sv_apply_controlled": [vp, i, ip, i, ip, i, dp, dp, i],
        "sv_apply_general": [vp, ip, i, dp],
        "sv_apply_dense": [vp, ip, i, dp],
        "sv_apply_phases": [vp, i, ctypes.POINTER(ctypes.c_uint64), dp],
        "sv_norm2": [vp, dp],
        "sv_expval_pauli": [vp, ctypes.c_char_p, ip, i, dp],
        "sv_expval_obs": [vp, ctypes.POINTER(SvObs), dp],
        "sv_expval_obs_dev": [vp, ctypes.POINTER(SvObs), vp],
        "sv_expval_pauli_dev": [vp, ctypes.c_char_p, ip, i, vp],
        "sv_expval_obs_dev_noalloc": [vp, ctypes.POINTER(SvObs), vp],
        "sv_circuit_create": [i, ctypes.POINTER(SvOp), i, i, ctypes.POINTER(vp)],
        "sv_circuit_free": [vp],
        "sv_circuit_apply": [vp, vp, dp],
        "sv_circuit_apply_fused": [vp, vp, dp],
        "sv_circuit_apply_blocks": [vp, vp, dp, i, ip],
        "sv_block_plan": [i, ctypes.POINTER(SvOp), i, i, ctypes.POINTER(ctypes.c_int64)],
        "sv_adjoint_grad": [vp, vp, vp, dp, ctypes.POINTER(SvObs), dp, dp],
        "sv_batch_create": [ctypes.POINTER(SvBatchCircuit), i, i, ctypes.POINTER(SvBatchOpts), ctypes.POINTER(vp)],
        "sv_batch_free": [vp],
        "sv_batch_plan": [ctypes.POINTER(SvBatchCircuit), i, i, ctypes.POINTER(SvBatchOpts),
                          ctypes.POINTER(ctypes.c_int64)],
        "sv_batch_run": [vp, vp, i, vp, vp, i],
        "sv_batch_set_stream": [vp, vp],
        "sv_batch_info": [vp, ctypes.POINTER(ctypes.c_int64)],
        "sv_batch_state": [vp, i, ctypes.POINTER(vp), ip],
        "sv_batch_copy_state": [vp, i, vp, ctypes.c_size_t],
        "sv_tune_set": [i, i, i, i, i, i],
        "sv_tune_get": [i, i, i, ip, ip, ip],
        "sv_set_block_order": [i],
        "sv_get_block_order": [ip],
        "sv_tune_engine_set": [i, i, i, i],
        "sv_tune_engine_get": [i, i, ip, ip],
        "sv_plan_info": [i, i, i, ip, i, ip, i, ip, ip, ip, ip, ip, ip],
        "sv_stream_bench": [i, vp, vp, ctypes.c_size_t, i, i, vp],
    }
    for name, args in sig.items():
        if hasattr(lib, name):
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
    lib.sv_state_bytes.argtypes = [i, i]
    lib.sv_state_bytes.restype = ctypes.c_size_t
    lib.sv_last_error.restype = ctypes.c_char_p
    lib.sv_status_string.argtypes = [i]
    lib.sv_status_string.restype = ctypes.c_char_p
    lib.sv_version.restype = ctypes.c_int
    return lib


lib = _load()


def check(status: int) -> None:
    if status != 0:
        raise SvError(status, lib.sv_last_error().decode())
