"""MI355X-native state-vector gate engine: Python binding over libsv (HIP).

Argument marshalling only: every step of gate application, measurement and
differentiation runs in libsv's HIP kernels (include/sv.h).  torch provides the
device memory (states are torch tensors wrapped by ``sv_wrap``) and the stream
(the current torch stream at wrap time).  There is no CPU fallback: importing
this package fails if libsv.so is not built, and every call on a machine
without a GPU reports SV_ERR_HIP.

Conventions (Kang & Ryu, arXiv 2508.13615, Sec. 2): qubit q is bit q of the
amplitude index; controls are 1-controls; matrices put the first-listed target
in the most significant bit of their index.
"""
from __future__ import annotations

import ctypes
import os
import sys
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np
import torch

from ._lib import (GATES, OP_MAX_QUBITS, SV_C64, SV_C128, SvBatchCircuit, SvBatchOpts, SvError, SvObs, SvOp,
                   check, lib)

__all__ = ["State", "Circuit", "Batch", "Observable", "AdjointExpval", "SvError", "lib", "tune_set", "tune_get",
           "plan_info", "batch_plan", "sv_version", "stream_bench", "set_block_order", "get_block_order"]

_TORCH_DT = {"c128": torch.complex128, "c64": torch.complex64}
_SV_DT = {"c128": SV_C128, "c64": SV_C64}


def _ints(seq: Sequence[int]):
    return (ctypes.c_int * max(1, len(seq)))(*[int(q) for q in seq])


def _dbl(seq):
    arr = np.ascontiguousarray(np.asarray(seq, dtype=np.float64).reshape(-1))
    return arr, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _matrix(m):
    if m is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
    flat = a.view(np.float64).reshape(-1).copy()
    return flat, flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def sv_version() -> int:
    return int(lib.sv_version())


def tune_set(kernel_class: int, dtype: str, tier: int, block: int, unroll: int, nt: int) -> None:
    check(lib.sv_tune_set(kernel_class, _SV_DT[dtype], tier, block, unroll, nt))


def tune_get(kernel_class: int, dtype: str, tier: int) -> Tuple[int, int, int]:
    b, u, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(lib.sv_tune_get(kernel_class, _SV_DT[dtype], tier, ctypes.byref(b), ctypes.byref(u), ctypes.byref(t)))
    return b.value, u.value, t.value


def set_block_order(order: int) -> None:
    """Workgroup walk order of the gate kernels: -1 picks per launch, 0 is
    launch order, 1 gives each XCD a contiguous eighth of the state."""
    check(lib.sv_set_block_order(int(order)))


def get_block_order() -> int:
    o = ctypes.c_int()
    check(lib.sv_get_block_order(ctypes.byref(o)))
    return o.value


def tune_engine_set(dtype: str, with_grad: bool, tile_qubits: int, amps_per_thread: int) -> None:
    """Fused-engine tile shape for batches of this dtype and stage mix created
    with the shape options at 0 (0 = built-in default)."""
    check(lib.sv_tune_engine_set(_SV_DT[dtype], int(bool(with_grad)), int(tile_qubits), int(amps_per_thread)))


def tune_engine_get(dtype: str, with_grad: bool) -> Tuple[int, int]:
    """(tile_qubits, amps_per_thread) a batch with default shape options gets."""
    t, a = ctypes.c_int(), ctypes.c_int()
    check(lib.sv_tune_engine_get(_SV_DT[dtype], int(bool(with_grad)), ctypes.byref(t), ctypes.byref(a)))
    return t.value, a.value


KERNEL_CLASSES = {0: "k_pair", 1: "k_one", 3: "k_quad", 4: "k_general", 5: "k_wpair", 6: "k_lds_gate"}


def stream_bench(mode: int, dst: Optional[torch.Tensor], src: Optional[torch.Tensor], nbytes: int, block: int = 256,
                 unroll: int = 4) -> None:
    """Queue the HBM-ceiling kernel on torch's current stream (sv_stream_bench):
    mode 0 copies src to dst, 1 reads src, 2 writes dst."""
    check(lib.sv_stream_bench(int(mode), ctypes.c_void_p(dst.data_ptr() if dst is not None else 0),
                              ctypes.c_void_p(src.data_ptr() if src is not None else 0), int(nbytes), int(block),
                              int(unroll), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))


def plan_info(n: int, dtype: str, gate: str, targets: Sequence[int], controls: Sequence[int] = ()) -> dict:
    """How libsv would launch a gate (host only).  gate = "GENERAL" asks about
    the dense baseline kernel on `targets`."""
    out = [ctypes.c_int() for _ in range(6)]
    g = -1 if gate == "GENERAL" else GATES[gate]
    check(lib.sv_plan_info(n, _SV_DT[dtype], g, _ints(controls), len(controls), _ints(targets), len(targets),
                           *[ctypes.byref(o) for o in out]))
    kc, tier, op, block, unroll, nt = (o.value for o in out)
    T = "double" if dtype == "c128" else "float"
    if kc == 3:
        name = f"{KERNEL_CLASSES[kc]}<{T}, {unroll}, {'true' if nt else 'false'}>"
    elif kc == 6:
        name = f"k_lds_gate<{T}, {op >> 4}, {op & 15}, {'true' if nt else 'false'}, {unroll}>"
    else:
        name = f"{KERNEL_CLASSES[kc]}<{T}, {op}, {unroll}, {'true' if nt else 'false'}>"
    return {"class": kc, "tier": tier, "op": op, "block": block, "unroll": unroll, "nt": nt, "kernel": name}


class Observable:
    """Pauli sum sum_k c_k P_k, terms given as (coeff, letters, qubits); marshalled
    into the sv_obs bit-mask form (X/Y positions in xmask, Z/Y in zmask)."""

    def __init__(self, terms: Iterable[Tuple[float, str, Sequence[int]]]):
        terms = list(terms)
        self.coeffs = np.array([float(t[0]) for t in terms] or [0.0], dtype=np.float64)
        xm, zm = [], []
        for _, letters, qubits in terms:
            x = z = 0
            for p, q in zip(letters, qubits):
                if p not in "IXYZ":
                    raise ValueError(f"bad Pauli letter {p!r}")
                if p in "XY":
                    x |= 1 << int(q)
                if p in "ZY":
                    z |= 1 << int(q)
            xm.append(x)
            zm.append(z)
        self.xmask = np.array(xm or [0], dtype=np.uint64)
        self.zmask = np.array(zm or [0], dtype=np.uint64)
        self.c = SvObs(len(terms), self.coeffs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       self.xmask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                       self.zmask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))


class State:
    """A 2^n state vector in a torch tensor on the current GPU, wrapped by libsv."""

    def __init__(self, n: int, dtype: str = "c128", tensor: Optional[torch.Tensor] = None,
                 stream: Optional[torch.cuda.Stream] = None, basis: Optional[int] = 0):
        if dtype not in _TORCH_DT:
            raise ValueError("dtype must be 'c128' or 'c64'")
        self.n, self.dtype = int(n), dtype
        if tensor is None:
            tensor = torch.empty(1 << self.n, dtype=_TORCH_DT[dtype], device="cuda")
        elif tensor.dtype != _TORCH_DT[dtype] or tensor.numel() != (1 << self.n) or not tensor.is_contiguous():
            raise ValueError("tensor must be a contiguous 2^n vector of the state dtype")
        self.tensor = tensor
        self.stream = stream if stream is not None else torch.cuda.current_stream(tensor.device)
        h = ctypes.c_void_p()
        check(lib.sv_wrap(ctypes.c_void_p(tensor.data_ptr()), self.n, _SV_DT[dtype],
                          ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        if basis is not None:
            self.set_basis(basis)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:
            lib.sv_free(h)
            self.handle = None

    # ---- data movement ---------------------------------------------------
    def set_basis(self, index: int) -> "State":
        check(lib.sv_set_basis(self.handle, int(index)))
        return self

    def load(self, host: np.ndarray) -> "State":
        a = np.ascontiguousarray(host, dtype=np.complex128 if self.dtype == "c128" else np.complex64)
        check(lib.sv_copy_from_host(self.handle, ctypes.c_void_p(a.ctypes.data), a.nbytes))
        return self

    def numpy(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=np.complex128 if self.dtype == "c128" else np.complex64)
        check(lib.sv_copy_to_host(self.handle, ctypes.c_void_p(out.ctypes.data), out.nbytes))
        return out

    def copy_from(self, other: "State") -> "State":
        check(lib.sv_copy_state(self.handle, other.handle))
        return self

    def synchronize(self) -> None:
        check(lib.sv_synchronize(self.handle))

    # ---- gates -------------------------------------------------------------
    def apply(self, gate: str, targets: Sequence[int], controls: Sequence[int] = (),
              params: Sequence[float] = (), matrix=None, adjoint: bool = False) -> "State":
        p, pp = _dbl(list(params) or [0.0])
        m, mp = _matrix(matrix)
        check(lib.sv_apply_controlled(self.handle, GATES[gate], _ints(controls), len(controls), _ints(targets),
                                      len(targets), pp, mp, int(bool(adjoint))))
        return self

    def apply_general(self, qubits: Sequence[int], matrix) -> "State":
        m, mp = _matrix(matrix)
        check(lib.sv_apply_general(self.handle, _ints(qubits), len(qubits), mp))
        return self

    def apply_phases(self, masks: Sequence[int], angles: Sequence[float]) -> "State":
        """psi[x] *= exp(i sum of angles[t] over the terms whose mask bits x contains) (sv_apply_phases)."""
        m = np.ascontiguousarray(np.asarray(masks, dtype=np.uint64))
        a = np.ascontiguousarray(np.asarray(angles, dtype=np.float64))
        if m.shape != a.shape:
            raise ValueError("one angle per mask")
        check(lib.sv_apply_phases(self.handle, len(m), m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                  a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return self

    def apply_dense(self, qubits: Sequence[int], matrix) -> "State":
        """Dense 2^k x 2^k unitary, 4 <= k <= 6, on the matrix cores (sv_apply_dense)."""
        m, mp = _matrix(matrix)
        check(lib.sv_apply_dense(self.handle, _ints(qubits), len(qubits), mp))
        return self

    # ---- measurement -------------------------------------------------------
    def norm2(self) -> float:
        out = ctypes.c_double()
        check(lib.sv_norm2(self.handle, ctypes.byref(out)))
        return out.value

    def expval_pauli(self, paulis: str, qubits: Sequence[int]) -> float:
        out = ctypes.c_double()
        check(lib.sv_expval_pauli(self.handle, paulis.encode(), _ints(qubits), len(qubits), ctypes.byref(out)))
        return out.value

    def expval(self, obs) -> float:
        obs = obs if isinstance(obs, Observable) else Observable(obs)
        out = ctypes.c_double()
        check(lib.sv_expval_obs(self.handle, ctypes.byref(obs.c), ctypes.byref(out)))
        return out.value

    def expval_dev(self, obs, out: torch.Tensor) -> None:
        obs = obs if isinstance(obs, Observable) else Observable(obs)
        check(lib.sv_expval_obs_dev(self.handle, ctypes.byref(obs.c), ctypes.c_void_p(out.data_ptr())))

    def expval_dev_noalloc(self, obs, out: torch.Tensor) -> None:
        """As expval_dev with no device allocation: the partials live in the
        library's static per-GPU array (sv_expval_obs_dev_noalloc; at most 64
        reduction passes; overlapping calls on one GPU race)."""
        obs = obs if isinstance(obs, Observable) else Observable(obs)
        check(lib.sv_expval_obs_dev_noalloc(self.handle, ctypes.byref(obs.c), ctypes.c_void_p(out.data_ptr())))

    def expval_pauli_dev(self, paulis: str, qubits: Sequence[int], out: torch.Tensor) -> None:
        """<psi|P|psi> of one Pauli string into out[0] (a float64 CUDA tensor),
        queued on the state's stream (sv_expval_pauli_dev)."""
        check(lib.sv_expval_pauli_dev(self.handle, paulis.encode(), _ints(qubits), len(qubits),
                                      ctypes.c_void_p(out.data_ptr())))


def _sv_op(op) -> Tuple[SvOp, Optional[np.ndarray]]:
    """workloads.Op -> sv_op (matrix kept alive by the caller)."""
    qs = list(op.controls) + list(op.targets)
    if len(qs) > OP_MAX_QUBITS:
        raise ValueError("too many qubits in one op")
    s = SvOp()
    s.gate = GATES[op.gate]
    s.n_controls = len(op.controls)
    s.n_targets = len(op.targets)
    s.param_index = int(op.pidx)
    for j, q in enumerate(qs):
        s.qubits[j] = int(q)
    s.value = float(op.value)
    keep = None
    if op.matrix is not None:
        keep, mp = _matrix(op.matrix)
        s.matrix = mp
    return s, keep


def block_plan(n: int, ops, k: int) -> dict:
    """How Circuit.apply(dense_block=k) packs an op list (host only, sv_block_plan)."""
    ops = list(ops)
    arr = (SvOp * max(1, len(ops)))()
    keep = []
    for i, op in enumerate(ops):
        arr[i], kp = _sv_op(op)
        keep.append(kp)
    a = (ctypes.c_int64 * 4)()
    check(lib.sv_block_plan(int(n), arr, len(ops), int(k), a))
    return dict(zip(["dense_blocks", "single_ops", "ops_in_dense", "widest"], list(a)))


class Circuit:
    """An op list bound into libsv (sv_circuit_create)."""

    def __init__(self, n: int, ops, n_params: int = 0):
        ops = list(ops)
        self.n, self.n_params = int(n), int(n_params)
        arr = (SvOp * max(1, len(ops)))()
        keep = []
        for i, op in enumerate(ops):
            arr[i], k = _sv_op(op)
            keep.append(k)
        h = ctypes.c_void_p()
        check(lib.sv_circuit_create(self.n, arr, len(ops), self.n_params, ctypes.byref(h)))
        self.handle = h
        self.n_ops = len(ops)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:
            lib.sv_circuit_free(h)
            self.handle = None

    def apply(self, state: State, params=(), fuse_diagonal: bool = False, dense_block: int = 0) -> State:
        """Apply op by op; with fuse_diagonal, each run of consecutive diagonal
        ops is one phase pass and consecutive one-target gates on one qubit
        one 2x2 (sv_circuit_apply_fused); with dense_block = k
        (4..6), the circuit runs as dense k-qubit blocks on the matrix cores
        (sv_circuit_apply_blocks)."""
        p, pp = _dbl(list(params) if len(params) else [0.0])
        if dense_block:
            nb = ctypes.c_int()
            check(lib.sv_circuit_apply_blocks(self.handle, state.handle, pp, int(dense_block), ctypes.byref(nb)))
            self.last_dense_blocks = nb.value
            return state
        fn = lib.sv_circuit_apply_fused if fuse_diagonal else lib.sv_circuit_apply
        check(fn(self.handle, state.handle, pp))
        return state


    def adjoint_grad(self, psi: State, lam: State, params, obs) -> Tuple[float, np.ndarray]:
        """Returns (E, dE/dparams); psi holds the input state on entry and again
        (up to rounding) on exit."""
        obs = obs if isinstance(obs, Observable) else Observable(obs)
        p, pp = _dbl(list(params) if len(params) else [0.0])
        g = np.zeros(max(1, self.n_params), dtype=np.float64)
        e = ctypes.c_double()
        check(lib.sv_adjoint_grad(self.handle, psi.handle, lam.handle, pp, ctypes.byref(obs.c), ctypes.byref(e),
                                  g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return e.value, g[: self.n_params]


_OBS_KIND = {"sum_z": 1, "sum_zz": 2}
_INFO_KEYS = ["circuits", "items", "passes", "max_passes", "fused_ops", "params", "state_bytes", "pass_bytes",
              "levels", "lds_bytes", "layout_changes", "threads"]


def _batch_structs(circuits):
    keep = []
    arr = (SvBatchCircuit * max(1, len(circuits)))()
    for i, (n, ops, npar, obs) in enumerate(circuits):
        ops = list(ops)
        oa = (SvOp * max(1, len(ops)))()
        for j, op in enumerate(ops):
            oa[j], k = _sv_op(op)
            keep.append(k)
        keep.append(oa)
        arr[i] = SvBatchCircuit(int(n), len(ops), oa, int(npar), _OBS_KIND[obs])
    return arr, keep


def batch_plan(circuits, dtype: str = "c128", tile_qubits: int = 0, amps_per_thread: int = 0,
               with_grad: bool = True) -> dict:
    """Schedule a batch on the host only (no GPU needed) and report its figures."""
    circuits = list(circuits)
    arr, keep = _batch_structs(circuits)
    opts = SvBatchOpts(int(tile_qubits), int(amps_per_thread), 1, int(bool(with_grad)))
    a = (ctypes.c_int64 * 12)()
    check(lib.sv_batch_plan(arr, len(circuits), _SV_DT[dtype], ctypes.byref(opts), a))
    return dict(zip(_INFO_KEYS, list(a)))


class Batch:
    """Many circuits (or one large one) in one fused graph launch
    (sv_batch_*).  circuits: sequence of (n_qubits, ops, n_params, observable)
    with observable "sum_z" or "sum_zz"."""

    def __init__(self, circuits, dtype: str = "c128", tile_qubits: int = 0, amps_per_thread: int = 0,
                 use_graph: bool = True, with_grad: bool = True):
        circuits = list(circuits)
        self.dtype = dtype
        self.n_circuits = len(circuits)
        self.n_qubits = [int(c[0]) for c in circuits]
        self.n_params = [int(c[2]) for c in circuits]
        self.with_grad = bool(with_grad)
        arr, keep = _batch_structs(circuits)
        opts = SvBatchOpts(int(tile_qubits), int(amps_per_thread), int(bool(use_graph)), int(bool(with_grad)))
        h = ctypes.c_void_p()
        check(lib.sv_batch_create(arr, len(circuits), _SV_DT[dtype], ctypes.byref(opts), ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and lib is not None:
            lib.sv_batch_free(h)
            self.handle = None

    def run(self, params=()):
        """Returns (expvals[n_circuits], grads[sum n_params] or None)."""
        p, pp = _dbl(list(params) if len(params) else [0.0])
        e = np.zeros(self.n_circuits)
        g = np.zeros(max(1, sum(self.n_params)))
        check(lib.sv_batch_run(self.handle, ctypes.c_void_p(p.ctypes.data), 0, ctypes.c_void_p(e.ctypes.data),
                               ctypes.c_void_p(g.ctypes.data), 0))
        return e, (g[: sum(self.n_params)] if self.with_grad else None)

    def run_device(self, params: torch.Tensor, expvals: torch.Tensor, grads: torch.Tensor) -> None:
        """Device-resident parameters and outputs (float64 CUDA tensors).  The
        run is ordered after the work queued on torch's current stream, and
        work queued there afterwards sees the outputs (sv_batch_set_stream)."""
        check(lib.sv_batch_set_stream(self.handle, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
        check(lib.sv_batch_run(self.handle, ctypes.c_void_p(params.data_ptr()), 1,
                               ctypes.c_void_p(expvals.data_ptr()), ctypes.c_void_p(grads.data_ptr()), 1))

    def info(self) -> dict:
        a = (ctypes.c_int64 * 12)()
        check(lib.sv_batch_info(self.handle, a))
        return dict(zip(_INFO_KEYS, list(a)))

    def state(self, i: int) -> np.ndarray:
        out = np.empty(1 << self.n_qubits[i], dtype=np.complex128 if self.dtype == "c128" else np.complex64)
        check(lib.sv_batch_copy_state(self.handle, i, ctypes.c_void_p(out.ctypes.data), out.nbytes))
        return out

    def state_tensor(self, i: int) -> torch.Tensor:
        """Zero-copy torch view of circuit i's device state (valid while the
        batch lives; the next run overwrites it)."""
        ptr, nq = ctypes.c_void_p(), ctypes.c_int()
        check(lib.sv_batch_state(self.handle, i, ctypes.byref(ptr), ctypes.byref(nq)))

        class _View:
            __cuda_array_interface__ = {"shape": (1 << nq.value,), "typestr": "<c16" if self.dtype == "c128" else "<c8",
                                        "data": (ptr.value, False), "version": 3}

        return torch.as_tensor(_View(), device="cuda")


class AdjointExpval(torch.autograd.Function):
    """E(params) = <psi|O|psi> with psi = U(params)|0...0>, differentiated by the
    adjoint method: the autograd loop of the paper's Listing 1, with the
    gradient from one backward sweep instead of per-parameter reruns.

    Two forms:
      * AdjointExpval.apply(params, circuit, psi, lam, obs): a Circuit run op
        by op on the states psi and lam (any observable).  The C entry point
        takes host parameters, so params are copied to the host.  When no
        gradient is needed (params does not require one, or under
        torch.no_grad) only the forward pass and the expectation run, outside
        autograd;
        otherwise the adjoint sweep computes E and the gradient together.
      * AdjointExpval.apply(params, batch): a one-circuit Batch of the fused
        engine (observable sum_z or sum_zz).  params stay in device memory
        (float64 on the batch's GPU), E and the gradient are written there,
        ordered on torch's current stream; without a needed gradient a batch
        built with with_grad=False runs forward only.
    backward returns dL/dE times the saved gradient."""

    @classmethod
    def apply(cls, params: torch.Tensor, circuit, psi: Optional[State] = None, lam: Optional[State] = None,
              obs=None):
        # whether a gradient is needed is known here, before autograd's
        # forward (which always runs with gradients off)
        if torch.is_grad_enabled() and params.requires_grad:
            return super().apply(params, circuit, psi, lam, obs)
        with torch.no_grad():
            return cls._run(None, params, circuit, psi, lam, obs)

    @staticmethod
    def forward(ctx, params: torch.Tensor, circuit, psi: Optional[State] = None, lam: Optional[State] = None,
                obs=None):
        return AdjointExpval._run(ctx, params, circuit, psi, lam, obs)

    @staticmethod
    def _run(ctx, params, circuit, psi, lam, obs):
        """E, and with ctx the gradient saved for backward; ctx None: forward only."""
        need = ctx is not None
        if isinstance(circuit, Batch):
            if circuit.n_circuits != 1:
                raise ValueError("AdjointExpval takes a Batch of one circuit")
            if need and not circuit.with_grad:
                raise ValueError("a gradient is needed but the batch was built with with_grad=False")
            if not params.is_cuda:
                raise ValueError("the engine form takes parameters in device memory")
            p = params.detach().to(torch.float64).contiguous()
            e = torch.empty(1, dtype=torch.float64, device=p.device)
            g = torch.empty(max(1, circuit.n_params[0]), dtype=torch.float64, device=p.device)
            circuit.run_device(p, e, g)
            if need:
                ctx.save_for_backward(g[: circuit.n_params[0]].to(params.dtype))
            return e[0].to(params.dtype)
        th = params.detach().cpu().double().numpy()
        psi.set_basis(0)
        if not need:
            circuit.apply(psi, th)
            return torch.tensor(psi.expval(obs), dtype=params.dtype, device=params.device)
        e, g = circuit.adjoint_grad(psi, lam, th, obs)
        ctx.save_for_backward(torch.from_numpy(g).to(params.device, params.dtype))
        return torch.tensor(e, dtype=params.dtype, device=params.device)

    @staticmethod
    def backward(ctx, grad_e):
        (g,) = ctx.saved_tensors
        return grad_e * g, None, None, None, None


# Launch shapes measured by the autotuner (paper_2508_13615_amd/autotune.py),
# applied once at import when the table exists.
from . import autotune as _autotune  # noqa: E402

def _tuning_path() -> Optional[str]:
    """The tuning table loaded at import: SV_TUNING_FILE names another file
    ("none": load none and keep the built-in shapes); a named file that does
    not exist is an error, not a silent fallback."""
    p = os.environ.get("SV_TUNING_FILE", "")
    if not p:
        return _autotune.TABLE
    if p.lower() == "none":
        return None
    if not os.path.exists(p):
        raise FileNotFoundError(f"SV_TUNING_FILE={p!r} does not exist")
    return p


_TUNING_PATH = _tuning_path()
TUNED_ENTRIES = _autotune.apply_table(sys.modules[__name__], _TUNING_PATH) if _TUNING_PATH else 0
