"""Host-side tests of the C ABI: the library loads, exports every symbol
include/sv.h declares, and rejects bad arguments before any device work.

No compute call is made: states are wrapped around a dummy, never
dereferenced address, and every call below fails validation on the host.
"""
import ctypes
import json
import os
import re
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

sv = pytest.importorskip("paper_2508_13615_amd", reason="libsv.so not built")
from paper_2508_13615_amd import _lib  # noqa: E402

lib = sv.lib
OK, ARG, QUBIT, OOM, HIP, UNSUP, HANDLE = range(7)
FAKE = 0x100000  # 16-byte aligned, never dereferenced by validation paths


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "sv.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z0-9_]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    syms = header_symbols()
    assert len(syms) >= 25
    for s in syms:
        assert hasattr(lib, s), f"libsv.so does not export {s}"
    assert sorted(_lib.EXPORTS) == syms


def test_library_is_the_in_tree_build():
    assert os.path.dirname(_lib.LIB_PATH) == os.path.join(ROOT, "paper_2508_13615_amd")


def test_one_hip_runtime_in_process():
    maps = open("/proc/self/maps").read()
    hips = {l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l}
    assert len(hips) == 1, hips


def test_state_bytes_matches_paper_memory_figures():
    # Sec. 1: a 30-qubit state needs about 16 GB, a 40-qubit one about 16 TB
    # (complex128, 16 bytes per amplitude).
    assert lib.sv_state_bytes(30, 2) == 16 * 2 ** 30
    assert lib.sv_state_bytes(40, 2) == 16 * 2 ** 40
    assert lib.sv_state_bytes(30, 1) == 8 * 2 ** 30
    assert lib.sv_state_bytes(0, 2) == 0 and lib.sv_state_bytes(41, 2) == 0 and lib.sv_state_bytes(10, 3) == 0


def wrap(n=6, dtype=2):
    h = ctypes.c_void_p()
    assert lib.sv_wrap(ctypes.c_void_p(FAKE), n, dtype, None, ctypes.byref(h)) == OK
    return h


def ints(*q):
    return (ctypes.c_int * max(1, len(q)))(*q)


def test_wrap_validation():
    h = ctypes.c_void_p()
    assert lib.sv_wrap(ctypes.c_void_p(FAKE), 0, 2, None, ctypes.byref(h)) == ARG
    assert lib.sv_wrap(ctypes.c_void_p(FAKE), 41, 2, None, ctypes.byref(h)) == ARG
    assert lib.sv_wrap(ctypes.c_void_p(FAKE), 5, 7, None, ctypes.byref(h)) == ARG
    assert lib.sv_wrap(ctypes.c_void_p(FAKE + 8), 5, 2, None, ctypes.byref(h)) == ARG
    assert lib.sv_wrap(None, 5, 2, None, ctypes.byref(h)) == ARG
    assert lib.sv_wrap(ctypes.c_void_p(FAKE), 5, 2, None, None) == ARG
    assert lib.sv_alloc(0, 2, None, ctypes.byref(h)) == ARG
    assert lib.sv_alloc(41, 2, None, ctypes.byref(h)) == ARG


def test_gate_validation():
    h = wrap(6)
    p = (ctypes.c_double * 1)(0.3)
    try:
        assert lib.sv_apply_gate(h, 1, ints(6), 1, None, None, 0) == QUBIT
        assert lib.sv_apply_gate(h, 1, ints(-1), 1, None, None, 0) == QUBIT
        assert lib.sv_apply_gate(h, 11, ints(2, 2), 2, None, None, 0) == QUBIT  # repeated
        assert lib.sv_apply_controlled(h, 1, ints(3), 1, ints(3), 1, None, None, 0) == QUBIT  # control = target
        assert lib.sv_apply_gate(h, 1, ints(0, 1), 2, None, None, 0) == ARG  # X takes 1 target
        assert lib.sv_apply_gate(h, 11, ints(0), 1, None, None, 0) == ARG  # SWAP takes 2
        assert lib.sv_apply_gate(h, 99, ints(0), 1, None, None, 0) == ARG
        assert lib.sv_apply_gate(h, 8, ints(0), 1, None, None, 0) == ARG  # RY without params
        assert lib.sv_apply_gate(h, 12, ints(0), 1, p, None, 0) == ARG  # U2 without matrix
        assert lib.sv_apply_gate(h, 1, None, 1, None, None, 0) == ARG
        ctl = ints(*range(1, 10))
        assert lib.sv_apply_controlled(h, 1, ctl, 9, ints(0), 1, None, None, 0) == ARG  # > 8 controls
        m = (ctypes.c_double * 128)()
        assert lib.sv_apply_general(h, ints(0, 1, 2, 3), 4, m) == ARG  # k > 3
        assert lib.sv_apply_general(h, ints(0), 1, None) == ARG
        assert lib.sv_apply_general(h, ints(0, 0), 2, m) == QUBIT
        md = (ctypes.c_double * (2 * 4 ** 6))()
        assert lib.sv_apply_dense(h, ints(0, 1, 2), 3, md) == ARG  # k < 4: the vector kernels
        assert lib.sv_apply_dense(h, ints(0, 1, 2, 3, 4, 5, 6), 7, md) == ARG  # k > 6
        assert lib.sv_apply_dense(h, ints(0, 1, 2, 3), 4, None) == ARG
        assert lib.sv_apply_dense(h, ints(0, 1, 2, 2), 4, md) == QUBIT  # repeated
        assert lib.sv_apply_dense(h, ints(0, 1, 2, 6), 4, md) == QUBIT  # out of range
        assert lib.sv_apply_dense(h, None, 4, md) == ARG
        u64 = lambda *v: (ctypes.c_uint64 * max(1, len(v)))(*v)  # noqa: E731
        ang = (ctypes.c_double * 65)()
        assert lib.sv_apply_phases(h, 0, u64(1), ang) == ARG
        assert lib.sv_apply_phases(h, 65, u64(*([1] * 65)), ang) == ARG  # more than 64 terms
        assert lib.sv_apply_phases(h, 1, None, ang) == ARG
        assert lib.sv_apply_phases(h, 1, u64(1), None) == ARG
        assert lib.sv_apply_phases(h, 2, u64(1, 1 << 6), ang) == QUBIT  # bit 6 of a 6-qubit state
        assert lib.sv_set_basis(h, 64) == ARG
    finally:
        assert lib.sv_free(h) == OK


def test_measurement_validation():
    h = wrap(4)
    out = ctypes.c_double()
    try:
        assert lib.sv_expval_pauli(h, b"Z", ints(4), 1, ctypes.byref(out)) == QUBIT
        assert lib.sv_expval_pauli(h, b"Q", ints(0), 1, ctypes.byref(out)) == ARG
        assert lib.sv_expval_pauli(h, b"ZZ", ints(1, 1), 2, ctypes.byref(out)) == QUBIT
        assert lib.sv_norm2(h, None) == ARG
        c = (ctypes.c_double * 1)(1.0)
        x = (ctypes.c_uint64 * 1)(0)
        z = (ctypes.c_uint64 * 1)(1 << 4)  # outside a 4-qubit state
        obs = _lib.SvObs(1, c, x, z)
        assert lib.sv_expval_obs(h, ctypes.byref(obs), ctypes.byref(out)) == QUBIT
        assert lib.sv_expval_obs(h, None, ctypes.byref(out)) == ARG
    finally:
        lib.sv_free(h)


def test_handle_errors():
    h = wrap(3)
    assert lib.sv_free(h) == OK
    assert lib.sv_free(h) == HANDLE
    assert lib.sv_apply_gate(h, 1, ints(0), 1, None, None, 0) == HANDLE
    assert lib.sv_set_basis(ctypes.c_void_p(0xdead0), 0) == HANDLE
    assert lib.sv_circuit_free(ctypes.c_void_p(0)) == HANDLE
    assert b"invalid" in lib.sv_last_error()


def test_stale_handle_rejected_after_reuse():
    # A handle freed and a new object created in its place: the old handle
    # (and every copy of it) is rejected by its generation, the new one works.
    old = wrap(3)
    stale = ctypes.c_void_p(old.value)
    assert lib.sv_free(old) == OK
    fresh = [wrap(3) for _ in range(4)]
    try:
        assert all(f.value != stale.value for f in fresh)
        assert lib.sv_set_basis(stale, 0) == HANDLE
        assert lib.sv_free(stale) == HANDLE
        n = ctypes.c_int()
        assert lib.sv_get_info(fresh[0], ctypes.byref(n), None, None) == OK and n.value == 3
    finally:
        for f in fresh:
            assert lib.sv_free(f) == OK


def test_handle_kinds_are_not_interchangeable():
    # a state handle is not a circuit or a batch handle, and the reverse
    h = wrap(3)
    try:
        assert lib.sv_circuit_free(h) == HANDLE
        assert lib.sv_batch_free(h) == HANDLE
        assert lib.sv_batch_set_stream(h, None) == HANDLE
        info = (ctypes.c_int64 * 12)()
        assert lib.sv_batch_info(h, info) == HANDLE
        # an address-like value is never a handle
        assert lib.sv_set_basis(ctypes.c_void_p(FAKE), 0) == HANDLE
    finally:
        assert lib.sv_free(h) == OK


def test_device_output_expval_validation():
    h = wrap(4)
    try:
        assert lib.sv_expval_pauli_dev(h, b"Z", ints(0), 1, None) == ARG
        assert lib.sv_expval_pauli_dev(h, b"Z", ints(4), 1, ctypes.c_void_p(FAKE)) == QUBIT
        assert lib.sv_expval_pauli_dev(h, b"W", ints(0), 1, ctypes.c_void_p(FAKE)) == ARG
        assert lib.sv_expval_pauli_dev(h, b"XX", ints(2, 2), 2, ctypes.c_void_p(FAKE)) == QUBIT
        assert lib.sv_expval_obs_dev(h, None, ctypes.c_void_p(FAKE)) == ARG
    finally:
        lib.sv_free(h)


def test_stream_bench_validation():
    f = ctypes.c_void_p(FAKE)
    assert lib.sv_stream_bench(4, f, f, 1024, 256, 4, None) == ARG  # mode
    assert lib.sv_stream_bench(3, None, f, 1024, 256, 4, None) == ARG  # in place needs dst
    assert lib.sv_stream_bench(0, f, f, 0, 256, 4, None) == ARG  # empty
    assert lib.sv_stream_bench(0, f, f, 1000, 256, 4, None) == ARG  # not a multiple of 16
    assert lib.sv_stream_bench(0, f, f, 1024, 100, 4, None) == ARG  # block
    assert lib.sv_stream_bench(0, f, f, 1024, 256, 3, None) == ARG  # unroll
    assert lib.sv_stream_bench(0, ctypes.c_void_p(FAKE + 8), f, 1024, 256, 4, None) == ARG  # alignment
    assert lib.sv_stream_bench(1, None, None, 1024, 256, 4, None) == ARG  # read needs src
    assert lib.sv_stream_bench(2, None, f, 1024, 256, 4, None) == ARG  # write needs dst
    assert lib.sv_stream_bench(3, ctypes.c_void_p(FAKE + 8), None, 1024, 256, 4, None) == ARG  # in place: dst aligned


def test_circuit_create_validation_is_host_side():
    ops = (_lib.SvOp * 1)()
    ops[0].gate = 8
    ops[0].n_controls = 0
    ops[0].n_targets = 1
    ops[0].param_index = 3  # out of range for n_params = 2
    ops[0].qubits[0] = 0
    h = ctypes.c_void_p()
    assert lib.sv_circuit_create(4, ops, 1, 2, ctypes.byref(h)) == ARG
    ops[0].param_index = 0
    ops[0].qubits[0] = 9
    assert lib.sv_circuit_create(4, ops, 1, 2, ctypes.byref(h)) == QUBIT
    ops[0].gate = 1  # X takes no parameter
    ops[0].qubits[0] = 0
    assert lib.sv_circuit_create(4, ops, 1, 2, ctypes.byref(h)) == ARG


def test_tuning_table_validation():
    b, u, nt = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert lib.sv_tune_get(0, 2, 2, ctypes.byref(b), ctypes.byref(u), ctypes.byref(nt)) == OK
    assert b.value % 64 == 0 and u.value in (1, 2, 4) and nt.value in (0, 1)
    assert lib.sv_tune_set(0, 2, 2, 100, 1, 0) == ARG
    assert lib.sv_tune_set(0, 2, 2, 256, 3, 0) == ARG
    assert lib.sv_tune_set(0, 2, 2, 256, 1, 2) == ARG
    assert lib.sv_tune_set(9, 2, 2, 256, 1, 0) == ARG
    assert lib.sv_tune_set(0, 2, 3, 256, 1, 0) == ARG
    assert lib.sv_tune_set(2, 2, 1, 256, 1, 0) == ARG  # retired class
    assert lib.sv_tune_set(0, 2, 2, b.value, u.value, nt.value) == OK


def test_block_order_setting_validation():
    o = ctypes.c_int()
    assert lib.sv_get_block_order(ctypes.byref(o)) == OK
    saved = o.value
    assert saved in (-1, 0, 1)
    try:
        for bad in (-2, 2, 7):
            assert lib.sv_set_block_order(bad) == ARG
        assert lib.sv_get_block_order(None) == ARG
        for good in (-1, 0, 1):
            assert lib.sv_set_block_order(good) == OK
            assert sv.get_block_order() == good
    finally:
        sv.set_block_order(saved)


def _run_with_env(env_extra, code):
    import subprocess
    env = dict(os.environ, **env_extra)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    return subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True, text=True,
                          timeout=120)


def test_environment_settings_force_tier_tuning_file_and_order(tmp_path):
    """SV_FORCE_TIER changes the launch-shape tier a gate reports (never its
    kernel), SV_TUNING_FILE loads the named table ("none": built-in shapes
    only; a missing file is an error) and SV_BLOCK_ORDER sets the walk
    order; each in a fresh process, host-only calls."""
    probe = ("import paper_2508_13615_amd as sv; i = sv.plan_info(20, 'c128', 'H', (12,)); "
             "j = sv.plan_info(20, 'c128', 'U4', (19, 0)); "
             "print(i['class'], i['tier'], j['class'], j['tier'], sv.TUNED_ENTRIES, sv.get_block_order(), "
             "sv.tune_get(0, 'c128', 2))")
    base = _run_with_env({}, probe)
    assert base.returncode == 0, base.stderr
    kc_h, tier_h, kc_u, tier_u, n_tuned, order, shape = base.stdout.split(None, 6)
    assert (tier_h, tier_u) == ("2", "0") and int(n_tuned) > 0 and order == "-1"
    forced = _run_with_env({"SV_FORCE_TIER": "1", "SV_BLOCK_ORDER": "1"}, probe)
    assert forced.returncode == 0, forced.stderr
    f = forced.stdout.split(None, 6)
    assert (f[0], f[2]) == (kc_h, kc_u) and (f[1], f[3]) == ("1", "1") and f[5] == "1"
    none = _run_with_env({"SV_TUNING_FILE": "none"}, probe)
    assert none.returncode == 0, none.stderr
    assert none.stdout.split(None, 6)[4] == "0"
    tab = tmp_path / "tab.json"
    tab.write_text(json.dumps({"entries": [{"class": 0, "dtype": "c128", "tier": 2, "block": 320, "unroll": 2,
                                            "nt": 0}]}))
    own = _run_with_env({"SV_TUNING_FILE": str(tab)}, probe)
    assert own.returncode == 0, own.stderr
    o = own.stdout.split(None, 6)
    assert o[4] == "1" and o[6].strip() == "(320, 2, 0)"
    missing = _run_with_env({"SV_TUNING_FILE": str(tmp_path / "nope.json")}, probe)
    assert missing.returncode != 0 and "SV_TUNING_FILE" in missing.stderr


def test_lds_staging_depth_reported_per_form():
    """The LDS-staged class's unroll sets the staging depth of 3-qubit gates
    only; sv_plan_info reports the depth each launch uses, which names the
    kernel instantiation the bench attributes time to (host only)."""
    saved = {t: sv.tune_get(6, "c128", t) for t in range(3)}
    try:
        for u in (1, 2, 4):
            for t in range(3):
                sv.tune_set(6, "c128", t, 128, u, 1)
            two = sv.plan_info(30, "c128", "GENERAL", (29, 0))
            three = sv.plan_info(30, "c128", "GENERAL", (29, 15, 0))
            swap = sv.plan_info(30, "c128", "SWAP", (29, 0))
            assert (two["class"], three["class"], swap["class"]) == (6, 6, 6)
            assert two["unroll"] == 1 and swap["unroll"] == 1 and three["unroll"] == u
            assert two["kernel"] == "k_lds_gate<double, 2, 0, true, 1>"
            assert three["kernel"] == f"k_lds_gate<double, 3, 0, true, {u}>"
            assert swap["kernel"] == "k_lds_gate<double, 2, 1, true, 1>"
    finally:
        for t, shp in saved.items():
            sv.tune_set(6, "c128", t, *shp)


def test_status_strings():
    assert lib.sv_status_string(4) == b"SV_ERR_HIP"
    assert lib.sv_version() >= 1


def test_batch_create_validation_is_host_side():
    ops = (_lib.SvOp * 1)()
    ops[0].gate = 8
    ops[0].n_targets = 1
    ops[0].param_index = 0
    ops[0].qubits[0] = 7  # outside a 4-qubit circuit
    circ = (_lib.SvBatchCircuit * 1)()
    circ[0] = _lib.SvBatchCircuit(4, 1, ops, 1, 1)
    h = ctypes.c_void_p()
    opts = _lib.SvBatchOpts(0, 0, 1, 1)
    assert lib.sv_batch_create(circ, 1, 2, ctypes.byref(opts), ctypes.byref(h)) == QUBIT
    ops[0].qubits[0] = 1
    circ[0] = _lib.SvBatchCircuit(4, 1, ops, 1, 3)  # unknown observable
    assert lib.sv_batch_create(circ, 1, 2, ctypes.byref(opts), ctypes.byref(h)) == ARG
    circ[0] = _lib.SvBatchCircuit(4, 1, ops, 1, 1)
    bad = _lib.SvBatchOpts(14, 0, 1, 1)  # tile too large
    assert lib.sv_batch_create(circ, 1, 2, ctypes.byref(bad), ctypes.byref(h)) == ARG
    bad = _lib.SvBatchOpts(0, 100, 1, 1)  # amplitudes per thread neither 8 nor 16
    assert lib.sv_batch_create(circ, 1, 2, ctypes.byref(bad), ctypes.byref(h)) == ARG
    assert lib.sv_batch_run(ctypes.c_void_p(0x1234), None, 0, None, None, 0) == HANDLE


def test_batch_plan_far_controls_host_only():
    # The universal circuit's CNOTs reach across the register: with their
    # controls left outside the tile, each target needs one pass, and each
    # run of CNOTs from qubits outside the tile with the rotations between
    # them becomes one op per tile (a table of at most 32 products), so the
    # 2080 gates leave far fewer fused ops than the per-gate count.
    import workloads as W
    n = 32
    ops = W.universal_ops(n)
    for tq in (10, 12):
        p = sv.batch_plan([(n, ops, 0, "sum_z")], "c128", with_grad=False, tile_qubits=tq, amps_per_thread=16)
        assert p["passes"] <= 12, (tq, p["passes"])
        assert p["fused_ops"] < len(ops) // 3, (tq, p["fused_ops"])


def test_batch_plan_fuses_gates_host_only():
    # The pass scheduler runs on the host: a 32-qubit, 10-layer hardware-efficient
    # ansatz (950 gates) needs far fewer state passes than gates, every pass
    # fits a 2^12-amplitude tile, and the adjoint doubles the stage count.
    import workloads as W
    ops = W.hea_ops(32, 10)
    shape = dict(tile_qubits=12, amps_per_thread=16)
    fwd = sv.batch_plan([(32, ops, W.hea_n_params(32, 10), "sum_z")], "c128", with_grad=False, **shape)
    adj = sv.batch_plan([(32, ops, W.hea_n_params(32, 10), "sum_z")], "c128", with_grad=True, **shape)
    # forward passes fuse each RY with the RZ after it on the same qubit, and a
    # CNOT with the rotation of its target when both sit in one pass (a 2x2
    # chosen by the control bit): 320 fewer ops, and between 1 and 310 more
    assert len(ops) - 32 * 10 - 31 * 10 <= fwd["fused_ops"] < len(ops) - 32 * 10
    assert adj["fused_ops"] == fwd["fused_ops"]
    assert fwd["passes"] <= len(ops) // 20
    # register tiling: LDS exchanges of the tile are rare next to gates
    assert fwd["layout_changes"] <= len(ops) // 5
    assert fwd["threads"] == 2 ** 12 // 16
    assert fwd["items"] == (fwd["passes"] + 1) * 2 ** 20
    assert adj["levels"] == 2 * adj["passes"] + 1
    assert fwd["lds_bytes"] <= 160 * 1024 and adj["lds_bytes"] <= 160 * 1024
    q = sv.batch_plan([(32, W.qft_ops(32), 0, "sum_z")], "c128", with_grad=False, **shape)
    assert q["passes"] < len(W.qft_ops(32)) // 4
    # tiny tiles: more passes, same gates
    small = sv.batch_plan([(10, W.hea_ops(10, 3), 60, "sum_z")], "c64", tile_qubits=4, with_grad=False)
    big = sv.batch_plan([(10, W.hea_ops(10, 3), 60, "sum_z")], "c64", tile_qubits=0, with_grad=False)
    assert small["passes"] > big["passes"] == 1


def test_engine_tile_shape_tuning_host_only():
    # Zeroed batch shape options take the engine shape of sv_tune_engine_set
    # for the batch's dtype and stage mix; shapes that break the 512-thread
    # limit or the allowed values are refused and leave the setting unchanged.
    import workloads as W
    circ = [(16, W.hea_ops(16, 2), W.hea_n_params(16, 2), "sum_z")]
    keys = [(dt, g) for dt in ("c128", "c64") for g in (False, True)]
    saved = {k: sv.tune_engine_get(*k) for k in keys}
    try:
        for k in keys:
            sv.tune_engine_set(*k, 0, 0)
        assert sv.tune_engine_get("c128", True) == (12, 16)
        assert sv.tune_engine_get("c64", False) == (13, 16)
        sv.tune_engine_set("c64", False, 0, 8)  # 13 would need 1024 threads of 8 amplitudes
        assert sv.tune_engine_get("c64", False) == (12, 8)
        sv.tune_engine_set("c128", True, 10, 8)
        sv.tune_engine_set("c128", False, 11, 16)
        p = sv.batch_plan(circ, "c128", with_grad=True)
        assert p["threads"] == 2 ** 10 // 8 and p["items"] % 2 ** 6 == 0
        p = sv.batch_plan(circ, "c128", with_grad=False)
        assert p["threads"] == 2 ** 11 // 16 and p["items"] % 2 ** 5 == 0
        explicit = sv.batch_plan(circ, "c128", tile_qubits=12, amps_per_thread=16)
        assert explicit["threads"] == 2 ** 12 // 16
        for dt, tq, apt in (("c128", 13, 16), ("c128", 13, 8), ("c64", 13, 8), ("c128", 1, 16), ("c128", 14, 0),
                            ("c128", 12, 4), ("c64", 0, 32)):
            with pytest.raises(sv.SvError):
                sv.tune_engine_set(dt, True, tq, apt)
        # forward-only: no reverse workgroups, so a complex128 2^13 tile of 16 per thread fits
        sv.tune_engine_set("c128", False, 13, 16)
        assert sv.tune_engine_get("c128", False) == (13, 16)
        assert sv.batch_plan(circ, "c128", with_grad=False)["threads"] == 512
        with pytest.raises(sv.SvError):
            sv.tune_engine_set("c128", False, 13, 8)
        assert sv.tune_engine_get("c128", True) == (10, 8)
        assert sv.lib.sv_tune_engine_set(7, 1, 0, 0) == ARG  # bad dtype
        assert sv.lib.sv_tune_engine_set(2, 2, 0, 0) == ARG  # with_grad not 0/1
    finally:
        for k, (tq, apt) in saved.items():
            sv.tune_engine_set(*k, tq, apt)


def test_block_plan_host_only():
    # every op lands in exactly one block; blocks span at most k qubits; the
    # 10-layer 32-qubit HEA packs into about 8 five-qubit blocks per layer
    import workloads as W
    for n, ops in ((32, W.hea_ops(32, 10)), (32, W.qft_ops(32)), (32, W.universal_ops(32)), (9, W.ghz_ops(9))):
        for k in (4, 5, 6):
            p = sv.block_plan(n, ops, k)
            assert p["single_ops"] + p["ops_in_dense"] == len(ops)
            assert p["widest"] <= k
    assert sv.block_plan(32, W.hea_ops(32, 10), 5)["dense_blocks"] <= 9 * 10
    # a Toffoli with two more controls (5 qubits) cannot join a 4-qubit block
    big = [W.Op("X", (0, 1, 2, 3), (4,)), W.Op("H", (), (0,))]
    p = sv.block_plan(6, big, 4)
    assert p["single_ops"] == 2 and p["dense_blocks"] == 0 and p["widest"] == 5
    with pytest.raises(sv.SvError):
        sv.block_plan(6, big, 3)
    with pytest.raises(sv.SvError):
        sv.block_plan(6, [W.Op("H", (), (6,))], 4)
