"""Initialization on the GPU (sp_symbolize_device through the C ABI).

The device pass is checked against the oracle: the paper's printed
examples, (M, c) read off the oracle by probing one variable at a time,
and M b + c against the oracle's outcomes for random fault codes.  Larger
circuits, which the oracle cannot probe in seconds, are checked against
the host pass (itself pinned to the oracle in test_symbolize.py) and by
sampling the device-built model on the GPU against the oracle."""

from __future__ import annotations

import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2311_03906_amd as sp
from paper_2311_03906_amd import _capi
from golden_io import example
from workloads import random_clifford_circuit, random_layered_circuit, repetition_memory, surface_memory

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


def _device_model(text, outputs="measurements", mode="auto"):
    return sp.Model(text, outputs=outputs, init="device", init_mode=mode)


MODES = ["one_pass", "two_pass"]


def _same_model(a, b):
    """Bit-identical models: sizes, variable table, column lists, c."""
    for f in ("n_qubits", "n_meas", "n_locs", "n_vars", "n_random_meas", "n_drawn", "n_draw_blocks", "nnz"):
        assert getattr(a.dims, f) == getattr(b.dims, f), f
    for x, y in zip(a.export_vars(), b.export_vars()):
        assert np.array_equal(x, y)
    for x, y in zip(a.export_csc(), b.export_csc()):
        assert np.array_equal(x, y)
    assert np.array_equal(a.export_dense()[1], b.export_dense()[1])


def _assignment(model_vars, codes):
    var_loc, var_bit = model_vars
    return ((codes[var_loc] >> var_bit) & 1).astype(np.uint8)


def _evaluate(M, c, b):
    return ((M.astype(np.int64) @ b.astype(np.int64)) + c) % 2


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", ["fig1.txt", "bell.txt"])
def test_paper_examples_on_device(name, mode):
    """The paper's printed outcome expressions (Fig. 1 and the Bell
    example), built on the GPU."""
    text, symbols, outcomes = example(name)
    _say(f"device init {name} {mode}")
    m = _device_model(text, mode=mode)
    M, c = m.export_dense()
    var_loc, var_bit = m.export_vars()
    col_of = {(int(l), int(b)): j for j, (l, b) in enumerate(zip(var_loc, var_bit))}
    assert m.n_vars == len(symbols)
    want = np.zeros((len(outcomes), m.n_vars), dtype=np.uint8)
    for k, terms in enumerate(outcomes):
        for s in terms:
            want[k, col_of[symbols[s]]] ^= 1
    assert np.array_equal(M, want)
    assert not c.any()


_SMALL = [("rep3", repetition_memory(3, 3, 1e-3, detectors=True)),
          ("surf3", surface_memory(3, 3, "0.01", detectors=True)),
          ("surf3_feedback", surface_memory(3, 3, "0.01", detectors=True, reset="feedback")),
          ("layered12", random_layered_circuit(12, seed=1, cnot_pairs=6, p_dep="0.01")),
          ("random_feedback", random_clifford_circuit(11, 4, 40, feedback=True, detectors=True))]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("outputs", ["measurements", "detectors"])
@pytest.mark.parametrize("name,circ", _SMALL, ids=[n for n, _ in _SMALL])
def test_device_model_equals_oracle_probing(name, circ, outputs, mode):
    """(M, c) of the device pass equal the oracle's outputs with one code
    bit set at a time (columns) and none set (c)."""
    if outputs == "detectors" and circ.n_detectors + circ.n_observables == 0:
        pytest.skip("no detectors")
    text = circ.text()
    _say(f"device init probing {name} {outputs} {mode}")
    m = _device_model(text, outputs, mode)
    oc = oracle.Circuit(text, outputs=outputs)
    var_loc, var_bit = m.export_vars()
    zero = np.zeros(oc.n_locs, dtype=np.uint8)
    c0 = oc.rows_from_outcomes(oc.run_codes(zero)[0])
    cols = []
    for l, b in zip(var_loc, var_bit):
        codes = zero.copy()
        codes[l] = 1 << b
        cols.append(oc.rows_from_outcomes(oc.run_codes(codes)[0]) ^ c0)
    M_or = np.array(cols, dtype=np.uint8).T if cols else np.zeros((oc.n_rows, 0), dtype=np.uint8)
    M, c = m.export_dense()
    assert np.array_equal(M, M_or)
    assert np.array_equal(c, c0)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(40))
def test_device_model_matches_oracle_on_random_circuits(seed, mode):
    """Random noisy Clifford circuits with resets, feedback, detectors and
    observables: M b + c of the device model equals the oracle's outputs for
    random codes at every location (a location the device wrongly took as
    determined, or a wrong variable, changes some output)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 9))
    n_ops = int(rng.integers(1, 80))
    text = random_clifford_circuit(seed, n, n_ops, feedback=True, detectors=True).text()
    for outputs in ("measurements", "detectors"):
        oc = oracle.Circuit(text, outputs=outputs)
        m = _device_model(text, outputs, mode)
        M, c = m.export_dense()
        mv = m.export_vars()
        kinds = oc.location_kinds()
        for _ in range(4):
            codes = np.array([rng.integers(0, 2 ** oracle.CODE_BITS[int(k)]) for k in kinds], dtype=np.uint8)
            want = oc.rows_from_outcomes(oc.run_codes(codes)[0])
            assert np.array_equal(_evaluate(M, c, _assignment(mv, codes)), want)


def _repeated_target_circuit(seed):
    """Noisy Clifford circuit whose M, R and MR instructions have several
    targets with repeats, so that one instruction holds runs of determined
    outcomes in which the same qubit is measured or reset again."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 7))
    lines = []
    for _ in range(int(rng.integers(5, 40))):
        kind = rng.integers(7)
        if kind == 0:
            lines.append("H " + " ".join(str(q) for q in rng.choice(n, int(rng.integers(1, n + 1)), replace=False)))
        elif kind == 1:
            lines.append("S " + " ".join(str(q) for q in rng.choice(n, int(rng.integers(1, n + 1)), replace=False)))
        elif kind == 2:
            a, b = rng.choice(n, 2, replace=False)
            lines.append(f"CX {a} {b}")
        elif kind == 3:
            lines.append(f"X_ERROR(0.25) {rng.integers(n)}")
        elif kind == 4:
            lines.append(f"DEPOLARIZE1(0.5) {rng.integers(n)}")
        else:
            op = ("M", "R", "MR")[int(rng.integers(3))]
            lines.append(op + " " + " ".join(str(q) for q in rng.integers(0, n, int(rng.integers(2, 12)))))
    lines.append("M " + " ".join(str(q) for q in range(n)))
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(30))
def test_repeated_targets_in_one_instruction(seed, mode):
    """Measurements and resets of the same qubit again within one
    instruction (a reset's X then flips rows that a later outcome of the
    same instruction selects): the device model equals the host model and
    reproduces the oracle's outputs for random codes."""
    text = _repeated_target_circuit(seed)
    rng = np.random.default_rng(1000 + seed)
    oc = oracle.Circuit(text)
    m = _device_model(text, "measurements", mode)
    _same_model(m, sp.Model(text))
    M, c = m.export_dense()
    mv = m.export_vars()
    kinds = oc.location_kinds()
    for _ in range(4):
        codes = np.array([rng.integers(0, 2 ** oracle.CODE_BITS[int(k)]) for k in kinds], dtype=np.uint8)
        want = oc.rows_from_outcomes(oc.run_codes(codes)[0])
        assert np.array_equal(_evaluate(M, c, _assignment(mv, codes)), want)


_LARGE = [("surf5", lambda: surface_memory(5, 5, 1e-3, detectors=True)),
          ("surf7_feedback", lambda: surface_memory(7, 7, "0.005", detectors=True, reset="feedback")),
          ("rep25", lambda: repetition_memory(25, 25, "0.01", detectors=True)),
          ("fig3a_n60", lambda: random_layered_circuit(60, seed=2, cnot_pairs=5)),
          ("fig3b_n60", lambda: random_layered_circuit(60, seed=2)),
          ("fig3c_n60", lambda: random_layered_circuit(60, seed=2, p_dep="0.001")),
          ("fig3c_n130", lambda: random_layered_circuit(130, seed=4, p_dep="0.001")),
          ("random_feedback_64q", lambda: random_clifford_circuit(5, 64, 3000, feedback=True, detectors=True))]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("outputs", ["measurements", "detectors"])
@pytest.mark.parametrize("name,make", _LARGE, ids=[n for n, _ in _LARGE])
def test_device_model_equals_host_model(name, make, outputs, mode):
    """Several tableau words per column, several phase words per row, many
    instructions split into runs: the device model is bit-identical to the
    host pass."""
    circ = make()
    if outputs == "detectors" and circ.n_detectors + circ.n_observables == 0:
        pytest.skip("no detectors")
    text = circ.text()
    _say(f"device init vs host {name} {outputs} {mode}")
    _same_model(_device_model(text, outputs, mode), sp.Model(text, outputs=outputs))


@pytest.mark.parametrize("mode", MODES)
def test_surface_d15_detectors_device_model(mode):
    """The served workload's circuit (surface d=15, 15 rounds, 449 qubits,
    p = 5e-3, detector outputs): device model equals the host model."""
    text = surface_memory(15, 15, "0.005", detectors=True).text()
    _say("device init surface d15 detectors")
    _same_model(_device_model(text, "detectors", mode), sp.Model(text, outputs="detectors"))


@pytest.mark.parametrize("case", ["surface_d15_detectors", "surface_d15_measurements", "fig3c_n200"])
def test_two_pass_replay_repeats_exactly(case):
    """Surface d=15 (resets, runs of determined outcomes) and Fig. 3c at
    n = 200 (82,084 fault variables, mostly random outcomes) in two passes,
    four times in a row: every build equals the host model.  The replay's
    workgroups skip log entries that leave their slice unchanged without a
    barrier, and a missing one shows up as builds that differ from run to
    run."""
    if case == "fig3c_n200":
        outputs, text = "measurements", random_layered_circuit(200, seed=5, p_dep="0.001").text()
    else:
        outputs = case.split("_")[-1]
        text = surface_memory(15, 15, "0.005" if outputs == "detectors" else "0.001",
                              detectors=outputs == "detectors").text()
    host = sp.Model(text, outputs=outputs)
    circ = sp.Circuit(text)
    for i in range(4):
        _say(f"two-pass {case} build {i}")
        _same_model(sp.Model(circ, outputs=outputs, init="device", init_mode="two_pass"), host)


def _scrambled(n, seed=7):
    """n qubits scrambled by layers of CNOTs, S and depolarizing faults,
    with random-outcome measurements, Paulis controlled by them, resets
    and faults on the highest qubits."""
    rng = np.random.default_rng(seed)
    lines = [f"H {' '.join(map(str, range(0, n, 2)))}"]
    for _ in range(6):
        perm = rng.permutation(n)[: n - n % 2]
        lines.append("CX " + " ".join(map(str, perm)))
        lines.append("DEPOLARIZE1(0.001) " + " ".join(map(str, rng.choice(n, 64, replace=False))))
        lines.append("S " + " ".join(map(str, rng.choice(n, 300, replace=False))))
        lines.append("M " + " ".join(map(str, rng.choice(n, 40, replace=False))))
        lines.append(f"CX rec[-1] {n - 1} rec[-2] {n - 24}")
    lines.append(f"MR {n - 1} {n - 2} 0")
    lines.append("M " + " ".join(map(str, range(n))))
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("mode", MODES)
def test_max_qubits(mode):
    """1024 qubits (the limit: 32 tableau words per column) with
    measurements, resets and faults on the highest qubits."""
    text = _scrambled(1024)
    _say(f"device init 1024 qubits {mode}")
    _same_model(_device_model(text, mode=mode), sp.Model(text))


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n", [513, 520, 600, 777, 1023])
def test_global_tableau_ragged_words(n, mode):
    """Tableaux too large for LDS whose columns fill 17 to 32 of a
    half-wave's 32 lanes (the random outcome's column pass leaves the rest
    idle), with the last wave holding 1 to 64 columns: the device model
    equals the host's."""
    text = _scrambled(n, seed=n)
    _say(f"device init {n} qubits {mode}")
    _same_model(_device_model(text, mode=mode), sp.Model(text))


def test_device_model_samples_equal_oracle():
    """The whole device path: a model built on the GPU, uploaded and sampled
    on the GPU, equals the oracle's samples word for word."""
    text = surface_memory(5, 5, "0.005", detectors=True, reset="feedback").text()
    _say("device init + sample surface d5 feedback detectors")
    m = _device_model(text, "detectors")
    dm = sp.DeviceModel(m)
    out = dm.sample(20_000, seed=4)
    torch.cuda.synchronize()
    got = sp.to_numpy_bits(out)[: dm.n_meas]
    want = oracle.Circuit(text, outputs="detectors").sample(seed=4, first_shot=0, shots=20_000)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("mode", MODES)
def test_degenerate_circuits(mode):
    """No instructions, no measurements, only gates, only faults, determined
    outcomes without any variable."""
    for text in ["", "H 0\nS 1\nCX 0 1\n", "X_ERROR(0.1) 0 1 2\n", "M 0\n", "R 0 1\nM 1\n",
                 "M 0 1\nM 0\nCX rec[-1] 1\nM 1\n"]:
        _say(f"device init degenerate {text!r} {mode}")
        _same_model(_device_model(text, mode=mode), sp.Model(text))


def test_index_list_overflow_is_reported():
    """A buffer with no room for the determined outcomes' index lists gives
    SP_E_LIMIT (the kernel flags it and ends normally); a buffer of the size
    the message names then gives the host pass's model."""
    text = repetition_memory(5, 5, "0.01").text()
    c = sp.Circuit(text)
    L = _capi.lib()
    need = ctypes.c_size_t()
    _capi.check(L.sp_symbolize_device_work_bytes(c.handle, ctypes.byref(need)))
    work = torch.zeros(need.value + 256, dtype=torch.uint8, device="cuda")
    base = ctypes.c_void_p(work.data_ptr() + (-work.data_ptr()) % 256)
    h = ctypes.c_void_p()
    one = _capi.SP_INIT_ONE_PASS
    got = ctypes.c_size_t(12345)
    # too small for the fixed part: rejected before any device work, with
    # the size that suffices in the out-parameter and the message
    assert L.sp_symbolize_device_mode(c.handle, 0, one, base, 256, None, ctypes.byref(h),
                                      ctypes.byref(got)) == _capi.SP_E_INVALID
    fixed = got.value
    assert str(fixed).encode() in L.sp_last_error()
    assert 256 < fixed < need.value
    _say("device init list overflow")
    assert L.sp_symbolize_device_mode(c.handle, 0, one, base, fixed, None, ctypes.byref(h),
                                      ctypes.byref(got)) == _capi.SP_E_LIMIT
    enough = got.value
    assert str(enough).encode() + b" bytes suffice" in L.sp_last_error()
    assert fixed < enough <= need.value
    _capi.check(L.sp_symbolize_device_mode(c.handle, 0, one, base, enough, None, ctypes.byref(h),
                                           ctypes.byref(got)))
    assert got.value == 0
    try:
        ref = sp.Model(text)
        d = _capi.sp_dims()
        _capi.check(L.sp_model_dims(h, ctypes.byref(d)))
        assert (d.n_vars, d.nnz, d.n_meas) == (ref.dims.n_vars, ref.dims.nnz, ref.dims.n_meas)
        cp = np.zeros(d.n_vars + 1, dtype=np.uint32)
        ri = np.zeros(max(1, d.nnz), dtype=np.uint32)
        _capi.check(L.sp_model_export_csc(h, cp.ctypes.data, ri.ctypes.data))
        want_cp, want_ri = ref.export_csc()
        assert np.array_equal(cp, want_cp) and np.array_equal(ri[: d.nnz], want_ri)
    finally:
        L.sp_model_free(h)


def test_two_pass_on_fig3c_n200():
    """Fig. 3c at n = 200 (82,084 variables, phase rows of 1,283 words):
    both passes give the host's model; the replay spans several workgroups."""
    text = random_layered_circuit(200, seed=1, p_dep="0.001").text()
    host = sp.Model(text)
    for mode in MODES:
        _say(f"fig3c n=200 device init {mode}")
        _same_model(_device_model(text, mode=mode), host)


def test_two_pass_buffer_too_small_is_reported():
    """Two passes with no room after the log for the determined outcomes'
    rows: SP_E_LIMIT naming a size; with that size the call gives the host
    pass's model (the same protocol the binding retries once)."""
    text = surface_memory(5, 5, "0.01", detectors=True).text()
    c = sp.Circuit(text)
    L = _capi.lib()
    two = _capi.SP_INIT_TWO_PASS
    need = ctypes.c_size_t()
    _capi.check(L.sp_symbolize_device_work_bytes_mode(c.handle, two, ctypes.byref(need)))
    work = torch.zeros(need.value + 256, dtype=torch.uint8, device="cuda")
    base = ctypes.c_void_p(work.data_ptr() + (-work.data_ptr()) % 256)
    h = ctypes.c_void_p()
    got = ctypes.c_size_t()
    assert L.sp_symbolize_device_mode(c.handle, 0, two, base, 256, None, ctypes.byref(h),
                                      ctypes.byref(got)) == _capi.SP_E_INVALID
    fixed = got.value
    assert b"need at least %d" % fixed in L.sp_last_error()
    _say("two-pass buffer too small")
    assert L.sp_symbolize_device_mode(c.handle, 0, two, base, fixed, None, ctypes.byref(h),
                                      ctypes.byref(got)) == _capi.SP_E_LIMIT
    enough = got.value
    assert b"%d bytes" % enough in L.sp_last_error()
    assert fixed < enough <= need.value
    # the figure covers the rows of E and a bound on the lists; a size that
    # fits the lists' bound but not their real length would name that length
    rc = L.sp_symbolize_device_mode(c.handle, 0, two, base, enough, None, ctypes.byref(h), ctypes.byref(got))
    if rc == _capi.SP_E_LIMIT:
        assert enough < got.value <= need.value
        enough = got.value
        rc = L.sp_symbolize_device_mode(c.handle, 0, two, base, enough, None, ctypes.byref(h), ctypes.byref(got))
    _capi.check(rc)
    assert got.value == 0
    try:
        ref = sp.Model(text)
        d = _capi.sp_dims()
        _capi.check(L.sp_model_dims(h, ctypes.byref(d)))
        assert (d.n_vars, d.nnz, d.n_meas) == (ref.dims.n_vars, ref.dims.nnz, ref.dims.n_meas)
        cp = np.zeros(d.n_vars + 1, dtype=np.uint32)
        ri = np.zeros(max(1, d.nnz), dtype=np.uint32)
        _capi.check(L.sp_model_export_csc(h, cp.ctypes.data, ri.ctypes.data))
        want_cp, want_ri = ref.export_csc()
        assert np.array_equal(cp, want_cp) and np.array_equal(ri[: d.nnz], want_ri)
    finally:
        L.sp_model_free(h)
