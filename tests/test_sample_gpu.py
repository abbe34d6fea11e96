"""GPU sampling path (sp_sample through the C ABI) against the CPU oracle.

Bit-exact: the draws are keyed by (seed, shot, location), so the packed
outcome matrix is a unique function of the inputs and every word must
match.  At full workload sizes the oracle checks a sample of shots, one by
one, and the rest is checked by invariants that hold at any size."""

from __future__ import annotations

import math
import sys

import numpy as np
import pytest
import torch

import oracle
import piling_up
import paper_2311_03906_amd as sp
from workloads import random_clifford_circuit, random_layered_circuit, repetition_memory, surface_memory

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


_cache = {}


def _models(text, path="auto", outputs="measurements"):
    key = (text, path, outputs)
    if key not in _cache:
        m = sp.Model(text, outputs=outputs)
        _cache[key] = (m, sp.DeviceModel(m, path=path), oracle.Circuit(text, outputs=outputs))
    return _cache[key]


def _gpu(dm, shots, seed, first_shot=0, ld=None):
    out = dm.sample(shots, seed=seed, first_shot=first_shot, ld=ld)
    torch.cuda.synchronize()
    return sp.to_numpy_bits(out)[: dm.n_meas]


def _column(packed, i):
    return ((packed[:, i // 64] >> np.uint64(i % 64)) & np.uint64(1)).astype(np.uint8)


# ------------------------------------------------------------- full parity --

@pytest.mark.parametrize("path", ["sparse", "dense"])
def test_repetition_d3_full(path):
    """Distance-3 repetition memory, 3 rounds, p = 1e-3, 10^4 shots, seed 0:
    every word equals the oracle's."""
    text = repetition_memory(3, 3, 1e-3).text()
    _say(f"rep d3 10^4 shots path={path}")
    m, dm, oc = _models(text, path)
    got = _gpu(dm, 10_000, seed=0)
    want = oc.sample(seed=0, first_shot=0, shots=10_000)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("path", ["sparse", "dense"])
@pytest.mark.parametrize("p", ["0.001", "0.01"])
def test_surface_d5_full(path, p):
    text = surface_memory(5, 5, p).text()
    _say(f"surface d5 p={p} 20000 shots path={path}")
    m, dm, oc = _models(text, path)
    got = _gpu(dm, 20_000, seed=3, first_shot=123_456)
    want = oc.sample(seed=3, first_shot=123_456, shots=20_000)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("fig,kw", [("3a", {"cnot_pairs": 5}), ("3b", {}), ("3c", {"p_dep": "0.001"})])
@pytest.mark.parametrize("path", ["sparse", "dense"])
def test_paper_fig3_circuits_full(fig, kw, path):
    """The paper's benchmark family at n = 60 (Fig. 3a/b/c): 10^4 samples,
    every word equals the oracle's, on both evaluation paths."""
    text = random_layered_circuit(60, seed=2, **kw).text()
    _say(f"fig{fig} n=60 10^4 shots path={path}")
    m, dm, oc = _models(text, path)
    got = _gpu(dm, 10_000, seed=9)
    assert np.array_equal(got, oc.sample(seed=9, first_shot=0, shots=10_000))


def test_layered_random_circuit_full():
    text = random_layered_circuit(24, seed=5, cnot_pairs=12, p_dep="0.01").text()
    _say("layered n=24 3000 shots")
    m, dm, oc = _models(text)
    got = _gpu(dm, 3000, seed=8)
    assert np.array_equal(got, oc.sample(seed=8, first_shot=0, shots=3000))


@pytest.mark.parametrize("path", ["sparse", "dense"])
@pytest.mark.parametrize("name,circ", [("rep5", repetition_memory(5, 5, "0.01", detectors=True)),
                                       ("surf5", surface_memory(5, 5, "0.005", detectors=True)),
                                       ("surf3", surface_memory(3, 3, "0.02", detectors=True))])
def test_detector_outputs_full(name, circ, path):
    """Detector and observable rows (XORs of records) sampled on the GPU
    equal the oracle's detector rows, word for word."""
    text = circ.text()
    _say(f"detectors {name} 20000 shots path={path}")
    m, dm, oc = _models(text, path, "detectors")
    assert m.n_meas == oc.n_rows == circ.n_detectors + circ.n_observables
    got = _gpu(dm, 20_000, seed=11, first_shot=640)
    assert np.array_equal(got, oc.sample(seed=11, first_shot=640, shots=20_000))


@pytest.mark.parametrize("outputs", ["measurements", "detectors"])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_feedback_circuits_full(seed, outputs):
    """Random noisy circuits with Paulis controlled by earlier records
    (CX/CY/CZ rec[-k] q), detectors and observables: every word equals the
    oracle's."""
    text = random_clifford_circuit(seed, 8, 120, feedback=True, detectors=True).text()
    _say(f"feedback circuit seed={seed} outputs={outputs} 5000 shots")
    m, dm, oc = _models(text, "auto", outputs)
    got = _gpu(dm, 5000, seed=seed)
    assert np.array_equal(got, oc.sample(seed=seed, first_shot=0, shots=5000))


@pytest.mark.parametrize("outputs", ["measurements", "detectors"])
def test_surface_feedback_reset_full(outputs):
    """Surface d=5, 5 rounds, p = 5e-3, ancillas reset by X controlled by
    their previous outcome (a dynamic circuit): every word equals the
    oracle's."""
    text = surface_memory(5, 5, "0.005", detectors=True, reset="feedback").text()
    _say(f"surface d5 feedback reset outputs={outputs} 20000 shots")
    m, dm, oc = _models(text, "auto", outputs)
    got = _gpu(dm, 20_000, seed=6)
    assert np.array_equal(got, oc.sample(seed=6, first_shot=0, shots=20_000))


def test_surface_d15_detectors_sampled():
    """Surface d=15, 15 rounds, p = 5e-3, detector outputs, one 2^20-shot
    launch at first_shot = 2^20: 1024 shots equal the oracle's rows."""
    text = surface_memory(15, 15, "0.005", detectors=True).text()
    _say("surface d15 detectors 2^20 shots sampled")
    m, dm, oc = _models(text, "sparse", "detectors")
    shots = 1 << 20
    got = _gpu(dm, shots, seed=4, first_shot=shots)
    ids = np.random.default_rng(4).choice(shots, 1024, replace=False)
    want = oc.sample_shots(4, ids + shots)
    for i, s in enumerate(ids):
        assert np.array_equal(_column(got, int(s)), want[i]), int(s)


# ------------------------------------------------------ full-size, sampled --

def test_surface_d5_million_shots_sampled():
    """Surface d=5, 5 rounds, p = 1e-3, 10^6 shots in one launch: the first
    and last 4096 shots and 4096 seeded-random shots equal the oracle."""
    text = surface_memory(5, 5, 1e-3).text()
    _say("surface d5 10^6 shots sampled")
    m, dm, oc = _models(text)
    shots = 1_000_000
    got = _gpu(dm, shots, seed=0)
    ids = np.concatenate([np.arange(4096), np.arange(shots - 4096, shots),
                          np.random.default_rng(0).choice(shots, 4096, replace=False)])
    want = oc.sample_shots(0, ids)
    for i, s in enumerate(ids):
        assert np.array_equal(_column(got, int(s)), want[i]), int(s)
    # ragged tail: 10^6 = 15625 * 64 exactly, so every bit of the last word is live
    assert got.shape[1] == 15625


def _d15_oracle_ids(shots, n_words_run, total, seed):
    """Shots of a 2^20-shot d=15 batch for the oracle: every lane of the
    first and last word, lanes 0, 31 and 63 of the first and last word of
    every run of consecutive words one XCD takes (default launch: one word
    per workgroup, runs of n_words_run words), then seeded-random shots up to
    `total`."""
    words = (shots + 63) // 64
    fixed = set(range(64)) | set(range(64 * (words - 1), shots))
    for w0 in range(0, words, n_words_run):
        for w in (w0, min(words, w0 + n_words_run) - 1):
            fixed |= {64 * w + 0, 64 * w + 31, min(shots - 1, 64 * w + 63)}
    rng = np.random.default_rng(seed)
    ids = set(fixed)
    while len(ids) < total:
        ids |= set(int(x) for x in rng.choice(shots, total - len(ids), replace=False))
    return np.array(sorted(ids), dtype=np.int64)



@pytest.mark.parametrize("p", ["0.001", "0.005"])
def test_surface_d15_full_batch_both_paths(p):
    """Surface d=15, 15 rounds (3,585 rows, 101,489 variables), one whole
    2^20-shot batch at first_shot = 3 * 2^20, on the sparse (column-list)
    and the dense (bit-mask) path: every word of both equals the host
    sampler's (sp_sample_host, the same Eq. 4 from the host model), and 4,096
    shots spread over every XCD's run of words equal the oracle's.  The sparse
    launch writes rows 16,400 words apart, the row stride bench.py times."""
    text = surface_memory(15, 15, p).text()
    m = sp.Model(text)
    shots, first = 1 << 20, 3 << 20
    _say(f"surface d15 p={p} 2^20 shots: host sampler")
    host = m.sample_host(shots, seed=0, first_shot=first)
    assert host.shape == (3585, 16384)
    for path in ("sparse", "dense"):
        _say(f"surface d15 p={p} 2^20 shots: GPU {path}")
        dm = sp.DeviceModel(m, path=path)
        assert dm.launch == (8, 1) and dm.n_tiles == 1
        got = _gpu(dm, shots, seed=0, first_shot=first, ld=16400 if path == "sparse" else None)[:, :16384]
        bad = np.nonzero((got != host).any(axis=0))[0]
        assert bad.size == 0, (path, bad[:10])
        del dm, got
    ids = _d15_oracle_ids(shots, 16384 // 8, 4096, seed=int(float(p) * 1e4))
    _say(f"surface d15 p={p}: oracle on {len(ids)} shots")
    want = oracle.Circuit(text).sample_shots(0, first + ids)
    for i, s in enumerate(ids):
        assert np.array_equal(_column(host, int(s)), want[i]), int(s)


def test_surface_d15_last_partial_batch():
    """The last batch of 10^7 shots, 562,816 shots at first_shot = 9 * 2^20:
    every word equals the host sampler's, and 512 of its shots (the first and
    last 64, and random ones) equal the oracle's."""
    text = surface_memory(15, 15, "0.001").text()
    _say("surface d15 tail batch")
    m, dm, oc = _models(text, "sparse")
    shots, first = 10_000_000 - 9 * (1 << 20), 9 << 20
    got = _gpu(dm, shots, seed=0, first_shot=first)
    assert shots % 64 == 0 and got.shape[1] == shots // 64
    assert np.array_equal(got, m.sample_host(shots, seed=0, first_shot=first))
    rng = np.random.default_rng(9)
    idx = np.unique(np.concatenate([np.arange(64), np.arange(shots - 64, shots),
                                    rng.choice(shots, 384, replace=False)]))
    want = oc.sample_shots(0, first + idx)
    for i, s in enumerate(idx):
        assert np.array_equal(_column(got, int(s)), want[i]), int(s)


def test_surface_d7_ragged_batch():
    """A batch whose size is not a multiple of 64: the bits past the last
    shot are 0 and the live ones equal the oracle."""
    text = surface_memory(7, 7, "0.002").text()
    _, dm, oc = _models(text)
    shots = 100_003
    got = _gpu(dm, shots, seed=6, first_shot=5)
    rem = shots % 64
    assert (got[:, -1] >> np.uint64(rem) == 0).all()
    idx = np.array([0, 1, shots - 1, shots - rem, shots - rem - 1, 77_777])
    want = oc.sample_shots(6, 5 + idx)
    for i, s in enumerate(idx):
        assert np.array_equal(_column(got, int(s)), want[i]), int(s)


# ------------------------------------------------------------- invariants --

def test_paths_agree_on_d7():
    text = surface_memory(7, 7, "0.003").text()
    _say("d7 sparse vs dense")
    _, a, _ = _models(text, "sparse")
    _, b, _ = _models(text, "dense")
    assert np.array_equal(_gpu(a, 100_000, seed=4), _gpu(b, 100_000, seed=4))


def test_batch_split_is_identical():
    """Sampling is shot-addressable: words of one launch equal the launch of
    their shot range alone (keyed draws)."""
    text = surface_memory(5, 5, "0.005").text()
    _say("batch split")
    _, dm, _ = _models(text)
    whole = _gpu(dm, 64 * 1000, seed=9)
    part = _gpu(dm, 64 * 300, seed=9, first_shot=64 * 500)
    assert np.array_equal(whole[:, 500:800], part)


@pytest.mark.parametrize("shots", [1, 2, 63, 64, 65, 127, 129, 1000])
def test_ragged_sizes_and_unaligned_first_shot(shots):
    text = surface_memory(3, 3, "0.05").text()
    _, dm, oc = _models(text)
    first = 2 ** 33 + 17   # shot index above 2^32 exercises the counter's high word
    got = _gpu(dm, shots, seed=2 ** 40 + 5, first_shot=first)
    want = oc.sample(seed=2 ** 40 + 5, first_shot=first, shots=shots)
    assert np.array_equal(got, want)


def test_ld_padding_untouched():
    text = repetition_memory(5, 5, "0.02").text()
    _, dm, oc = _models(text)
    out = torch.full((dm.n_meas, 40), -1, dtype=torch.int64, device="cuda")
    dm.sample(1000, seed=1, out=out)
    torch.cuda.synchronize()
    got = sp.to_numpy_bits(out)
    assert np.array_equal(got[:, :16], oc.sample(seed=1, first_shot=0, shots=1000))
    assert (got[:, 16:] == np.uint64(2 ** 64 - 1)).all()


def test_zero_shots_and_no_measurements():
    _, dm, _ = _models(repetition_memory(3, 1, "0.1").text())
    out = torch.full((dm.n_meas, 1), 7, dtype=torch.int64, device="cuda")
    dm.sample(0, seed=1, out=out)
    torch.cuda.synchronize()
    assert (out == 7).all()
    m = sp.Model("H 0\nX_ERROR(0.5) 0\n")
    d = sp.DeviceModel(m)
    d.sample(100, seed=1, out=torch.zeros((1, 2), dtype=torch.int64, device="cuda"))
    torch.cuda.synchronize()


def test_deterministic_and_certain_channels():
    """p = 1 always fires, p = 0 never; a noiseless circuit returns c."""
    text = "X_ERROR(1) 0\nX_ERROR(0) 1\nDEPOLARIZE1(0) 2\nX 3\nM 0 1 2 3\n"
    _, dm, oc = _models(text)
    got = _gpu(dm, 4096, seed=5)
    assert (got[0] == np.uint64(2 ** 64 - 1)).all() and (got[1] == 0).all() and (got[2] == 0).all()
    assert (got[3] == np.uint64(2 ** 64 - 1)).all()
    assert np.array_equal(got, oc.sample(seed=5, first_shot=0, shots=4096))


def test_invalid_arguments_rejected():
    _, dm, _ = _models(repetition_memory(3, 1, "0.1").text())
    out = torch.zeros((dm.n_meas, 1), dtype=torch.int64, device="cuda")
    with pytest.raises(sp.SymphaseError):
        dm.sample(65, seed=1, out=out, ld=1)      # ld < words
    with pytest.raises(sp.SymphaseError):
        dm.sample(10, seed=1, first_shot=2 ** 64 - 5)


# ------------------------------------------------------------- statistics --

def test_fault_frequencies_match_channel_laws():
    """Outcome frequencies of directly measured faults are within 5 sigma of
    the channel law: X_ERROR(p) fires w.p. p; DEPOLARIZE1(p) flips Z w.p.
    2p/3 (X or Y); DEPOLARIZE2(p) flips the first qubit w.p. 8p/15."""
    n = 32
    text = (f"X_ERROR(0.01) " + " ".join(map(str, range(n))) + "\n"
            + f"DEPOLARIZE1(0.03) " + " ".join(map(str, range(n, 2 * n))) + "\n"
            + f"DEPOLARIZE2(0.15) " + " ".join(map(str, range(2 * n, 4 * n))) + "\n"
            + "M " + " ".join(map(str, range(4 * n))) + "\n")
    _, dm, _ = _models(text)
    shots = 1 << 20
    got = _gpu(dm, shots, seed=77)
    ones = np.array([sum(bin(int(w)).count("1") for w in row) for row in got[:, :4096]], dtype=np.float64)
    N = 4096 * 64
    checks = [(range(n), 0.01), (range(n, 2 * n), 0.02), (range(2 * n, 4 * n, 2), 0.08),
              (range(2 * n + 1, 4 * n, 2), 0.08)]
    for rows, q in checks:
        for r in rows:
            z = abs(ones[r] - N * q) / math.sqrt(N * q * (1 - q))
            assert z < 5, (r, ones[r], N * q)


@pytest.mark.parametrize("shape", [(1, 1), (4, 1), (8, 2), (16, 4), (3, 2), (16, 1)])
def test_launch_shape_invariance(shape):
    """The output depends only on (model, seed, first_shot, shots), never on
    the launch shape (waves per group, words per group)."""
    text = surface_memory(5, 3, "0.01").text()
    m, dm, oc = _models(text)
    ref = oc.sample(seed=12, first_shot=70, shots=5000)
    old = dm.launch
    try:
        dm.launch = shape
        got = _gpu(dm, 5000, seed=12, first_shot=70)
    finally:
        dm.launch = old
    assert np.array_equal(got, ref)


def test_launch_shape_rejects_oversized_slabs():
    m, dm, _ = _models(surface_memory(15, 15, "0.001").text())
    with pytest.raises(sp.SymphaseError):
        dm.launch = (8, 8)       # words_per_group must be 1, 2 or 4
    with pytest.raises(sp.SymphaseError):
        dm.launch = (0, 1)


@pytest.mark.parametrize("outputs", ["measurements", "detectors"])
def test_output_marginals_match_piling_up_lemma(outputs):
    """Surface d=5, 5 rounds, p = 5e-3, 2^20 shots on the GPU: every output
    row's frequency of ones is within 5 sigma of the piling-up closed form
    computed from the oracle (exact code probabilities, rows probed one code
    bit at a time)."""
    text = surface_memory(5, 5, "0.005", detectors=True).text()
    _say(f"piling-up marginals surface d5 {outputs} 2^20 shots")
    p = piling_up.expected_marginals(text, outputs)
    m, dm, oc = _models(text, "auto", outputs)
    shots = 1 << 20
    counts = piling_up.ones_per_row(_gpu(dm, shots, seed=17), shots)
    piling_up.check_marginals(counts, shots, p)


def test_noise_model_circuit_full():
    """A noiseless surface code (d=5, 5 rounds) with the noise model added
    through the C ABI (distinct probabilities per channel class), sampled on
    the GPU: every word equals the oracle's samples of the same circuit with
    the channels written out in the text."""
    noisy = surface_memory(5, 5, "0.001", detectors=True).text()
    clean = "\n".join(l for l in noisy.splitlines() if not l.startswith(("X_ERROR", "DEPOLARIZE"))) + "\n"
    ps = {"p_1q": "0.002", "p_2q": "0.006", "p_meas": "0.01", "p_reset": "0.003", "p_idle": "0.0005"}
    _say("noise model surface d5 20000 shots")
    circ = sp.Circuit(clean).with_noise(**ps)
    m = sp.Model(circ, outputs="detectors")
    dm = sp.DeviceModel(m)
    want_text = _written_noise(clean, ps, circ.n_qubits)
    oc = oracle.Circuit(want_text, outputs="detectors")
    got = _gpu(dm, 20_000, seed=2)
    assert np.array_equal(got, oc.sample(seed=2, first_shot=0, shots=20_000))


def _written_noise(text, ps, n_qubits):
    """The noise model's placement written out as circuit text."""
    out, touched = [], set()
    for line in text.splitlines():
        parts = line.split()
        head, targets = parts[0], parts[1:]
        if head == "TICK":
            idle = [q for q in range(n_qubits) if q not in touched]
            if idle:
                out.append(f"DEPOLARIZE1({ps['p_idle']}) " + " ".join(map(str, idle)))
            touched = set()
            out.append(line)
            continue
        if head in ("H", "S", "CX", "M", "R", "MR"):
            touched |= {int(q) for q in targets}
        if head in ("M", "MR"):
            out.append(f"X_ERROR({ps['p_meas']}) " + " ".join(targets))
        out.append(line)
        if head in ("H", "S"):
            out.append(f"DEPOLARIZE1({ps['p_1q']}) " + " ".join(targets))
        if head == "CX":
            out.append(f"DEPOLARIZE2({ps['p_2q']}) " + " ".join(targets))
        if head in ("R", "MR"):
            out.append(f"X_ERROR({ps['p_reset']}) " + " ".join(targets))
    return "\n".join(out) + "\n"


# ------------------------------------------------------------- row tiles --

@pytest.mark.parametrize("path", ["sparse", "dense"])
@pytest.mark.parametrize("tile_rows", [64, 128])
def test_row_tiles_equal_untiled_and_oracle(path, tile_rows):
    """Surface d=5, 5 rounds, p = 5e-3, split into row tiles of 64 or 128
    rows (each tile draws only the locations that reach its rows): every
    word equals the one-tile model's and the oracle's, for measurement and
    detector rows."""
    text = surface_memory(5, 5, "0.005", detectors=True).text()
    for outputs in ("measurements", "detectors"):
        _say(f"row tiles {tile_rows} path={path} outputs={outputs}")
        m = sp.Model(text, outputs=outputs)
        dm = sp.DeviceModel(m, path=path, tile_rows=tile_rows)
        assert dm.n_tiles == math.ceil(m.n_meas / tile_rows)
        ref = sp.DeviceModel(m, path=path)
        assert ref.n_tiles == 1
        got = _gpu(dm, 10_000, seed=3, first_shot=640)
        assert np.array_equal(got, _gpu(ref, 10_000, seed=3, first_shot=640))
        assert np.array_equal(got, oracle.Circuit(text, outputs=outputs).sample(seed=3, first_shot=640, shots=10_000))


@pytest.mark.parametrize("path", ["sparse", "dense"])
def test_row_tiles_one_launch_shapes_and_ragged_range(path):
    """All row tiles are sampled by one launch: for every launch shape, a
    ragged shot count, a padded output stride and a shot range that crosses
    2^32, the tiled model (tiles of 64 rows, the last one partial) writes
    exactly the one-tile model's words, and the padding stays untouched."""
    text = surface_memory(5, 5, "0.005", detectors=True).text()
    m = sp.Model(text, outputs="detectors")
    dm = sp.DeviceModel(m, path=path, tile_rows=64)
    assert dm.n_tiles == math.ceil(m.n_meas / 64) and m.n_meas % 64
    ref = sp.DeviceModel(m, path=path)
    shots, first, ld = 1000, 2**32 - 320, 19
    want = _gpu(ref, shots, seed=11, first_shot=first)
    for launch in [(1, 1), (4, 2), (8, 1), (8, 2), (16, 4)]:
        _say(f"one-launch row tiles path={path} launch={launch}")
        dm.launch = launch
        out = torch.full((m.n_meas, ld), 0x5A5A, dtype=torch.int64, device="cuda")
        dm.sample(shots, seed=11, first_shot=first, out=out)
        torch.cuda.synchronize()
        got = sp.to_numpy_bits(out)
        assert np.array_equal(got[:, :16], want), launch
        assert (got[:, 16:] == 0x5A5A).all(), launch


def _many_rows_circuit(rounds=5000):
    """25,000 recorded measurements: qubit 0 (random at first, then repeated
    without reset, so its outcome's symbol and its sparse X faults reach
    rows across the whole circuit) and four qubits measured and reset every
    round."""
    lines = ["H 0", "CX 0 1"]
    for k in range(rounds):
        if k % 100 == 0:
            lines.append("X_ERROR(0.05) 0")
        lines += ["DEPOLARIZE1(0.002) 1 2 3 4", "CX 1 2", "M 0", "MR 1 2 3 4"]
    return "\n".join(lines) + "\n"


def test_auto_row_tiles_beyond_one_slab():
    """25,000 output rows, more than one LDS slab holds: the upload splits
    them into row tiles of 3,840 rows, and 2,048 shots equal the oracle's
    word for word (every tile, every row)."""
    text = _many_rows_circuit()
    _say("auto row tiles 25000 rows 2048 shots")
    m = sp.Model(text)
    assert m.n_meas == 25_000
    dm = sp.DeviceModel(m)
    assert (dm.n_tiles, dm.tile_rows_max) == (7, 3840)
    got = _gpu(dm, 2048, seed=21, first_shot=64)
    assert np.array_equal(got, oracle.Circuit(text).sample(seed=21, first_shot=64, shots=2048))


def test_tile_rows_argument_checked():
    m = sp.Model(surface_memory(3, 3, "0.01").text())
    for bad in (63, 100, 19_520):
        with pytest.raises(sp.SymphaseError) as e:
            sp.DeviceModel(m, tile_rows=bad)
        assert e.value.code == sp._capi.SP_E_INVALID


def test_paper_fig3_n700_device_init_and_row_tiles():
    """Fig. 3a at n = 700 (25,200 rows): Initialization on the GPU with the
    tableau in device memory (too large for LDS) gives the host's model,
    and sampling in row tiles gives 48 of 2^16 shots equal to the oracle's."""
    text = random_layered_circuit(700, seed=3, cnot_pairs=5).text()
    _say("fig3a n=700 device init + row tiles, 48 sampled shots")
    m = sp.Model(text, init="device")
    host = sp.Model(text)
    assert (m.n_meas, m.n_vars, m.dims.nnz) == (host.n_meas, host.n_vars, host.dims.nnz)
    for x, y in zip(m.export_csc(), host.export_csc()):
        assert np.array_equal(x, y)
    dm = sp.DeviceModel(m)
    assert dm.n_tiles == math.ceil(m.n_meas / 3840)
    shots = 1 << 16
    got = _gpu(dm, shots, seed=5)
    ids = np.sort(np.random.default_rng(0).choice(shots, 48, replace=False))
    want = oracle.Circuit(text).sample_shots(seed=5, shot_ids=ids)
    for i, s in enumerate(ids):
        assert np.array_equal(_column(got, int(s)), want[i]), int(s)


def test_paper_fig3c_n700_device_init_sampled():
    """Fig. 3c at n = 700 (980,000 fault variables, 25,200 rows): the model
    built on the GPU (tableau in device memory, dense phase rows of about
    15,000 words), sampled in row tiles, gives 16 of 4,096 shots equal to the
    oracle's (the host pass takes minutes at this size)."""
    text = random_layered_circuit(700, seed=0, p_dep="0.001").text()
    _say("fig3c n=700 device init (about 10 s)")
    m = sp.Model(text, init="device")
    dm = sp.DeviceModel(m)
    assert dm.n_tiles > 1
    got = _gpu(dm, 4096, seed=7)
    ids = np.array([0, 1, 63, 64, 100, 1000, 2047, 2048, 3000, 3333, 4000, 4095, 17, 555, 777, 1234])
    _say("fig3c n=700 oracle, 16 shots")
    want = oracle.Circuit(text).sample_shots(seed=7, shot_ids=ids)
    for i, s in enumerate(ids):
        assert np.array_equal(_column(got, int(s)), want[i]), int(s)
