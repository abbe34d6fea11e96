"""Pins for the CPU oracle: each test ties it to something other than itself
(the paper's worked examples, a brute-force statevector, closed forms,
published known-answer vectors, an installed library, statistics)."""

from __future__ import annotations

import itertools
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import piling_up
import statevector
from golden_io import example, rows
from workloads import random_clifford_circuit, repetition_memory, surface_memory

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------- Philox --

def test_philox_known_answers():
    """Published Philox4x32-10 known-answer vectors (Salmon et al., SC'11)."""
    n = 0
    for r in rows("philox4x32_10_kat.txt"):
        vals = [int(v, 16) for v in r]
        ctr, key, want = vals[:4], vals[4:6], tuple(vals[6:10])
        assert oracle.philox4x32_10(ctr, key) == want
        n += 1
    assert n == 3


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/rocrand"),
                    reason="needs g++ and rocRAND headers")
def test_philox_matches_rocrand(tmp_path):
    """Third opinion: rocRAND's host-callable Philox4x32-10 engine."""
    exe = tmp_path / "rr"
    subprocess.check_call(["g++", "-O1", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                           os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", str(exe)])
    rng = np.random.default_rng(7)
    cases = rng.integers(0, 2 ** 32, size=(300, 6), dtype=np.uint64)
    cases[:5, 2:4] = 0
    inp = "\n".join(" ".join(f"{int(v):08x}" for v in c) for c in cases) + "\n"
    outp = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    for c, line in zip(cases, outp.strip().splitlines()):
        want = tuple(int(v, 16) for v in line.split())
        assert oracle.philox4x32_10([int(v) for v in c[:4]], [int(v) for v in c[4:]]) == want


def test_draw_counter_layout():
    """u(seed, shot, l) is word l mod 4 of the block at counter
    (l div 4, shot lo, shot hi, 0) under key (seed lo, seed hi)."""
    seed, shot = 0x0123456789ABCDEF, (5 << 32) | 77
    for loc in (0, 1, 2, 3, 4, 7, 1000, 2 ** 33 + 2):
        blk = oracle.philox4x32_10([loc >> 2 & 0xFFFFFFFF, shot & 0xFFFFFFFF, shot >> 32, 0],
                                   [seed & 0xFFFFFFFF, seed >> 32])
        assert oracle.draw(seed, shot, loc) == blk[loc & 3]


# ----------------------------------------------------------- thresholds --

def test_thresholds_closed_forms():
    n = 0
    for r in rows("thresholds.txt"):
        p, m, T = r[0], int(r[1]), [int(v) for v in r[2:]]
        assert oracle.thresholds(p, m) == T, p
        n += 1
    assert n >= 10


@pytest.mark.parametrize("bad", ["1.5", "-0.1", "abc", "1e", "0.1.2", "", "2e0"])
def test_thresholds_reject_bad_literals(bad):
    with pytest.raises(oracle.OracleError):
        oracle.thresholds(bad, 1)


def test_thresholds_monotone_and_bounded():
    for p in ("0.0001", "0.00123", "0.01", "0.3", "0.999999"):
        for m in (1, 3, 15):
            T = oracle.thresholds(p, m)
            assert all(a <= b for a, b in zip(T, T[1:]))
            # floor(p * 2^32) within m of T_m
            assert abs(T[-1] - math.floor(float(p) * 2 ** 32)) <= 2


# ------------------------------------------------------- paper examples --

@pytest.mark.parametrize("name", ["fig1.txt", "bell.txt"])
def test_paper_examples_exhaustive(name):
    """Every assignment of the example's symbols gives the printed outcomes."""
    text, symbols, outcomes = example(name)
    c = oracle.Circuit(text)
    names = sorted(symbols)
    for vals in itertools.product([0, 1], repeat=len(names)):
        codes = np.zeros(c.n_locs, dtype=np.uint8)
        env = dict(zip(names, vals))
        for nm, v in env.items():
            loc, bit = symbols[nm]
            codes[loc] |= v << bit
        out, _ = c.run_codes(codes, check_invariants=True)
        want = [sum(env[s] for s in terms) % 2 for terms in outcomes]
        assert list(out) == want, (name, env)


def test_bell_first_measurement_is_random():
    text, _, _ = example("bell.txt")
    c = oracle.Circuit(text)
    _, wr = c.run_codes(np.zeros(c.n_locs, dtype=np.uint8))
    assert list(wr) == [0, 0, 1, 0]


# ------------------------------------------------------------ brute force --

@settings(max_examples=250, deadline=None)
@given(seed=st.integers(0, 2 ** 31), n=st.integers(1, 6), n_ops=st.integers(1, 45))
def test_oracle_matches_statevector(seed, n, n_ops):
    """Forced-outcome statevector on random noisy stabilizer circuits: the
    oracle's deterministic outcomes have probability 1, its random ones
    probability 1/2, and the recorded outcomes agree."""
    circ = random_clifford_circuit(seed, n, n_ops)
    text = circ.text()
    c = oracle.Circuit(text)
    rng = np.random.default_rng(seed + 1)
    kinds = c.location_kinds()
    for _ in range(3):
        codes = np.array([rng.integers(0, 2 ** oracle.CODE_BITS[int(k)]) for k in kinds], dtype=np.uint8)
        got, got_rnd = c.run_codes(codes, check_invariants=True)
        want, want_rnd = statevector.run(text, c.n_qubits, codes)
        assert np.array_equal(got, want)
        assert np.array_equal(got_rnd, want_rnd)


@settings(max_examples=200, deadline=None)
@given(seed=st.integers(0, 2 ** 31), n=st.integers(1, 6), n_ops=st.integers(1, 45))
def test_oracle_matches_statevector_with_feedback(seed, n, n_ops):
    """The same with Paulis controlled by earlier records (CX/CY/CZ
    rec[-k] q): the statevector applies the Pauli matrix when the recorded
    outcome it reached was 1."""
    text = random_clifford_circuit(seed, n, n_ops, feedback=True, detectors=True).text()
    c = oracle.Circuit(text)
    rng = np.random.default_rng(seed + 2)
    kinds = c.location_kinds()
    for _ in range(3):
        codes = np.array([rng.integers(0, 2 ** oracle.CODE_BITS[int(k)]) for k in kinds], dtype=np.uint8)
        got, got_rnd = c.run_codes(codes, check_invariants=True)
        want, want_rnd = statevector.run(text, c.n_qubits, codes)
        assert np.array_equal(got, want)
        assert np.array_equal(got_rnd, want_rnd)


@pytest.mark.parametrize("pauli,prep,unprep", [("X", "", ""), ("Y", "", ""), ("Z", "H 1\n", "H 1\n"),
                                               ("Y", "H 1\n", "H 1\n")])
def test_feedback_copies_a_random_outcome(pauli, prep, unprep):
    """A random outcome m0 (H then M), then P on a fresh qubit controlled by
    it: with the qubit prepared so that P flips its measured value, the
    second outcome equals m0 in every shot, and m0 is fair."""
    text = f"H 0\nM 0\n{prep}C{pauli} rec[-1] 1\n{unprep}M 1\n"
    c = oracle.Circuit(text)
    out = c.sample(seed=5, first_shot=0, shots=4096)
    assert np.array_equal(out[0], out[1])
    ones = sum(bin(int(w)).count("1") for w in out[0])
    assert abs(ones - 2048) < 5 * math.sqrt(1024)


@pytest.mark.parametrize("d,rounds", [(3, 3), (5, 4)])
def test_repetition_detectors_closed_form(d, rounds):
    """Repetition memory with detectors: with no fault every detector and
    the observable are 0; a single X fault on data qubit j before round t
    fires exactly the detectors of the ancillas next to j in round t (an
    ancilla compares consecutive rounds, and the final parity check cancels
    the flip), and flips the observable iff j = 0."""
    circ = repetition_memory(d, rounds, "0.01", detectors=True)
    c = oracle.Circuit(circ.text(), outputs="detectors")
    na = d - 1
    assert (c.n_detectors, c.n_observables) == ((rounds + 1) * na, 1)
    per_round = d + na + 2 * na
    zero = np.zeros(c.n_locs, dtype=np.uint8)
    out, _ = c.run_codes(zero)
    assert not c.rows_from_outcomes(out).any()
    for t in range(rounds):
        for j in range(d):
            codes = zero.copy()
            codes[t * per_round + j] = 1
            rows = c.rows_from_outcomes(c.run_codes(codes)[0])
            want = np.zeros(c.n_rows, dtype=np.uint8)
            for i in (j - 1, j):
                if 0 <= i < na:
                    want[t * na + i] = 1
            want[-1] = int(j == 0)
            assert np.array_equal(rows, want), (t, j)


@pytest.mark.parametrize("reset", ["reset", "feedback"])
@pytest.mark.parametrize("d,rounds", [(3, 3), (5, 3)])
def test_surface_noiseless_detectors_are_zero(d, rounds, reset):
    """p = 0 memory-Z with detectors: every detector and the observable is
    0 in every shot, although the first round's X checks are random; also
    when the ancillas are reset by X controlled by their last outcome."""
    circ = surface_memory(d, rounds, "0", detectors=True, reset=reset)
    det = oracle.Circuit(circ.text(), outputs="detectors")
    meas = oracle.Circuit(circ.text())
    assert det.n_detectors == circ.n_detectors and det.n_observables == 1
    assert not det.sample(seed=1, first_shot=0, shots=1024).any()
    assert meas.sample(seed=1, first_shot=0, shots=1024).any()


def test_statevector_catches_planted_phase_error():
    """The brute-force check is sharp enough to see a single wrong phase:
    flipping one outcome bit of the oracle's result must be detected."""
    circ = random_clifford_circuit(3, 4, 30)
    text = circ.text()
    c = oracle.Circuit(text)
    codes = np.zeros(c.n_locs, dtype=np.uint8)
    got, _ = c.run_codes(codes)
    want, _ = statevector.run(text, c.n_qubits, codes)
    assert np.array_equal(got, want)
    bad = got.copy()
    bad[-1] ^= 1
    assert not np.array_equal(bad, want)


# ----------------------------------------------------------- closed forms --

@pytest.mark.parametrize("d,rounds", [(3, 3), (5, 4), (4, 1)])
def test_repetition_code_closed_form(d, rounds):
    """Bit-flip repetition memory: ancilla j in round t reports
    g_tj + sum_{t'<=t} (f_t'j + f_t'(j+1)); final data i reports
    h_i + sum_t f_ti (textbook syndrome of accumulated data flips)."""
    circ = repetition_memory(d, rounds, "0.01")
    c = oracle.Circuit(circ.text())
    per_round = d + (d - 1) + 2 * (d - 1)   # X_ERROR data, X_ERROR anc, M anc, R anc
    assert c.n_locs == rounds * per_round + 2 * d
    rng = np.random.default_rng(d * 100 + rounds)
    for _ in range(200):
        codes = np.zeros(c.n_locs, dtype=np.uint8)
        f = rng.integers(0, 2, size=(rounds, d))
        g = rng.integers(0, 2, size=(rounds, d - 1))
        h = rng.integers(0, 2, size=d)
        for t in range(rounds):
            base = t * per_round
            codes[base:base + d] = f[t]
            codes[base + d:base + 2 * d - 1] = g[t]
            codes[base + 2 * d - 1:base + per_round] = rng.integers(0, 2, size=2 * (d - 1))
        codes[rounds * per_round:rounds * per_round + d] = h
        codes[rounds * per_round + d:] = rng.integers(0, 2, size=d)
        out, wr = c.run_codes(codes)
        assert wr.sum() == 0
        want = []
        acc = np.zeros(d, dtype=np.int64)
        for t in range(rounds):
            acc ^= f[t]
            want += [int(g[t, j] ^ acc[j] ^ acc[j + 1]) for j in range(d - 1)]
        want += [int(h[i] ^ acc[i]) for i in range(d)]
        assert list(out) == want


@pytest.mark.parametrize("d,rounds", [(3, 3), (5, 2)])
def test_surface_noiseless_structure(d, rounds):
    """p = 0 memory-Z: Z checks always report 0; X checks are random in the
    first round and repeat it afterwards; the final data parities of every Z
    check are 0; exactly (d^2-1)/2 measurements are random in round one and
    (d^2-1)/2 among the final data measurements."""
    circ = surface_memory(d, rounds, "0")
    c = oracle.Circuit(circ.text())
    n_chk = d * d - 1
    from workloads.circuits import _surface_layout
    checks = _surface_layout(d)
    kinds = c.location_kinds()
    meas_locs = [i for i, k in enumerate(kinds) if k == oracle.LOC_M]
    rng = np.random.default_rng(1)
    for trial in range(4):
        codes = rng.integers(0, 2, size=c.n_locs).astype(np.uint8)
        codes[[i for i, k in enumerate(kinds) if k not in oracle.MEAS_KINDS]] = 0
        out, wr = c.run_codes(codes, check_invariants=(d == 3 and trial == 0))
        m = out[: rounds * n_chk].reshape(rounds, n_chk)
        final = out[rounds * n_chk:]
        for i, (typ, corners) in enumerate(checks):
            if typ == "Z":
                assert (m[:, i] == 0).all()
                assert sum(int(final[q]) for q in corners.values()) % 2 == 0
            else:
                assert (m[:, i] == m[0, i]).all()
        rnd_m = wr[meas_locs]
        assert rnd_m[:n_chk].sum() == n_chk // 2
        assert rnd_m[n_chk:rounds * n_chk].sum() == 0
        assert rnd_m[rounds * n_chk:].sum() == n_chk // 2
        # a random outcome is the drawn bit
        for j, l in enumerate(meas_locs):
            if wr[l]:
                assert out[j] == codes[l] & 1


# ------------------------------------------------------------- statistics --

@pytest.mark.parametrize("name,p,m", [("X_ERROR", "0.01", 1), ("DEPOLARIZE1", "0.03", 3),
                                      ("DEPOLARIZE2", "0.15", 15), ("Z_ERROR", "0.5", 1)])
def test_code_frequencies(name, p, m):
    """Drawn codes follow the channel law of Section 3.1 (each non-identity
    outcome with p/m) within a 5-sigma binomial bound."""
    q = 2 if name == "DEPOLARIZE2" else 1
    text = f"{name}({p}) " + " ".join(str(i) for i in range(8 * q)) + "\nM 0\n"
    c = oracle.Circuit(text)
    n_shots = 6000
    counts = np.zeros(m + 1, dtype=np.int64)
    for s in range(n_shots):
        codes = c.draw_codes(11, s)[:8]
        counts += np.bincount(codes, minlength=m + 1)
    N = n_shots * 8
    for k in range(m + 1):
        prob = (1 - float(p)) if k == 0 else float(p) / m
        z = abs(counts[k] - N * prob) / math.sqrt(N * prob * (1 - prob))
        assert z < 5, (k, counts[k], N * prob)


def test_random_measurement_bit_is_fair():
    c = oracle.Circuit("H 0\nM 0\n")
    out = c.sample(seed=3, first_shot=0, shots=20000)
    ones = sum(bin(int(w)).count("1") for w in out[0])
    assert abs(ones - 10000) / math.sqrt(5000) < 5


# ----------------------------------------------------------- packed output --

def test_sample_layout_matches_single_shots():
    circ = surface_memory(3, 2, "0.02")
    c = oracle.Circuit(circ.text())
    shots, first = 150, 1000
    packed = c.sample(seed=5, first_shot=first, shots=shots, ld=4, n_threads=3)
    assert packed.shape == (c.n_meas, 4)
    per = c.sample_shots(5, np.arange(first, first + shots))
    for i in range(shots):
        col = (packed[:, i // 64] >> np.uint64(i % 64)) & np.uint64(1)
        assert np.array_equal(col.astype(np.uint8), per[i])
    # bits past `shots` and the padding word are zero
    assert (packed[:, 3] == 0).all()
    assert (packed[:, 2] >> np.uint64(shots - 128) == 0).all()


def test_sample_is_shot_addressable():
    circ = repetition_memory(3, 3, "0.05")
    c = oracle.Circuit(circ.text())
    whole = c.sample(seed=9, first_shot=0, shots=256)
    part = c.sample(seed=9, first_shot=128, shots=128)
    assert np.array_equal(whole[:, 2:], part)


@pytest.mark.parametrize("text", ["T 0\n", "CX 0\n", "CX 1 1\n", "X_ERROR 0\n", "H(0.1) 0\n",
                                  "X_ERROR(1.2) 0\n", "M a\n", "DEPOLARIZE2(0.1) 0 1 2\n",
                                  "TICK 3\n", "CX rec[-1] 0\n", "M 0\nCX rec[-2] 1\n", "M 0\nCX 1 rec[-1]\n",
                                  "CZ 0 1\n", "M 0\nDETECTOR 0\n", "M 0\nOBSERVABLE_INCLUDE rec[-1]\n",
                                  "M 0\nOBSERVABLE_INCLUDE(a) rec[-1]\n", "M 0\nH rec[-1]\n",
                                  "M 0\nDETECTOR rec[0]\n"])
def test_parse_rejects(text):
    with pytest.raises(oracle.OracleError):
        oracle.Circuit(text)


@pytest.mark.parametrize("name,circ,outputs", [
    ("surf3_meas", surface_memory(3, 3, "0.02", detectors=True), "measurements"),
    ("surf3_det", surface_memory(3, 3, "0.02", detectors=True), "detectors"),
    ("rep5_det", repetition_memory(5, 5, "0.03", detectors=True), "detectors"),
    ("random_all_channels", random_clifford_circuit(21, 6, 90, feedback=True, detectors=True), "measurements"),
])
def test_output_marginals_match_piling_up_lemma(name, circ, outputs):
    """Per-row frequencies of the oracle's sampled outputs against the
    piling-up closed form (independent locations, exact code
    probabilities, rows built by probing): within 5 sigma, and rows of
    probability 0 or 1 constant."""
    text = circ.text()
    p = piling_up.expected_marginals(text, outputs)
    assert ((p > 0.01) & (p < 0.99)).sum() >= 5   # the check has teeth
    oc = oracle.Circuit(text, outputs=outputs)
    shots = 40_000
    counts = piling_up.ones_per_row(oc.sample(seed=5, first_shot=0, shots=shots), shots)
    piling_up.check_marginals(counts, shots, p)
