"""Circuit-text generators for the sampling workloads.

Text format (one instruction per line, '#' starts a comment)::

    NAME t0 t1 ...            gates / measurements / resets
    NAME(p) t0 t1 ...         noise channels with probability p (exact decimal)
    TICK                      layer separator (no effect on the state)

Instruction set:
  H S X Y Z            single-qubit Clifford and Pauli gates
  CX                   CNOT, targets taken in (control, target) pairs
  M                    recorded Z-basis measurement
  R                    reset to |0> (not recorded)
  MR                   recorded Z measurement, then reset
  X_ERROR(p) Y_ERROR(p) Z_ERROR(p)   single Pauli with probability p
  DEPOLARIZE1(p)       X, Y, Z each with probability p/3
  DEPOLARIZE2(p)       each of the 15 non-identity two-qubit Paulis w.p. p/15,
                       targets taken in pairs
  CX/CY/CZ rec[-k] q   X/Y/Z on q when the k-th most recent recorded
                       measurement was 1 (a Pauli controlled by an outcome)
  DETECTOR rec[-k] ... XOR of recorded measurements (a detector)
  OBSERVABLE_INCLUDE(i) rec[-k] ...  XOR of records into observable i

The gate set is that of stabilizer circuits (H, S, CNOT, Z measurement,
|0...0> start) from the paper's background section, plus the Pauli gates and
Pauli noise channels of its phase-symbolization section.  Probabilities are
written as decimal literals so that every reader derives the same exact
rational number from them.
"""

from __future__ import annotations

import json
import math
from dataclasses import dataclass, field

import numpy as np


def format_prob(p: float) -> str:
    """Decimal literal for a probability, 6 significant digits."""
    if p < 0 or p > 1:
        raise ValueError(f"probability out of range: {p}")
    if p == 0:
        return "0"
    s = f"{p:.6g}"
    return s


@dataclass
class Circuit:
    """A circuit under construction; `text()` renders it."""

    lines: list = field(default_factory=list)
    n_qubits: int = 0
    n_meas: int = 0
    meta: dict = field(default_factory=dict)
    n_detectors: int = 0
    n_observables: int = 0

    def op(self, name: str, targets, p: float | str | None = None):
        targets = [int(t) for t in targets]
        if not targets and name != "TICK":
            return self
        if targets:
            self.n_qubits = max(self.n_qubits, max(targets) + 1)
        if name in ("M", "MR"):
            self.n_meas += len(targets)
        if p is None:
            head = name
        else:
            ps = p if isinstance(p, str) else format_prob(p)
            head = f"{name}({ps})"
        self.lines.append(" ".join([head] + [str(t) for t in targets]))
        return self

    def tick(self):
        self.lines.append("TICK")
        return self

    def feedback(self, pauli: str, pairs):
        """Pauli X/Y/Z on q when record rec[-k] was 1, for each (k, q)."""
        if pauli not in ("X", "Y", "Z"):
            raise ValueError(pauli)
        tg = []
        for k, q in pairs:
            if not 1 <= int(k) <= self.n_meas:
                raise ValueError(f"rec[-{k}] with {self.n_meas} measurements recorded")
            tg += [f"rec[-{int(k)}]", str(int(q))]
            self.n_qubits = max(self.n_qubits, int(q) + 1)
        if tg:
            self.lines.append(" ".join([f"C{pauli}"] + tg))
        return self

    def _recs(self, ks):
        for k in ks:
            if not 1 <= int(k) <= self.n_meas:
                raise ValueError(f"rec[-{k}] with {self.n_meas} measurements recorded")
        return [f"rec[-{int(k)}]" for k in ks]

    def detector(self, ks, coords=None):
        head = "DETECTOR" if coords is None else "DETECTOR(" + ", ".join(str(x) for x in coords) + ")"
        self.lines.append(" ".join([head] + self._recs(ks)))
        self.n_detectors += 1
        return self

    def observable(self, index: int, ks):
        self.lines.append(" ".join([f"OBSERVABLE_INCLUDE({int(index)})"] + self._recs(ks)))
        self.n_observables = max(self.n_observables, int(index) + 1)
        return self

    def text(self) -> str:
        return "\n".join(self.lines) + "\n"


# --------------------------------------------------------------------------
# The paper's two worked examples.
# --------------------------------------------------------------------------

def fig1_example(p: str = "0.1") -> Circuit:
    """Figure 1: GHZ encode on 4 qubits, faults Z^{s1} on q1 and X^{s2..s4}
    on q2..q4, decode, H on q1, measure all.  Printed outcomes:
    m1=s1, m2=s2, m3=s2+s3, m4=s3+s4."""
    c = Circuit()
    c.op("H", [0]).op("CX", [0, 1]).op("CX", [1, 2]).op("CX", [2, 3])
    c.op("Z_ERROR", [0], p).op("X_ERROR", [1, 2, 3], p)
    c.op("CX", [2, 3]).op("CX", [1, 2]).op("CX", [0, 1]).op("H", [0])
    c.op("M", [0, 1, 2, 3])
    return c


def bell_example(p: str = "0.1") -> Circuit:
    """Section 3.1 example: H, CNOT, X^{s1} on q1, X^{s2} on q2, measure both.
    Printed outcomes: m1 = s3 (random), m2 = s1+s2+s3."""
    c = Circuit()
    c.op("H", [0]).op("CX", [0, 1])
    c.op("X_ERROR", [0], p).op("X_ERROR", [1], p)
    c.op("M", [0]).op("M", [1])
    return c


# --------------------------------------------------------------------------
# QEC memory experiments.
# --------------------------------------------------------------------------

def repetition_memory(d: int, rounds: int, p: float | str = 1e-3, detectors: bool = False) -> Circuit:
    """Bit-flip repetition-code memory.

    Data qubits 0,2,..,2(d-1); ancilla 2i+1 checks data 2i and 2i+2.  Each
    round: X_ERROR(p) on data, CNOT data->ancilla (ancilla 2i+1 collects
    2i then 2i+2), X_ERROR(p) on the ancillas, M ancillas, R ancillas.
    After the rounds: X_ERROR(p) on data, M data.

    With detectors: each round, one detector per ancilla (its outcome, XORed
    with its previous outcome after the first round); after the data
    measurement, one per ancilla comparing the parity of its two data qubits
    with its last outcome; observable 0 = data qubit 0.  Without noise every
    detector and the observable are 0.
    """
    if d < 2 or rounds < 1:
        raise ValueError("need d >= 2 and rounds >= 1")
    data = [2 * i for i in range(d)]
    anc = [2 * i + 1 for i in range(d - 1)]
    c = Circuit(meta={"family": "repetition", "d": d, "rounds": rounds, "p": str(p)})
    for r in range(rounds):
        c.op("X_ERROR", data, p)
        pairs = []
        for i, a in enumerate(anc):
            pairs += [data[i], a]
        c.op("CX", pairs)
        pairs = []
        for i, a in enumerate(anc):
            pairs += [data[i + 1], a]
        c.op("CX", pairs)
        c.op("X_ERROR", anc, p)
        c.op("M", anc)
        if detectors:
            na = d - 1
            for i in range(na):
                ks = [na - i] if r == 0 else [na - i, 2 * na - i]
                c.detector(ks, coords=(2 * i + 1, r))
        c.op("R", anc)
        c.tick()
    c.op("X_ERROR", data, p)
    c.op("M", data)
    if detectors:
        na = d - 1
        for i in range(na):
            c.detector([d - i, d - i - 1, d + na - i], coords=(2 * i + 1, rounds))
        c.observable(0, [d])
    c.n_qubits = 2 * d - 1
    return c


def _surface_layout(d: int):
    """Rotated surface code of odd distance d.

    Data qubit (r, c), 0 <= r, c < d, has index r*d + c.  A plaquette sits on
    the face whose top-left corner is (r, c), r, c in [-1, d-1]; its type is
    X when r+c is even, Z when odd.  All interior faces are kept (weight 4);
    on the top/bottom edges only X faces are kept, on the left/right edges
    only Z faces (weight 2).  That gives (d-1)^2 + 2(d-1) = d^2 - 1 checks.
    Returns a list of (type, {corner: data index}) in face order.
    """
    checks = []
    for r in range(-1, d):
        for c in range(-1, d):
            typ = "X" if (r + c) % 2 == 0 else "Z"
            corners = {}
            for name, (dr, dc) in (("NW", (0, 0)), ("NE", (0, 1)),
                                   ("SW", (1, 0)), ("SE", (1, 1))):
                rr, cc = r + dr, c + dc
                if 0 <= rr < d and 0 <= cc < d:
                    corners[name] = rr * d + cc
            interior = 0 <= r < d - 1 and 0 <= c < d - 1
            if interior:
                checks.append((typ, corners))
            elif len(corners) == 2:
                top_bottom = r in (-1, d - 1)
                if (top_bottom and typ == "X") or (not top_bottom and typ == "Z"):
                    checks.append((typ, corners))
    return checks


# CNOT order per check type; with these orders no data qubit is touched twice
# in one layer (checked below), and a fault on an X ancilla half-way through
# spreads along the direction that does not shorten the logical operator.
_ORDER = {"X": ("NW", "NE", "SW", "SE"), "Z": ("NW", "SW", "NE", "SE")}


def _logical_z_support(d: int, checks) -> list:
    """Data qubits of a Z-type logical: a full row or column of the d x d
    data grid that overlaps every X check on an even number of qubits."""
    cands = [[r * d + col for col in range(d)] for r in range(d)] + \
            [[r * d + col for r in range(d)] for col in range(d)]
    for cand in cands:
        s = set(cand)
        if all(len(s & set(corners.values())) % 2 == 0 for typ, corners in checks if typ == "X"):
            return cand
    raise AssertionError("no Z logical among rows and columns")


def surface_memory(d: int, rounds: int, p: float | str = 1e-3, detectors: bool = False,
                   reset: str = "reset") -> Circuit:
    """Rotated surface-code memory-Z experiment with circuit-level noise.

    Per round, TICK-separated layers:
      [R anc | H on X-anc | CX x4 | H on X-anc | M anc]
    Noise: X_ERROR(p) after R and before M; DEPOLARIZE1(p) after each H and
    on every qubit idle in a layer; DEPOLARIZE2(p) after each CNOT.
    Finally X_ERROR(p) on data and M on all data qubits.

    With detectors: every round, one detector per Z check (its outcome, XORed
    with its previous one after the first round) and, from the second round
    on, one per X check (XOR of consecutive outcomes; the first X outcomes
    are random); after the data measurement, one per Z check comparing the
    parity of its data qubits with its last outcome; observable 0 = the
    parity of a row of data qubits that commutes with every X check.
    Without noise every detector and the observable are 0.

    reset="feedback" replaces the ancilla reset of every round after the
    first by an X controlled by the ancilla's previous outcome (an active
    reset: CX rec[-k] a), so the circuit is dynamic.
    """
    if reset not in ("reset", "feedback"):
        raise ValueError(reset)
    if d < 3 or d % 2 == 0 or rounds < 1:
        raise ValueError("need odd d >= 3 and rounds >= 1")
    checks = _surface_layout(d)
    n_data = d * d
    anc = [n_data + i for i in range(len(checks))]
    x_anc = [anc[i] for i, (t, _) in enumerate(checks) if t == "X"]
    z_anc = [anc[i] for i, (t, _) in enumerate(checks) if t == "Z"]
    data = list(range(n_data))
    n = n_data + len(checks)
    allq = set(range(n))

    layers = []
    for k in range(4):
        pairs = []
        for i, (typ, corners) in enumerate(checks):
            name = _ORDER[typ][k]
            if name not in corners:
                continue
            q = corners[name]
            pairs.append((anc[i], q) if typ == "X" else (q, anc[i]))
        used = [q for pr in pairs for q in pr]
        assert len(used) == len(set(used)), "CNOT layer touches a qubit twice"
        layers.append(pairs)

    c = Circuit(meta={"family": "surface", "d": d, "rounds": rounds, "p": str(p), "reset": reset})
    nc = len(checks)
    for r in range(rounds):
        if reset == "feedback" and r > 0:
            c.feedback("X", [(nc - i, a) for i, a in enumerate(anc)])
        else:
            c.op("R", anc)
        c.op("X_ERROR", anc, p)
        c.op("DEPOLARIZE1", data, p)
        c.tick()
        c.op("H", x_anc)
        c.op("DEPOLARIZE1", x_anc, p)
        c.op("DEPOLARIZE1", sorted(allq - set(x_anc)), p)
        c.tick()
        for pairs in layers:
            flat = [q for pr in pairs for q in pr]
            c.op("CX", flat)
            c.op("DEPOLARIZE2", flat, p)
            c.op("DEPOLARIZE1", sorted(allq - set(flat)), p)
            c.tick()
        c.op("H", x_anc)
        c.op("DEPOLARIZE1", x_anc, p)
        c.op("DEPOLARIZE1", sorted(allq - set(x_anc)), p)
        c.tick()
        c.op("X_ERROR", anc, p)
        c.op("M", anc)
        if detectors:
            for i, (typ, _) in enumerate(checks):
                if r == 0 and typ == "Z":
                    c.detector([nc - i], coords=(i, r))
                elif r > 0:
                    c.detector([nc - i, 2 * nc - i], coords=(i, r))
        c.op("DEPOLARIZE1", data, p)
        c.tick()
    c.op("X_ERROR", data, p)
    c.op("M", data)
    if detectors:
        for i, (typ, corners) in enumerate(checks):
            if typ != "Z":
                continue
            ks = [n_data - q for q in sorted(corners.values())]
            c.detector(ks + [n_data + nc - i], coords=(i, rounds))
        row = _logical_z_support(d, checks)
        c.observable(0, [n_data - q for q in row])
    c.n_qubits = n
    c.meta.update({"n_x_checks": len(x_anc), "n_z_checks": len(z_anc)})
    return c


# --------------------------------------------------------------------------
# Random circuits.
# --------------------------------------------------------------------------

_GATES1 = ("H", "S", "X", "Y", "Z")
_NOISE1 = ("X_ERROR", "Y_ERROR", "Z_ERROR", "DEPOLARIZE1")


def random_clifford_circuit(seed: int, n: int, n_ops: int,
                            p_choices=("0.1", "0.25", "0.5", "0.75", "1"),
                            feedback: bool = False, detectors: bool = False) -> Circuit:
    """Random noisy stabilizer circuit on n qubits (for brute-force checks).
    Mixes every instruction of the format uniformly; with `feedback`, also
    Paulis controlled by earlier records; with `detectors`, ends with a few
    detectors and observables over random records."""
    rng = np.random.default_rng(seed)
    c = Circuit(meta={"family": "random_clifford", "seed": seed, "n": n})
    kinds = ("g1", "cx", "m", "r", "mr", "n1", "n2") + (("fb",) if feedback else ())
    for _ in range(n_ops):
        k = kinds[rng.integers(len(kinds))]
        if k == "g1":
            c.op(_GATES1[rng.integers(len(_GATES1))], [rng.integers(n)])
        elif k == "cx" and n >= 2:
            a, b = rng.choice(n, 2, replace=False)
            c.op("CX", [a, b])
        elif k == "m":
            c.op("M", [rng.integers(n)])
        elif k == "r":
            c.op("R", [rng.integers(n)])
        elif k == "mr":
            c.op("MR", [rng.integers(n)])
        elif k == "n1":
            p = p_choices[rng.integers(len(p_choices))]
            c.op(_NOISE1[rng.integers(len(_NOISE1))], [rng.integers(n)], p)
        elif k == "n2" and n >= 2:
            a, b = rng.choice(n, 2, replace=False)
            p = p_choices[rng.integers(len(p_choices))]
            c.op("DEPOLARIZE2", [a, b], p)
        elif k == "fb" and c.n_meas > 0:
            c.feedback("XYZ"[rng.integers(3)], [(1 + rng.integers(c.n_meas), rng.integers(n))])
    c.op("M", list(range(n)))
    if detectors:
        for _ in range(1 + rng.integers(4)):
            k = 1 + rng.integers(min(4, c.n_meas))
            c.detector(sorted(set(1 + rng.integers(c.n_meas, size=k))))
        for i in range(1 + rng.integers(2)):
            c.observable(i, sorted(set(1 + rng.integers(c.n_meas, size=1 + rng.integers(3)))))
    c.n_qubits = max(c.n_qubits, n)
    return c


def random_layered_circuit(n: int, seed: int, cnot_pairs: int | None = None,
                           p_dep: float | str | None = None,
                           meas_frac: float = 0.05) -> Circuit:
    """Layered random interaction circuit of the paper's evaluation (Fig. 3).

    n qubits, n layers.  Each layer applies H, S or nothing to every qubit
    uniformly at random, then CNOTs on `cnot_pairs` random disjoint pairs
    (5 in Fig. 3a, floor(n/2) in 3b/3c), optionally single-qubit
    depolarizing noise on every qubit (Fig. 3c), then measures a random 5%
    of the qubits.  Finally every qubit is measured.
    """
    rng = np.random.default_rng(seed)
    if cnot_pairs is None:
        cnot_pairs = n // 2
    cnot_pairs = min(cnot_pairs, n // 2)
    c = Circuit(meta={"family": "layered", "n": n, "seed": seed,
                      "cnot_pairs": cnot_pairs, "p_dep": p_dep})
    n_meas = max(1, int(round(meas_frac * n)))
    for _ in range(n):
        choice = rng.integers(3, size=n)
        c.op("H", np.nonzero(choice == 0)[0])
        c.op("S", np.nonzero(choice == 1)[0])
        perm = rng.permutation(n)[: 2 * cnot_pairs]
        c.op("CX", perm)
        if p_dep is not None:
            c.op("DEPOLARIZE1", range(n), p_dep)
        c.op("M", np.sort(rng.choice(n, n_meas, replace=False)))
        c.tick()
    c.op("M", range(n))
    c.n_qubits = n
    return c


# --------------------------------------------------------------------------
# Multi-circuit workloads.
# --------------------------------------------------------------------------

def batched_mix(seed: int = 0, n_circuits: int = 64):
    """Mix of repetition codes d in {3..25 odd} and rotated surface codes
    d in {3..11 odd}, rounds = d, p log-uniform in [1e-4, 1e-2], shots
    log-uniform in [1e4, 1e6].  Circuit i uses family/distance i mod 17 and
    sampling seed i.  Returns a list of dicts (circuit, shots, seed, meta)."""
    rng = np.random.default_rng(seed)
    fams = [("repetition", d) for d in range(3, 26, 2)] + \
           [("surface", d) for d in range(3, 12, 2)]
    out = []
    for i in range(n_circuits):
        fam, d = fams[i % len(fams)]
        u, v = rng.random(), rng.random()
        p = float(f"{10 ** (-4 + 2 * u):.3g}")
        shots = int(round(10 ** (4 + 2 * v)))
        circ = repetition_memory(d, d, p) if fam == "repetition" else surface_memory(d, d, p)
        out.append({"index": i, "family": fam, "d": d, "rounds": d, "p": p,
                    "shots": shots, "seed": i, "circuit": circ})
    return out


def serving_pool(seed: int = 0, n_circuits: int = 16, d: int = 15, rounds: int = 15):
    """Pool of rotated-surface memory circuits, p log-uniform in
    [1e-3, 5e-3]; the first two are exactly 1e-3 and 5e-3."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_circuits):
        if i == 0:
            p = 1e-3
        elif i == 1:
            p = 5e-3
        else:
            p = float(f"{math.exp(rng.uniform(math.log(1e-3), math.log(5e-3))):.3g}")
        out.append({"index": i, "p": p, "circuit": surface_memory(d, rounds, p)})
    return out


def mix_to_json(mix) -> str:
    return json.dumps([{k: v for k, v in m.items() if k != "circuit"} for m in mix])
