"""Brute-force statevector simulator used to pin the oracle (tests only).

Dense 2^n complex amplitudes, qubit q = bit q of the basis index.  Gates
are the textbook matrices of the paper's background section (H, S, CNOT,
the Paulis); a Z measurement computes P(1) from the amplitudes and projects;
"CX/CY/CZ rec[-k] q" applies the Pauli matrix when that recorded outcome was 1.
It has its own reader of the circuit text and its own location numbering
(program order: each 1-qubit channel target, each DEPOLARIZE2 pair, each
M/R/MR target).  It never draws random numbers: per-location codes are
inputs, with the same meaning as the oracle's (see oracle.h).
"""

from __future__ import annotations

import numpy as np

_S2 = 1.0 / np.sqrt(2.0)
MATS = {
    "H": np.array([[_S2, _S2], [_S2, -_S2]], dtype=complex),
    "S": np.array([[1, 0], [0, 1j]], dtype=complex),
    "X": np.array([[0, 1], [1, 0]], dtype=complex),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=complex),
    "Z": np.array([[1, 0], [0, -1]], dtype=complex),
}


def parse(text: str):
    """(name, targets) per instruction; a record target rec[-k] becomes the
    string 'rec', k; detector and observable lines are skipped (they do not
    act on the state)."""
    ops = []
    for line in text.splitlines():
        line = line.split("#")[0].strip()
        if not line:
            continue
        name = line.split("(")[0].split()[0]
        if name in ("DETECTOR", "OBSERVABLE_INCLUDE"):
            continue
        rest = line[len(name):]
        if rest.startswith("("):
            rest = rest[rest.index(")") + 1:]
        tg = []
        for t in rest.split():
            if t.startswith("rec[-"):
                tg.append(("rec", int(t[5:-1])))
            else:
                tg.append(int(t))
        ops.append((name, tg))
    return ops


class State:
    def __init__(self, n: int):
        self.n = n
        self.psi = np.zeros(2 ** n, dtype=complex)
        self.psi[0] = 1.0

    def _view(self, q):
        # axis for qubit q in a (2,)*n reshape with basis index bit q
        return self.psi.reshape([2] * self.n), self.n - 1 - q

    def apply1(self, U, q):
        t, ax = self._view(q)
        t = np.moveaxis(t, ax, 0)
        t = np.tensordot(U, t, axes=([1], [0]))
        self.psi = np.moveaxis(t, 0, ax).reshape(-1)

    def cx(self, c, t):
        idx = np.arange(2 ** self.n)
        sel = ((idx >> c) & 1) == 1
        src = idx ^ (1 << t)
        new = self.psi.copy()
        new[sel] = self.psi[src[sel]]
        self.psi = new

    def prob1(self, q):
        idx = np.arange(2 ** self.n)
        return float(np.sum(np.abs(self.psi[((idx >> q) & 1) == 1]) ** 2))

    def project(self, q, v):
        idx = np.arange(2 ** self.n)
        self.psi[((idx >> q) & 1) != v] = 0
        self.psi /= np.linalg.norm(self.psi)


def run(text: str, n: int, codes, tol: float = 1e-9):
    """Simulate with per-location codes.  Returns (outcomes, was_random),
    where was_random[l] = 1 for measurement locations whose outcome had
    probability 1/2.  Raises if a measurement probability is neither 0, 1/2
    nor 1 (which a stabilizer circuit never produces)."""
    st = State(n)
    outcomes = []
    was_random = []
    l = 0
    for name, tg in parse(text):
        if name in MATS:
            for q in tg:
                st.apply1(MATS[name], q)
        elif name in ("CX", "CNOT", "CY", "CZ"):
            for i in range(0, len(tg), 2):
                if isinstance(tg[i], tuple):   # Pauli on tg[i+1] if record rec[-k] was 1
                    if outcomes[len(outcomes) - tg[i][1]]:
                        st.apply1(MATS[name[1]], tg[i + 1])
                else:
                    st.cx(tg[i], tg[i + 1])
        elif name in ("X_ERROR", "Y_ERROR", "Z_ERROR"):
            P = MATS[name[0]]
            for q in tg:
                if codes[l] & 1:
                    st.apply1(P, q)
                was_random.append(0)
                l += 1
        elif name == "DEPOLARIZE1":
            for q in tg:
                k = int(codes[l])
                if k & 1:
                    st.apply1(MATS["X"], q)
                if k & 2:
                    st.apply1(MATS["Z"], q)
                was_random.append(0)
                l += 1
        elif name == "DEPOLARIZE2":
            for i in range(0, len(tg), 2):
                k = int(codes[l])
                a, b = tg[i], tg[i + 1]
                if k & 1:
                    st.apply1(MATS["X"], a)
                if k & 2:
                    st.apply1(MATS["Z"], a)
                if k & 4:
                    st.apply1(MATS["X"], b)
                if k & 8:
                    st.apply1(MATS["Z"], b)
                was_random.append(0)
                l += 1
        elif name in ("M", "R", "MR"):
            for q in tg:
                p1 = st.prob1(q)
                if p1 < tol:
                    v, rnd = 0, 0
                elif p1 > 1 - tol:
                    v, rnd = 1, 0
                elif abs(p1 - 0.5) < tol:
                    v, rnd = int(codes[l]) & 1, 1
                else:
                    raise AssertionError(f"measurement probability {p1}")
                st.project(q, v)
                if name != "R":
                    outcomes.append(v)
                if name != "M" and v:
                    st.apply1(MATS["X"], q)
                was_random.append(rnd)
                l += 1
        elif name == "TICK":
            pass
        else:
            raise ValueError(name)
    return np.array(outcomes, dtype=np.uint8), np.array(was_random, dtype=np.uint8)
