"""Closed-form output marginals of a noisy stabilizer circuit (test helper).

Every output row is an affine function of the per-location codes (Eq. 4):
out_k = c_k + sum over locations l of <code_l, mask_lk>, where mask_lk holds
the code bits of location l that row k depends on.  The locations' codes
are independent, so by the piling-up lemma

    P(out_k = 1) = (1 - prod_l (1 - 2 q_lk)) / 2, flipped when c_k = 1,

with q_lk the probability that location l's code has odd overlap with
mask_lk.  A row that depends on a random measurement's bit is 1/2.  The
code probabilities come from the oracle's exact thresholds, and (c, masks)
from probing the oracle one code bit at a time, so nothing here uses the
library.
"""

from __future__ import annotations

import re

import numpy as np

import oracle

_PARITY = np.array([bin(v).count("1") & 1 for v in range(16)], dtype=np.int64)
_ONE_BIT = {"X_ERROR": oracle.LOC_X_ERROR, "Y_ERROR": oracle.LOC_Y_ERROR, "Z_ERROR": oracle.LOC_Z_ERROR}


def location_probabilities(text: str) -> list:
    """Per location, in program order: (kind, {code: probability}).  A
    measurement location gets None (its bit is random or unused)."""
    locs = []
    for line in text.splitlines():
        line = line.split("#")[0].strip()
        if not line:
            continue
        m = re.match(r"([A-Z_0-9]+)(?:\(([^)]*)\))?\s*(.*)", line)
        head, arg, rest = m.group(1), m.group(2), m.group(3).split()
        if head in _ONE_BIT or head == "DEPOLARIZE1" or head == "DEPOLARIZE2":
            n_codes = {"DEPOLARIZE1": 3, "DEPOLARIZE2": 15}.get(head, 1)
            T = [0] + oracle.thresholds(arg.strip(), n_codes)
            probs = {k: (T[k] - T[k - 1]) / 2.0 ** 32 for k in range(1, n_codes + 1)}
            kind = _ONE_BIT.get(head, oracle.LOC_DEPOLARIZE1 if head == "DEPOLARIZE1" else oracle.LOC_DEPOLARIZE2)
            n_targets = len(rest) // 2 if head == "DEPOLARIZE2" else len(rest)
            locs += [(kind, probs)] * n_targets
        elif head in ("M", "R", "MR"):
            kind = {"M": oracle.LOC_M, "R": oracle.LOC_R, "MR": oracle.LOC_MR}[head]
            locs += [(kind, None)] * len(rest)
    return locs


def expected_marginals(text: str, outputs: str = "measurements") -> np.ndarray:
    """P(out_k = 1) for every output row, from the oracle and the lemma."""
    oc = oracle.Circuit(text, outputs=outputs)
    locs = location_probabilities(text)
    kinds = oc.location_kinds()
    assert [k for k, _ in locs] == [int(k) for k in kinds], "location order"
    zero = np.zeros(oc.n_locs, dtype=np.uint8)
    out0, was_random = oc.run_codes(zero)
    c = oc.rows_from_outcomes(out0).astype(np.int64)
    half = np.zeros(oc.n_rows, dtype=bool)
    prod = np.ones(oc.n_rows)
    for l, (kind, probs) in enumerate(locs):
        bits = oracle.CODE_BITS[kind]
        mask = np.zeros(oc.n_rows, dtype=np.int64)   # code bits each row depends on
        for b in range(bits):
            codes = zero.copy()
            codes[l] = 1 << b
            col = oc.rows_from_outcomes(oc.run_codes(codes)[0]).astype(np.int64) ^ c
            mask |= col << b
        if probs is None:
            if was_random[l]:
                half |= mask != 0
            continue
        q = np.zeros(oc.n_rows)
        for code, pr in probs.items():
            odd = _PARITY[code & mask].astype(bool)
            q += np.where(odd, pr, 0.0)
        prod *= 1.0 - 2.0 * q
    pi = (1.0 - prod) / 2.0
    p1 = np.where(c == 1, 1.0 - pi, pi)
    return np.where(half, 0.5, p1)


def ones_per_row(packed: np.ndarray, shots: int) -> np.ndarray:
    """Count of 1 bits per row of a packed (rows, words) uint64 array."""
    bits = np.unpackbits(np.ascontiguousarray(packed).view(np.uint8), axis=1, bitorder="little")
    return bits[:, :shots].sum(axis=1)


def check_marginals(counts: np.ndarray, shots: int, p: np.ndarray, sigmas: float = 5.0):
    """Every row's count within `sigmas` binomial standard deviations (rows
    of probability exactly 0 or 1 must be constant)."""
    sd = np.sqrt(shots * p * (1.0 - p))
    dev = np.abs(counts - shots * p)
    bad = np.nonzero(dev > sigmas * sd + 1e-9)[0]
    assert bad.size == 0, [(int(k), int(counts[k]), float(shots * p[k]), float(sd[k])) for k in bad[:5]]
