"""Readers for the text fixtures under tests/golden/."""

import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def sections(name: str) -> dict:
    out, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            s = line.rstrip("\n")
            if s.startswith("#") or not s.strip():
                continue
            if s.startswith("[") and s.endswith("]"):
                cur = s[1:-1]
                out[cur] = []
            else:
                out[cur].append(s)
    return out


def example(name: str):
    """(circuit_text, {symbol: (loc, bit)}, [set of symbols per outcome])."""
    sec = sections(name)
    text = "\n".join(sec["circuit"]) + "\n"
    symbols = {}
    for s in sec["symbols"]:
        nm, loc, bit = s.split()
        symbols[nm] = (int(loc), int(bit))
    outcomes = []
    for s in sec["outcomes"]:
        rhs = s.split("=")[1]
        outcomes.append(frozenset(t.strip() for t in rhs.split("+")))
    return text, symbols, outcomes


def rows(name: str):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            s = line.split("#")[0].strip()
            if s:
                yield s.split()
