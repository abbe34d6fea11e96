"""CPU oracle for the sampling path -- TEST INFRASTRUCTURE ONLY.

A plain concrete Aaronson-Gottesman tableau simulation of every shot
(paper Section 2.2, Eq. 1; faults applied by the Pauli-gate rules of Fact 1),
written in C (`oracle.c`) and loaded here through ctypes.  It shares no code
with the sampling library.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import this package.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LOC_X_ERROR, LOC_Y_ERROR, LOC_Z_ERROR, LOC_DEPOLARIZE1, LOC_DEPOLARIZE2, LOC_M, LOC_R, LOC_MR = range(1, 9)
NOISE_KINDS = (LOC_X_ERROR, LOC_Y_ERROR, LOC_Z_ERROR, LOC_DEPOLARIZE1, LOC_DEPOLARIZE2)
MEAS_KINDS = (LOC_M, LOC_R, LOC_MR)
#: number of code bits per location kind
CODE_BITS = {LOC_X_ERROR: 1, LOC_Y_ERROR: 1, LOC_Z_ERROR: 1, LOC_DEPOLARIZE1: 2,
             LOC_DEPOLARIZE2: 4, LOC_M: 1, LOC_R: 1, LOC_MR: 1}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C11, pthreads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-Wall", "-Wextra",
                               "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P, U8P, U32P, U64P, IP = (ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8),
                                  ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64),
                                  ctypes.POINTER(ctypes.c_int))
        L.oracle_parse.argtypes = [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(P)]
        L.oracle_free.argtypes = [P]
        L.oracle_free.restype = None
        L.oracle_dims.argtypes = [P, IP, IP, IP]
        L.oracle_location_kinds.argtypes = [P, IP]
        L.oracle_run_codes.argtypes = [P, U8P, U8P, U8P, ctypes.c_int]
        L.oracle_philox4x32_10.argtypes = [U32P, U32P, U32P]
        L.oracle_philox4x32_10.restype = None
        L.oracle_draw.argtypes = [ctypes.c_uint64] * 3
        L.oracle_draw.restype = ctypes.c_uint32
        L.oracle_thresholds.argtypes = [ctypes.c_char_p, ctypes.c_int, U64P]
        L.oracle_draw_codes.argtypes = [P, ctypes.c_uint64, ctypes.c_uint64, U8P]
        L.oracle_sample.argtypes = [P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, U64P,
                                    ctypes.c_size_t, ctypes.c_int]
        L.oracle_sample_shots.argtypes = [P, ctypes.c_uint64, U64P, ctypes.c_size_t, U8P, ctypes.c_int]
        L.oracle_output_dims.argtypes = [P, IP, IP]
        L.oracle_rows_from_outcomes.argtypes = [P, ctypes.c_int, U8P, U8P]
        L.oracle_sample_outputs.argtypes = [P, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                            U64P, ctypes.c_size_t, ctypes.c_int]
        L.oracle_sample_shots_outputs.argtypes = [P, ctypes.c_int, ctypes.c_uint64, U64P, ctypes.c_size_t, U8P,
                                                  ctypes.c_int]
        L.oracle_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _check(rc: int):
    if rc != 0:
        raise OracleError(lib().oracle_last_error().decode())


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


OUTPUTS = {"measurements": 0, "detectors": 1}


class Circuit:
    """A parsed circuit held by the oracle library.  `outputs` picks the rows
    that sample/sample_shots return: "measurements" (every recorded outcome)
    or "detectors" (every detector, then every observable)."""

    def __init__(self, text: str, outputs: str = "measurements"):
        h = ctypes.c_void_p()
        b = text.encode()
        _check(lib().oracle_parse(b, len(b), ctypes.byref(h)))
        self._h = h
        nq, nl, nm = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().oracle_dims(h, ctypes.byref(nq), ctypes.byref(nl), ctypes.byref(nm)))
        self.n_qubits, self.n_locs, self.n_meas = nq.value, nl.value, nm.value
        nd, no = ctypes.c_int(), ctypes.c_int()
        _check(lib().oracle_output_dims(h, ctypes.byref(nd), ctypes.byref(no)))
        self.n_detectors, self.n_observables = nd.value, no.value
        self._out = OUTPUTS[outputs]
        self.n_rows = self.n_meas if self._out == 0 else self.n_detectors + self.n_observables

    def rows_from_outcomes(self, outcomes) -> np.ndarray:
        """Output rows (per `outputs`) of one shot from its recorded outcomes."""
        oc = np.ascontiguousarray(outcomes, dtype=np.uint8)
        if oc.size == 0:
            oc = np.zeros(1, dtype=np.uint8)
        rows = np.zeros(max(self.n_rows, 1), dtype=np.uint8)
        _check(lib().oracle_rows_from_outcomes(self._h, self._out, _ptr(oc, ctypes.c_uint8),
                                               _ptr(rows, ctypes.c_uint8)))
        return rows[: self.n_rows]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.oracle_free(h)
            self._h = None

    def location_kinds(self) -> np.ndarray:
        k = np.zeros(max(self.n_locs, 1), dtype=np.int32)
        _check(lib().oracle_location_kinds(self._h, _ptr(k, ctypes.c_int)))
        return k[: self.n_locs]

    def run_codes(self, codes, check_invariants: bool = False):
        """One shot with explicit codes; returns (outcomes, was_random)."""
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        assert codes.shape == (self.n_locs,)
        out = np.zeros(max(self.n_meas, 1), dtype=np.uint8)
        wr = np.zeros(max(self.n_locs, 1), dtype=np.uint8)
        c = codes if self.n_locs else np.zeros(1, dtype=np.uint8)
        _check(lib().oracle_run_codes(self._h, _ptr(c, ctypes.c_uint8), _ptr(out, ctypes.c_uint8),
                                      _ptr(wr, ctypes.c_uint8), int(check_invariants)))
        return out[: self.n_meas], wr[: self.n_locs]

    def draw_codes(self, seed: int, shot: int) -> np.ndarray:
        codes = np.zeros(max(self.n_locs, 1), dtype=np.uint8)
        _check(lib().oracle_draw_codes(self._h, seed, shot, _ptr(codes, ctypes.c_uint8)))
        return codes[: self.n_locs]

    def sample(self, seed: int, first_shot: int, shots: int, ld: int | None = None,
               n_threads: int = 0) -> np.ndarray:
        """Packed output rows, shape (n_rows, ld) uint64."""
        words = (shots + 63) // 64
        ld = words if ld is None else ld
        out = np.zeros((max(self.n_rows, 1), max(ld, 1)), dtype=np.uint64)
        _check(lib().oracle_sample_outputs(self._h, self._out, seed, first_shot, shots,
                                           _ptr(out, ctypes.c_uint64), max(ld, 1), n_threads))
        return out[: self.n_rows, :ld]

    def sample_shots(self, seed: int, shot_ids, n_threads: int = 0) -> np.ndarray:
        """Output rows of the listed absolute shots, shape (len(shot_ids), n_rows) uint8."""
        ids = np.ascontiguousarray(shot_ids, dtype=np.uint64)
        out = np.zeros((max(len(ids), 1), max(self.n_rows, 1)), dtype=np.uint8)
        _check(lib().oracle_sample_shots_outputs(self._h, self._out, seed, _ptr(ids, ctypes.c_uint64), len(ids),
                                                 _ptr(out, ctypes.c_uint8), n_threads))
        return out[: len(ids), : self.n_rows]


def philox4x32_10(ctr, key) -> tuple:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(o, ctypes.c_uint32))
    return tuple(int(v) for v in o)


def draw(seed: int, shot: int, loc: int) -> int:
    return int(lib().oracle_draw(seed, shot, loc))


def thresholds(p: str, m: int) -> list:
    T = np.zeros(m, dtype=np.uint64)
    _check(lib().oracle_thresholds(p.encode(), m, _ptr(T, ctypes.c_uint64)))
    return [int(t) for t in T]
