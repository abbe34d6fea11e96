"""Phase-symbolization sampler for AMD Instinct MI355X.

Thin Python binding over the C ABI (include/symphase.h).  The functions
named like the C entry points forward their arguments; the classes below
only own handles and torch buffers.  All computation happens in the native
library: symbolize on the host, sampling in the HIP kernels.  There is no
fallback: without the built library, importing the binding raises.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _capi
from ._capi import (  # noqa: F401
    EXPORTS,
    SP_PATH_AUTO,
    SP_PATH_DENSE,
    SP_PATH_SPARSE,
    SP_SCHED_FLAT,
    SP_SCHED_PERSISTENT,
    SymphaseError,
    check,
    lib,
    SP_REQ_ACTIVE,
    SP_REQ_DONE,
    SP_REQ_FAILED,
    SP_REQ_QUEUED,
    sp_batch_item,
    sp_dims,
    sp_launch,
    sp_request_status,
    sp_server_config,
    sp_server_counters,
)

_PATHS = {"auto": SP_PATH_AUTO, "sparse": SP_PATH_SPARSE, "dense": SP_PATH_DENSE}


def _release(obj, fn: str, _c=_capi):
    h = getattr(obj, "_h", None)
    L = _c._lib
    if h and L is not None:
        try:
            getattr(L, fn)(h)
        except Exception:
            pass
    obj._h = None


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class Circuit:
    """Parsed circuit (sp_circuit_parse)."""

    def __init__(self, text: str | None = None, _handle=None):
        h = _handle
        if h is None:
            b = text.encode()
            h = ctypes.c_void_p()
            check(lib().sp_circuit_parse(b, len(b), ctypes.byref(h)))
        self._h = h
        v = [ctypes.c_uint32() for _ in range(4)]
        check(lib().sp_circuit_counts(h, *[ctypes.byref(x) for x in v]))
        self.n_qubits, self.n_meas, self.n_detectors, self.n_observables = (x.value for x in v)

    @property
    def handle(self):
        return self._h

    def with_noise(self, p_1q=None, p_2q=None, p_meas=None, p_reset=None, p_idle=None) -> "Circuit":
        """A new circuit with a circuit-level noise model added
        (sp_circuit_add_noise); each probability is a decimal string or None."""
        enc = lambda p: None if p is None else str(p).encode()
        nz = _capi.sp_noise(enc(p_1q), enc(p_2q), enc(p_meas), enc(p_reset), enc(p_idle))
        h = ctypes.c_void_p()
        check(lib().sp_circuit_add_noise(self._h, ctypes.byref(nz), ctypes.byref(h)))
        return Circuit(_handle=h)

    def __del__(self, _rel=_release):
        _rel(self, "sp_circuit_free")


_OUTPUTS = {"measurements": _capi.SP_OUT_MEASUREMENTS, "detectors": _capi.SP_OUT_DETECTORS}
_INIT_MODES = {"auto": _capi.SP_INIT_AUTO, "one_pass": _capi.SP_INIT_ONE_PASS, "two_pass": _capi.SP_INIT_TWO_PASS}


class Model:
    """(M, c) and the location table: Algorithm 1, Initialization.
    outputs="measurements" gives one row per recorded measurement;
    outputs="detectors" one row per detector, then one per observable.
    init="host" runs the pass on the CPU (sp_symbolize_outputs),
    init="device" on the GPU (sp_symbolize_device, up to 1024 qubits) with a
    work buffer from torch on `device`; both give the same model."""

    def __init__(self, circuit: Circuit | str, outputs: str = "measurements", init: str = "host", device=None,
                 stream=None, init_mode: str = "auto"):
        if isinstance(circuit, str):
            circuit = Circuit(circuit)
        if outputs not in _OUTPUTS:
            raise ValueError(f"outputs must be one of {sorted(_OUTPUTS)}")
        if init not in ("host", "device"):
            raise ValueError("init must be 'host' or 'device'")
        self.outputs = outputs
        h = ctypes.c_void_p()
        if init == "host":
            check(lib().sp_symbolize_outputs(circuit.handle, _OUTPUTS[outputs], ctypes.byref(h)))
        else:
            if not torch.cuda.is_available():
                raise SymphaseError(-5, "no GPU: device Initialization runs only on the device")
            device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
            mode = _INIT_MODES[init_mode]
            n = ctypes.c_size_t()
            check(lib().sp_symbolize_device_work_bytes_mode(circuit.handle, mode, ctypes.byref(n)))
            size = n.value
            need = ctypes.c_size_t()
            with torch.cuda.device(device):
                # A too-small buffer fails with the size that suffices for the
                # failed step; the lists' length is known only after the
                # replay, so a second retry may be needed.
                for attempt in range(3):
                    work = torch.empty(size + 256, dtype=torch.uint8, device=device)
                    base = work.data_ptr()
                    off = (-base) % 256
                    rc = lib().sp_symbolize_device_mode(circuit.handle, _OUTPUTS[outputs], mode,
                                                        ctypes.c_void_p(base + off), size,
                                                        ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(h),
                                                        ctypes.byref(need))
                    del work
                    if rc == _capi.SP_OK or need.value <= size or attempt == 2:
                        check(rc)
                        break
                    size = need.value
        self._h = h
        d = sp_dims()
        check(lib().sp_model_dims(h, ctypes.byref(d)))
        self.dims = d
        self.n_meas, self.n_vars, self.n_locs = d.n_meas, d.n_vars, d.n_locs

    @property
    def handle(self):
        return self._h

    def __del__(self, _rel=_release):
        _rel(self, "sp_model_free")

    def expected_work(self) -> tuple:
        """(fired locations, touched sparse entries) per 64-shot word."""
        f, e = ctypes.c_double(), ctypes.c_double()
        check(lib().sp_model_expected_work(self._h, ctypes.byref(f), ctypes.byref(e)))
        return f.value, e.value

    def export_dense(self):
        """(M as a (n_meas, n_vars) uint8 0/1 array, c as a uint8 0/1 vector)."""
        rw = max(1, (self.n_vars + 63) // 64)
        M = np.zeros((max(self.n_meas, 1), rw), dtype=np.uint64)
        c = np.zeros(max(1, (self.n_meas + 63) // 64), dtype=np.uint64)
        check(lib().sp_model_export_dense(self._h, M.ctypes.data, rw, c.ctypes.data))
        bits = np.unpackbits(M.view(np.uint8), axis=1, bitorder="little")[: self.n_meas, : self.n_vars]
        cb = np.unpackbits(c.view(np.uint8), bitorder="little")[: self.n_meas]
        return bits, cb

    def export_csc(self):
        cp = np.zeros(self.n_vars + 1, dtype=np.uint32)
        ri = np.zeros(max(1, self.dims.nnz), dtype=np.uint32)
        check(lib().sp_model_export_csc(self._h, cp.ctypes.data, ri.ctypes.data))
        return cp, ri[: self.dims.nnz]

    def export_vars(self):
        vl = np.zeros(max(1, self.n_vars), dtype=np.uint32)
        vb = np.zeros(max(1, self.n_vars), dtype=np.uint8)
        check(lib().sp_model_export_vars(self._h, vl.ctypes.data, vb.ctypes.data))
        return vl[: self.n_vars], vb[: self.n_vars]

    def sample_host(self, shots: int, seed: int = 0, first_shot: int = 0, ld: int | None = None,
                    n_threads: int = 0) -> np.ndarray:
        """Sampling on the host CPU (sp_sample_host): packed outcomes
        (n_meas, ld) uint64, bit for bit what DeviceModel.sample writes."""
        words = (shots + 63) // 64
        ld = max(words, 1) if ld is None else ld
        out = np.zeros((max(self.n_meas, 1), ld), dtype=np.uint64)
        check(lib().sp_sample_host(self._h, seed, first_shot, shots, out.ctypes.data, ld, n_threads))
        return out[: self.n_meas]

    def device_bytes(self, path: str = "auto", tile_rows: int = 0) -> int:
        n = ctypes.c_size_t()
        check(lib().sp_model_device_bytes_tiled(self._h, _PATHS[path], tile_rows, ctypes.byref(n)))
        return n.value


class DeviceModel:
    """Device-resident model (sp_model_upload) in a torch-owned buffer."""

    def __init__(self, model: Model, path: str = "auto", device=None, stream=None, tile_rows: int = 0):
        """tile_rows: 0 for the library's choice (one tile while the rows fit
        one LDS slab), else row tiles of that many rows."""
        if not torch.cuda.is_available():
            raise SymphaseError(-5, "no GPU: the sampler runs only on the device")
        device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        nbytes = model.device_bytes(path, tile_rows)
        with torch.cuda.device(device):
            self.buffer = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            base = self.buffer.data_ptr()
            off = (-base) % 256
            h = ctypes.c_void_p()
            check(lib().sp_model_upload_tiled(model.handle, _PATHS[path], tile_rows, ctypes.c_void_p(base + off),
                                              nbytes, ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(h)))
        self._h = h
        self.device = device
        self.n_meas = model.n_meas
        self.path = path
        self.expected_work = model.expected_work()
        d = sp_dims()
        check(lib().sp_dmodel_dims(h, ctypes.byref(d)))
        self.dims = d
        nt, rm = ctypes.c_uint32(), ctypes.c_uint32()
        check(lib().sp_dmodel_tiles(h, ctypes.byref(nt), ctypes.byref(rm)))
        self.n_tiles, self.tile_rows_max = nt.value, rm.value

    @property
    def handle(self):
        return self._h

    def __del__(self, _rel=_release):
        _rel(self, "sp_dmodel_free")

    @property
    def launch(self):
        L = sp_launch()
        check(lib().sp_dmodel_get_launch(self._h, ctypes.byref(L)))
        return (L.waves_per_group, L.words_per_group)

    @launch.setter
    def launch(self, value):
        """(waves_per_group, words_per_group), or None for the default."""
        if value is None:
            check(lib().sp_dmodel_set_launch(self._h, None))
        else:
            L = sp_launch(int(value[0]), int(value[1]))
            check(lib().sp_dmodel_set_launch(self._h, ctypes.byref(L)))

    def sample(self, shots: int, seed: int = 0, first_shot: int = 0, out: torch.Tensor | None = None,
               ld: int | None = None, stream=None) -> torch.Tensor:
        """Packed outcomes (n_meas, ld) int64 (bit patterns of uint64 words).
        `out` may be a row-strided view; rows an odd number of 128-byte lines
        apart (ld = words + 16 for 2^20 shots) write each output line once."""
        words = (shots + 63) // 64
        if out is None:
            ld = max(words, 1) if ld is None else ld
            out = torch.empty((max(self.n_meas, 1), ld), dtype=torch.int64, device=self.device)
        else:
            ld = out.stride(0) if ld is None else ld
            if out.dtype != torch.int64 or out.device != self.device or out.stride(1) != 1:
                raise SymphaseError(-1, "out must be a row-contiguous int64 tensor on the model's device")
            if out.numel() and out.shape[0] < self.n_meas:
                raise SymphaseError(-1, "out has fewer rows than measurements")
        with torch.cuda.device(self.device):
            check(lib().sp_sample(self._h, seed, first_shot, shots, ctypes.c_void_p(out.data_ptr()), ld,
                                  ctypes.c_void_p(_stream_handle(stream))))
        return out


class Job:
    """One sampling job of a batch: the arguments of DeviceModel.sample."""

    def __init__(self, model: DeviceModel, shots: int, seed: int = 0, first_shot: int = 0,
                 out: torch.Tensor | None = None):
        self.model, self.shots, self.seed, self.first_shot = model, shots, seed, first_shot
        words = max((shots + 63) // 64, 1)
        if out is None:
            out = torch.empty((max(model.n_meas, 1), words), dtype=torch.int64, device=model.device)
        if out.dtype != torch.int64 or out.stride(1) != 1 or out.shape[0] < model.n_meas or out.shape[1] < (shots + 63) // 64:
            raise SymphaseError(-1, "job output must be a row-contiguous int64 (n_meas, >= words) tensor")
        self.out = out

    def item(self) -> sp_batch_item:
        return sp_batch_item(self.model.handle.value, self.seed, self.first_shot, self.shots,
                             self.out.data_ptr(), self.out.stride(0))


def _items(jobs):
    arr = (sp_batch_item * max(len(jobs), 1))()
    for i, j in enumerate(jobs):
        arr[i] = j.item()
    return arr


class Batch:
    """Many jobs in one persistent launch (sp_batch_create / sp_batch_launch)."""

    def __init__(self, jobs: list, launch=None, schedule: str = "persistent", stream=None):
        self.jobs = list(jobs)
        items = _items(self.jobs)
        L = None if launch is None else ctypes.byref(sp_launch(int(launch[0]), int(launch[1])))
        sched = {"persistent": SP_SCHED_PERSISTENT, "flat": SP_SCHED_FLAT}[schedule]
        self.schedule = schedule
        n = ctypes.c_size_t()
        check(lib().sp_batch_work_bytes(items, len(self.jobs), L, sched, ctypes.byref(n)))
        dev = self.jobs[0].model.device if self.jobs else torch.device("cuda", torch.cuda.current_device())
        self.work = torch.empty(n.value + 256, dtype=torch.uint8, device=dev)
        base = self.work.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            check(lib().sp_batch_create(items, len(self.jobs), L, sched, ctypes.c_void_p(base + off), n.value,
                                        ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(h)))
        self._h = h
        self.device = dev

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        nj, tg, gr, L = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), sp_launch()
        check(lib().sp_batch_info(self._h, ctypes.byref(nj), ctypes.byref(tg), ctypes.byref(gr), ctypes.byref(L)))
        return {"jobs": nj.value, "groups": tg.value, "grid": gr.value,
                "launch": (L.waves_per_group, L.words_per_group)}

    def launch(self, stream=None):
        with torch.cuda.device(self.device):
            check(lib().sp_batch_launch(self._h, ctypes.c_void_p(_stream_handle(stream))))

    def __del__(self, _rel=_release):
        _rel(self, "sp_batch_free")


def sample_batch_static(jobs: list, launch=None, schedule: str = "persistent", stream=None) -> None:
    """sp_sample_batch_static: the jobs' batched launch with the library's
    static device scratch for its tables (no work buffer is allocated)."""
    items = _items(jobs)
    L = None if launch is None else ctypes.byref(sp_launch(int(launch[0]), int(launch[1])))
    sched = {"persistent": SP_SCHED_PERSISTENT, "flat": SP_SCHED_FLAT}[schedule]
    check(lib().sp_sample_batch_static(items, len(jobs), L, sched, ctypes.c_void_p(_stream_handle(stream))))


class Graph:
    """A captured launch sequence (sp_graph_capture_batch / _plain)."""

    def __init__(self, handle, keep):
        self._h, self._keep = handle, keep

    @classmethod
    def capture_batch(cls, batch: Batch) -> "Graph":
        h = ctypes.c_void_p()
        with torch.cuda.device(batch.device):
            check(lib().sp_graph_capture_batch(batch.handle, ctypes.byref(h)))
        return cls(h, batch)

    @classmethod
    def capture_plain(cls, jobs: list) -> "Graph":
        items = _items(jobs)
        h = ctypes.c_void_p()
        check(lib().sp_graph_capture_plain(items, len(jobs), ctypes.byref(h)))
        return cls(h, list(jobs))

    def launch(self, stream=None):
        check(lib().sp_graph_launch(self._h, ctypes.c_void_p(_stream_handle(stream))))

    def __del__(self, _rel=_release):
        _rel(self, "sp_graph_free")


class Server:
    """Continuous-batching sampling server (sp_server_*).  Outputs live in an
    HBM arena of `arena_bytes`; requests are admitted first in first out as
    slots and arena space free up."""

    STATES = {SP_REQ_QUEUED: "queued", SP_REQ_ACTIVE: "active", SP_REQ_DONE: "done", SP_REQ_FAILED: "failed"}

    def __init__(self, arena_bytes: int, max_active: int = 16, max_queued: int = 0, tick_cost: int = 0,
                 launch=(0, 0), device=None):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        cfg = sp_server_config(max_active, max_queued, tick_cost, sp_launch(int(launch[0]), int(launch[1])))
        n = ctypes.c_size_t()
        check(lib().sp_server_work_bytes(ctypes.byref(cfg), ctypes.byref(n)))
        self.arena = torch.empty(arena_bytes + 256, dtype=torch.uint8, device=self.device)
        self.work = torch.empty(n.value + 256, dtype=torch.uint8, device=self.device)
        a0, w0 = self.arena.data_ptr(), self.work.data_ptr()
        self._arena_base = a0 + (-a0) % 256
        w = w0 + (-w0) % 256
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().sp_server_create(ctypes.byref(cfg), ctypes.c_void_p(self._arena_base), arena_bytes,
                                         ctypes.c_void_p(w), n.value, ctypes.byref(h)))
        self._h = h
        self._models = {}

    def submit(self, model: DeviceModel, shots: int, seed: int = 0, first_shot: int = 0) -> int:
        t = ctypes.c_uint64()
        check(lib().sp_server_submit(self._h, model.handle, seed, first_shot, shots, ctypes.byref(t)))
        self._models[t.value] = model
        return t.value

    def _status(self, st: sp_request_status) -> dict:
        return {"state": self.STATES[st.state], "n_meas": st.n_meas, "d_out": st.d_out, "ld": st.ld_words,
                "t_submit_ns": st.t_submit_ns, "t_admit_ns": st.t_admit_ns, "t_done_ns": st.t_done_ns}

    def status(self, ticket: int) -> dict:
        st = sp_request_status()
        check(lib().sp_server_status(self._h, ticket, ctypes.byref(st)))
        return self._status(st)

    def wait(self, ticket: int, timeout_ms: int = -1) -> dict:
        st = sp_request_status()
        check(lib().sp_server_wait(self._h, ticket, timeout_ms, ctypes.byref(st)))
        return self._status(st)

    def output(self, status: dict) -> torch.Tensor:
        """View of a finished request's output in the arena: (n_meas, ld) int64.
        Valid until release."""
        if status["d_out"] is None or status["n_meas"] == 0:
            return torch.empty((0, status["ld"]), dtype=torch.int64, device=self.device)
        off = status["d_out"] - self._arena_base
        nbytes = status["n_meas"] * status["ld"] * 8
        return self.arena[(self._arena_base - self.arena.data_ptr()) + off:][:nbytes].view(torch.int64).view(
            status["n_meas"], status["ld"])

    def release(self, ticket: int):
        check(lib().sp_server_release(self._h, ticket))
        self._models.pop(ticket, None)

    def stats(self) -> dict:
        c = sp_server_counters()
        check(lib().sp_server_stats(self._h, ctypes.byref(c)))
        return {k: getattr(c, k) for k, _ in sp_server_counters._fields_}

    def close(self):
        _release(self, "sp_server_destroy")

    def __del__(self, _rel=_release):
        _rel(self, "sp_server_destroy")


def sample(dmodel: DeviceModel, shots: int, seed: int = 0, first_shot: int = 0, **kw) -> torch.Tensor:
    return dmodel.sample(shots, seed=seed, first_shot=first_shot, **kw)


def to_numpy_bits(packed: torch.Tensor) -> np.ndarray:
    """Packed int64 tensor -> uint64 numpy array."""
    return packed.detach().cpu().numpy().view(np.uint64)
