"""Autotuner for the sampling kernels: evaluation path and launch shape.

Times every candidate (waves per group, words per group) on the device for
a model (plain launches) or for a batch, keeps the fastest, and caches the
choice per circuit class in a JSON file so that later models of the same
class start from it.  `tune_path` also searches the evaluation path of
Eq. 4 (sparse column lists or dense column masks), uploading the model in
each form.  A class is (device arch, and log2 buckets of the measurement
count, the Philox blocks per shot, the expected fired locations per 64-shot
word and the average column weight of M): the quantities that set LDS slab
size, draw work and the two paths' evaluate work; shape-only tuning keys
the class by the path as well.  The output never depends on the path or
the launch shape, only the speed does.
"""

from __future__ import annotations

import json
import math
import os

import torch

from . import Batch, DeviceModel, Model, SymphaseError

CANDIDATES = ((4, 1), (8, 1), (16, 1), (4, 2), (8, 2), (16, 2), (4, 4), (8, 4))
DEFAULT_CACHE = os.environ.get("SYMPHASE_TUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "symphase", "autotune.json"))


def _bucket(x: float) -> int:
    return int(math.floor(math.log2(max(x, 1.0))))


def model_class(dm: DeviceModel) -> str:
    arch = torch.cuda.get_device_properties(dm.device).gcnArchName.split(":")[0]
    fired, _ = dm.expected_work
    return (f"{arch}|{dm.path}|m{_bucket(dm.n_meas)}|b{_bucket(dm.dims.n_draw_blocks)}"
            f"|f{_bucket(fired * 16)}")


def _time_ms(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


class Cache:
    def __init__(self, path: str | None = DEFAULT_CACHE):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            try:
                with open(path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}

    def get(self, key):
        return self.data.get(key)

    def put(self, key, **entry):
        self.data[key] = entry
        if self.path:
            os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def _tune_shapes(dm: DeviceModel, shots: int, reps: int, candidates) -> tuple:
    """(fastest launch shape, its ms per plain launch of `shots` shots)."""
    out = torch.empty((max(dm.n_meas, 1), (shots + 63) // 64), dtype=torch.int64, device=dm.device)
    best, best_ms = None, float("inf")
    for shape in candidates:
        try:
            dm.launch = shape
        except SymphaseError:
            continue
        ms = _time_ms(lambda: dm.sample(shots, seed=1, out=out), reps)
        if ms < best_ms:
            best, best_ms = shape, ms
    dm.launch = best
    return best, best_ms


def tune_model(dm: DeviceModel, shots: int | None = None, reps: int = 3, cache: Cache | None = None,
               force: bool = False, candidates=CANDIDATES) -> tuple:
    """Sets and returns the fastest launch shape for plain sp_sample calls
    on this model.  `shots` defaults to enough 64-shot words to fill the
    device several times over."""
    key = model_class(dm)
    if cache is not None and not force:
        hit = cache.get(key)
        if hit is not None:
            try:
                dm.launch = tuple(hit["launch"])
                return tuple(hit["launch"])
            except SymphaseError:
                pass
    if shots is None:
        shots = 64 * 256 * 64
    best, best_ms = _tune_shapes(dm, shots, reps, candidates)
    if cache is not None:
        cache.put(key, launch=list(best), ms=best_ms, note=f"plain, {shots} shots")
    return best


def path_class(model: Model, device=None) -> str:
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    arch = torch.cuda.get_device_properties(dev).gcnArchName.split(":")[0]
    fired, _ = model.expected_work()
    col = model.dims.nnz / max(model.n_vars, 1)
    return (f"{arch}|m{_bucket(model.n_meas)}|b{_bucket(model.dims.n_draw_blocks)}"
            f"|f{_bucket(fired * 16)}|c{_bucket(col * 4)}")


def tune_path(model: Model, shots: int | None = None, reps: int = 3, cache: Cache | None = None,
              force: bool = False, paths=("sparse", "dense"), candidates=CANDIDATES,
              max_dense_bytes: int = 1 << 30, device=None) -> tuple:
    """Uploads `model` in each evaluation path, tunes each one's launch
    shape on plain launches of `shots` shots, and returns (the fastest
    DeviceModel with its shape set, {path: ms}).  A dense form above
    `max_dense_bytes` of device memory is not tried.  The choice is cached
    per path_class."""
    key = path_class(model, device)
    if cache is not None and not force:
        hit = cache.get(key)
        if hit is not None:
            try:
                dm = DeviceModel(model, path=hit["path"], device=device)
                dm.launch = tuple(hit["launch"])
                return dm, dict(hit["ms"])
            except SymphaseError:
                pass
    if shots is None:
        shots = 64 * 256 * 64
    best, times = None, {}
    for path in paths:
        if path == "dense" and model.device_bytes("dense") > max_dense_bytes:
            continue
        dm = DeviceModel(model, path=path, device=device)
        shape, ms = _tune_shapes(dm, shots, reps, candidates)
        times[path] = ms
        if shape is not None and (best is None or ms < best[2]):
            best = (dm, shape, ms)
        else:
            del dm
    if cache is not None:
        cache.put(key, path=best[0].path, launch=list(best[1]), ms=times, note=f"plain, {shots} shots")
    return best[0], times


def tune_batch(jobs: list, reps: int = 3, schedules=("flat", "persistent"), candidates=CANDIDATES,
               cache: Cache | None = None, key: str | None = None) -> tuple:
    """Returns (batch, launch, schedule, ms) of the fastest batched form of
    these jobs."""
    if cache is not None and key is not None:
        hit = cache.get(key)
        if hit is not None:
            b = Batch(jobs, launch=tuple(hit["launch"]), schedule=hit["schedule"])
            return b, tuple(hit["launch"]), hit["schedule"], hit["ms"]
    best = (None, None, None, float("inf"))
    for sched in schedules:
        for shape in candidates:
            try:
                b = Batch(jobs, launch=shape, schedule=sched)
            except SymphaseError:
                continue
            ms = _time_ms(b.launch, reps)
            if ms < best[3]:
                best = (b, shape, sched, ms)
    if cache is not None and key is not None and best[0] is not None:
        cache.put(key, launch=list(best[1]), schedule=best[2], ms=best[3], note="batch")
    return best
