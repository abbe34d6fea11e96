"""sp_sample_batch_static (the batched launch whose tables live in the
library's static device scratch, for callers that cannot allocate) against
the existing batched entry point, sp_batch_create + sp_batch_launch with a
caller's work buffer: every job's output equal bit for bit, on two calls in a
row, the second with a smaller input; and the scratch limit reported."""

from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import paper_2311_03906_amd as sp
from paper_2311_03906_amd import _capi
from workloads import repetition_memory, surface_memory

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


_dms = {}


def _dm(text, path="auto", tile_rows=0):
    key = (text, path, tile_rows)
    if key not in _dms:
        _dms[key] = sp.DeviceModel(sp.Model(text), path=path, tile_rows=tile_rows)
    return _dms[key]


def _jobs(specs):
    """Two copies of each job, one output filled with -1 for each path."""
    a, b = [], []
    for text, path, tile_rows, shots, seed, first in specs:
        dm = _dm(text, path, tile_rows)
        words = max(1, (shots + 63) // 64)
        for lst in (a, b):
            out = torch.full((dm.n_meas, words + 1), -1, dtype=torch.int64, device="cuda")
            lst.append(sp.Job(dm, shots, seed=seed, first_shot=first, out=out))
    return a, b


def _same(static_jobs, batch_jobs):
    for x, y in zip(static_jobs, batch_jobs):
        gx, gy = sp.to_numpy_bits(x.out), sp.to_numpy_bits(y.out)
        assert np.array_equal(gx, gy), (x.model.n_meas, x.shots, x.seed)


def test_static_scratch_batch_equals_work_buffer_batch():
    big = [(surface_memory(15, 15, "0.005").text(), "sparse", 0, 1 << 16, 7, 3 << 20),
           (surface_memory(9, 9, "0.003").text(), "sparse", 256, 20_000, 3, 64),    # four row tiles
           (surface_memory(5, 5, "0.001").text(), "dense", 0, 30_001, 2, 5),        # second kernel
           (repetition_memory(5, 5, "0.01").text(), "auto", 0, 1000, 4, 2 ** 32 - 100),
           (surface_memory(3, 3, "0.02").text(), "auto", 0, 0, 5, 0),               # dropped
           (repetition_memory(3, 3, "0.001").text(), "auto", 0, 10_000, 0, 0)]
    small = [(surface_memory(5, 5, "0.002").text(), "sparse", 0, 4_000, 11, 128),
             (repetition_memory(7, 7, "0.02").text(), "auto", 0, 65, 12, 1)]
    for call, (specs, schedule, launch) in enumerate(((big, "persistent", None), (small, "flat", (4, 1)))):
        _say(f"static scratch batch, call {call + 1}: {len(specs)} jobs, {schedule}")
        s_jobs, b_jobs = _jobs(specs)
        sp.sample_batch_static(s_jobs, launch=launch, schedule=schedule)
        b = sp.Batch(b_jobs, launch=launch, schedule=schedule)
        b.launch()
        torch.cuda.synchronize()
        _same(s_jobs, b_jobs)
        for j in s_jobs:   # the zero-shot job wrote nothing; the padding word is untouched
            assert (sp.to_numpy_bits(j.out)[:, -1] == np.uint64(2 ** 64 - 1)).all()


def test_static_scratch_limit():
    """Tables beyond the scratch are refused before any device work: a flat
    schedule's group map of 4 bytes per group outgrows 4 MiB at 2^20 groups."""
    dm = _dm(repetition_memory(3, 3, "0.001").text())
    out = torch.empty((dm.n_meas, 1), dtype=torch.int64, device="cuda")
    shots = 64 * (1 << 21)
    item = (_capi.sp_batch_item * 1)()
    item[0] = _capi.sp_batch_item(dm.handle.value, 0, 0, shots, out.data_ptr(), shots // 64)
    rc = _capi.lib().sp_sample_batch_static(item, 1, None, _capi.SP_SCHED_FLAT,
                                            torch.cuda.current_stream().cuda_stream)
    assert rc == _capi.SP_E_LIMIT
    assert b"scratch" in _capi.lib().sp_last_error()
