"""Batched (persistent, multi-circuit) sampling and captured graphs, through
the C ABI.  Every job of a batch must equal the oracle (small jobs) and the
plain one-launch-per-job path, bit for bit; replays must keep doing so."""

from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2311_03906_amd as sp
from workloads import repetition_memory, surface_memory
from workloads.circuits import batched_mix

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


_models = {}


def _dm(text, path="auto"):
    if (text, path) not in _models:
        m = sp.Model(text)
        _models[(text, path)] = (m, sp.DeviceModel(m, path=path), oracle.Circuit(text))
    return _models[(text, path)]


def _small_jobs(dense_too=True):
    specs = [(repetition_memory(3, 3, "0.01"), 1000, 1, 0), (surface_memory(3, 3, "0.02"), 777, 2, 64),
             (repetition_memory(5, 5, "0.005"), 64, 3, 5), (surface_memory(5, 2, "0.01"), 2049, 4, 2 ** 32 - 100),
             (repetition_memory(7, 2, "0.03"), 1, 5, 9), (surface_memory(3, 2, "0.05"), 0, 6, 0),
             (surface_memory(5, 2, "0.01"), 4000, 4, 77)]
    jobs = []
    for circ, shots, seed, first in specs:
        m, dm, oc = _dm(circ.text())
        out = torch.full((m.n_meas, max(1, (shots + 63) // 64) + 1), -1, dtype=torch.int64, device="cuda")
        jobs.append((sp.Job(dm, shots, seed=seed, first_shot=first, out=out), oc))
    if dense_too:   # a dense-path model puts a second kernel in the batch
        m, dm, oc = _dm(surface_memory(3, 3, "0.03").text(), "dense")
        out = torch.full((m.n_meas, 17), -1, dtype=torch.int64, device="cuda")
        jobs.append((sp.Job(dm, 1000, seed=8, first_shot=3, out=out), oc))
    return jobs


def _check_against_oracle(jobs):
    for job, oc in jobs:
        if job.shots == 0:
            assert (job.out == -1).all()
            continue
        words = (job.shots + 63) // 64
        got = sp.to_numpy_bits(job.out)[: job.model.n_meas, :words]
        want = oc.sample(seed=job.seed, first_shot=job.first_shot, shots=job.shots)
        assert np.array_equal(got, want), (job.shots, job.seed)
        assert (sp.to_numpy_bits(job.out)[:, words] == np.uint64(2 ** 64 - 1)).all()   # padding untouched


@pytest.mark.parametrize("schedule", ["persistent", "flat"])
@pytest.mark.parametrize("launch", [None, (4, 1), (8, 2), (16, 4), (2, 1)])
def test_batch_matches_oracle(launch, schedule):
    _say(f"batch small jobs launch={launch} schedule={schedule}")
    jobs = _small_jobs()
    b = sp.Batch([j for j, _ in jobs], launch=launch, schedule=schedule)
    info = b.info()
    assert info["jobs"] == len(jobs) - 1   # the zero-shot job is dropped
    b.launch()
    torch.cuda.synchronize()
    _check_against_oracle(jobs)


@pytest.mark.parametrize("schedule", ["persistent", "flat"])
def test_batch_relaunch_and_graph_replay(schedule):
    """The persistent kernel resets its own counters: repeated launches and
    graph replays, with other device work and synchronisations in between,
    all reproduce the eager result."""
    _say(f"batch relaunch + graph replay schedule={schedule}")
    jobs = _small_jobs()
    b = sp.Batch([j for j, _ in jobs], schedule=schedule)
    b.launch()
    torch.cuda.synchronize()
    ref = [j.out.clone() for j, _ in jobs]
    g = sp.Graph.capture_batch(b)
    other_m, other, _ = _dm(surface_memory(5, 3, "0.003").text())
    for rep in range(4):
        for j, _ in jobs:
            j.out.fill_(-1)
        other.sample(10_000, seed=rep)          # unrelated eager work on the same stream
        if rep % 2:
            torch.cuda.synchronize()
        if rep == 0:
            b.launch()
        else:
            g.launch()
        torch.cuda.synchronize()
        for (j, _), r in zip(jobs, ref):
            assert torch.equal(j.out, r), rep
    _check_against_oracle(jobs)


def test_plain_graph_replay():
    _say("plain graph replay")
    jobs = _small_jobs()
    g = sp.Graph.capture_plain([j for j, _ in jobs])
    for rep in range(3):
        for j, _ in jobs:
            j.out.fill_(-1)
        g.launch()
        torch.cuda.synchronize()
        _check_against_oracle(jobs)


@pytest.mark.parametrize("schedule", ["persistent", "flat"])
def test_mixed_batch_equals_plain_launches(schedule):
    """The 64-circuit mix (repetition d 3..25, surface d 3..11, rounds = d,
    p log-uniform in [1e-4, 1e-2], shots log-uniform in [1e4, 1e6]): each
    job of one batched launch equals its own sp_sample launch, and sampled
    shots of a few jobs equal the oracle."""
    _say(f"64-circuit mix batch vs plain schedule={schedule}")
    mix = batched_mix(0)
    jobs, plain_out = [], []
    for m in mix:
        text = m["circuit"].text()
        mod, dm, oc = _dm(text)
        jobs.append(sp.Job(dm, m["shots"], seed=m["seed"]))
        plain_out.append(dm.sample(m["shots"], seed=m["seed"]))
    b = sp.Batch(jobs, schedule=schedule)
    b.launch()
    torch.cuda.synchronize()
    for j, p in zip(jobs, plain_out):
        assert torch.equal(j.out[: j.model.n_meas], p[: j.model.n_meas])
    rng = np.random.default_rng(3)
    for idx in (0, 5, 13, 16, 33, 63):
        m = mix[idx]
        job = jobs[idx]
        oc = _dm(m["circuit"].text())[2]
        shots = rng.choice(m["shots"], 16, replace=False)
        want = oc.sample_shots(m["seed"], shots)
        got = sp.to_numpy_bits(job.out)[: job.model.n_meas]
        for i, s in enumerate(shots):
            col = ((got[:, s // 64] >> np.uint64(s % 64)) & np.uint64(1)).astype(np.uint8)
            assert np.array_equal(col, want[i]), (idx, int(s))


def test_batch_rejects_bad_items():
    m, dm, _ = _dm(repetition_memory(3, 3, "0.01").text())
    out = torch.zeros((m.n_meas, 1), dtype=torch.int64, device="cuda")
    with pytest.raises(sp.SymphaseError):
        sp.Batch([sp.Job(dm, 64, out=out)], launch=(8, 3))
    job = sp.Job(dm, 64, out=out)
    job.shots = 200                      # ld 1 < 4 words
    with pytest.raises(sp.SymphaseError):
        sp.Batch([job])


@pytest.mark.parametrize("schedule", ["persistent", "flat"])
def test_empty_batch(schedule):
    b = sp.Batch([], schedule=schedule)
    b.launch()
    torch.cuda.synchronize()
    assert b.info()["groups"] == 0


@pytest.mark.parametrize("schedule", ["persistent", "flat"])
def test_batch_with_row_tiled_models(schedule):
    """A model stored as row tiles becomes one job per tile inside a batch;
    with untiled jobs beside it, every job equals the oracle."""
    _say(f"batch with row-tiled models schedule={schedule}")
    jobs = _small_jobs(dense_too=False)
    for circ, tile_rows, path, shots, seed in [(surface_memory(5, 5, "0.005"), 64, "sparse", 3000, 11),
                                               (surface_memory(3, 3, "0.03"), 64, "dense", 700, 12)]:
        text = circ.text()
        m = sp.Model(text)
        dm = sp.DeviceModel(m, path=path, tile_rows=tile_rows)
        assert dm.n_tiles > 1 or m.n_meas <= tile_rows
        out = torch.full((m.n_meas, (shots + 63) // 64 + 1), -1, dtype=torch.int64, device="cuda")
        jobs.append((sp.Job(dm, shots, seed=seed, first_shot=128, out=out), oracle.Circuit(text)))
    b = sp.Batch([j for j, _ in jobs], schedule=schedule)
    b.launch()
    torch.cuda.synchronize()
    _check_against_oracle(jobs)


def test_autotuner_path_search_and_cache():
    """tune_path times both evaluation paths, keeps the faster, caches the
    choice per circuit class; the tuned model samples exactly the oracle's
    bits, and a cache hit rebuilds the same path and launch shape."""
    from paper_2311_03906_amd import autotune
    text = surface_memory(5, 5, "0.003").text()
    _say("autotune path search")
    m = sp.Model(text)
    cache = autotune.Cache(path=None)
    dm, times = autotune.tune_path(m, shots=64 * 512, reps=1, cache=cache,
                                   candidates=((4, 1), (8, 1), (8, 2)))
    assert set(times) == {"sparse", "dense"} and dm.path == min(times, key=times.get)
    got = sp.to_numpy_bits(dm.sample(5000, seed=3, first_shot=64))[: m.n_meas]
    torch.cuda.synchronize()
    want = oracle.Circuit(text).sample(seed=3, first_shot=64, shots=5000)
    assert np.array_equal(got, want)
    hit = cache.get(autotune.path_class(m))
    assert hit["path"] == dm.path and tuple(hit["launch"]) == dm.launch
    dm2, times2 = autotune.tune_path(m, cache=cache)
    assert dm2.path == dm.path and dm2.launch == dm.launch and times2 == times
