"""The sampling server through the C ABI: each request's output is the same
alone and in the mix (tolerance 0: bit-exact), requests that arrive while
others run are admitted as slots and arena space free up, and oversize
requests are refused."""

from __future__ import annotations

import sys
import threading
import time

import numpy as np
import pytest
import torch

import oracle
import paper_2311_03906_amd as sp
from workloads import repetition_memory, surface_memory

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, file=sys.stderr, flush=True)


_pool = {}


def _model(text, path="auto"):
    if (text, path) not in _pool:
        m = sp.Model(text)
        _pool[(text, path)] = (m, sp.DeviceModel(m, path=path))
    return _pool[(text, path)]


def _alone(dm, shots, seed, first):
    out = dm.sample(shots, seed=seed, first_shot=first)
    torch.cuda.synchronize()
    return out[: dm.n_meas]


def test_results_identical_alone_and_in_mix():
    _say("server: alone vs mix")
    pool = [_model(surface_memory(5, 5, p).text()) for p in ("0.001", "0.004")] + \
           [_model(surface_memory(7, 3, "0.002").text()), _model(repetition_memory(9, 9, "0.01").text()),
            _model(surface_memory(3, 3, "0.02").text(), "dense")]
    rng = np.random.default_rng(0)
    srv = sp.Server(arena_bytes=256 << 20, max_active=4, tick_cost=1 << 20)
    reqs = []
    for i in range(40):
        _, dm = pool[i % len(pool)]
        shots = int(10 ** rng.uniform(1, 5.3))
        first = int(rng.integers(0, 1 << 40))
        reqs.append((srv.submit(dm, shots, seed=i, first_shot=first), dm, shots, i, first))
    for t, dm, shots, seed, first in reqs:
        st = srv.wait(t, timeout_ms=60_000)
        assert st["state"] == "done"
        got = srv.output(st).clone()
        srv.release(t)
        assert torch.equal(got, _alone(dm, shots, seed, first)), (seed, shots)
        assert st["t_submit_ns"] <= st["t_admit_ns"] <= st["t_done_ns"]
    stats = srv.stats()
    assert stats["queued"] == 0 and stats["active"] == 0 and stats["arena_in_use"] == 0
    srv.close()


def test_d15_pool_alone_and_in_mix():
    """The serving pool's own circuits (rotated surface code d=15, 15 rounds,
    3,585 rows): five of them, one uploaded as two row tiles, serve 16
    requests of 10^3 to 10^5 shots with a small tick budget, so that the
    larger requests span several ticks while others are admitted.  Each
    output equals the same request sampled alone, word for word, and 16
    shots of each of four requests equal the oracle's."""
    from workloads.circuits import serving_pool
    pool = serving_pool(0)[:5]
    _say("server: d15 pool, 5 models")
    models = []
    for i, c in enumerate(pool):
        m = sp.Model(c["circuit"].text())
        dm = sp.DeviceModel(m, path="sparse", tile_rows=2048 if i == 4 else 0)
        models.append((c, m, dm))
    assert models[4][2].n_tiles == 2 and all(x[2].n_tiles == 1 for x in models[:4])
    rng = np.random.default_rng(3)
    srv = sp.Server(arena_bytes=2 << 30, max_active=6, tick_cost=1 << 22)
    reqs = []
    for i in range(16):
        k = i % len(models)
        shots = 100_000 if i == 0 else int(10 ** rng.uniform(3, 5))
        first = int(rng.integers(0, 1 << 36))
        reqs.append((srv.submit(models[k][2], shots, seed=1000 + i, first_shot=first), k, shots, 1000 + i, first))
    for n, (t, k, shots, seed, first) in enumerate(reqs):
        st = srv.wait(t, timeout_ms=120_000)
        assert st["state"] == "done"
        got = srv.output(st).clone()
        srv.release(t)
        c, m, dm = models[k]
        assert torch.equal(got, _alone(dm, shots, seed, first)), (k, seed, shots)
        if n < 4:
            _say(f"server: d15 request {n} (model {k}, {shots} shots) vs oracle, 16 shots")
            ids = np.concatenate([[0, shots - 1], np.random.default_rng(n).choice(shots, 14, replace=False)])
            want = oracle.Circuit(c["circuit"].text()).sample_shots(seed, first + ids)
            packed = sp.to_numpy_bits(got)
            for j, s in enumerate(ids):
                col = ((packed[:, int(s) // 64] >> np.uint64(int(s) % 64)) & np.uint64(1)).astype(np.uint8)
                assert np.array_equal(col, want[j]), (n, int(s))
    stats = srv.stats()
    # the 10^5-shot request alone needs 1,563 words x 10,502 blocks, four
    # ticks' budget and more
    assert stats["ticks"] >= 4
    assert stats["queued"] == 0 and stats["active"] == 0 and stats["arena_in_use"] == 0
    srv.close()


def test_small_request_against_oracle():
    text = surface_memory(3, 3, "0.03").text()
    _, dm = _model(text)
    srv = sp.Server(arena_bytes=1 << 20, max_active=2)
    t = srv.submit(dm, 1000, seed=5, first_shot=64 * 7 + 3)
    st = srv.wait(t, timeout_ms=30_000)
    got = sp.to_numpy_bits(srv.output(st))
    assert np.array_equal(got, oracle.Circuit(text).sample(seed=5, first_shot=64 * 7 + 3, shots=1000))
    srv.release(t)
    srv.close()


def test_arrivals_while_running_and_backpressure():
    """A small arena (room for about three outputs) and a producer thread
    that keeps submitting while earlier requests run: everything completes,
    the arena never overflows, and later arrivals are admitted as earlier
    ones are released."""
    _say("server: arrivals + back-pressure")
    m, dm = _model(surface_memory(5, 5, "0.002").text())
    one = m.n_meas * ((20_000 + 63) // 64) * 8
    srv = sp.Server(arena_bytes=3 * one + 4096, max_active=8, tick_cost=1 << 18)
    tickets, done = [], []
    stop = threading.Event()

    def consumer():
        while not stop.is_set() or tickets:
            if not tickets:
                time.sleep(0.001)
                continue
            t = tickets.pop(0)
            st = srv.wait(t, timeout_ms=60_000)
            done.append((t, st, srv.output(st).clone()))
            srv.release(t)

    th = threading.Thread(target=consumer)
    th.start()
    for i in range(24):
        tickets.append(srv.submit(dm, 20_000, seed=100 + i))
        s = srv.stats()
        assert s["arena_in_use"] <= s["arena_capacity"]
        time.sleep(0.0005)
    stop.set()
    th.join(timeout=120)
    assert not th.is_alive() and len(done) == 24
    admits = sorted(st["t_admit_ns"] for _, st, _ in done)
    firsts_done = sorted(st["t_done_ns"] for _, st, _ in done)
    assert admits[3] >= firsts_done[0]      # the fourth could only start after one finished and was released
    ref = _alone(dm, 20_000, 100, 0)
    t0, st0, out0 = min(done, key=lambda x: x[0])
    assert torch.equal(out0, ref)
    srv.close()


def test_refuses_requests_that_cannot_fit():
    m, dm = _model(surface_memory(5, 5, "0.001").text())
    srv = sp.Server(arena_bytes=1 << 16, max_active=2)
    with pytest.raises(sp.SymphaseError) as ei:
        srv.submit(dm, 1_000_000)
    assert ei.value.code == sp._capi.SP_E_BUDGET
    t = srv.submit(dm, 0)
    assert srv.wait(t, 1000)["state"] == "done"
    srv.release(t)
    srv.close()


def test_wait_timeout_and_unknown_ticket():
    m, dm = _model(surface_memory(5, 5, "0.001").text())
    srv = sp.Server(arena_bytes=64 << 20, max_active=1, tick_cost=1 << 12)
    t = srv.submit(dm, 2_000_000 // 64 * 64)
    with pytest.raises(sp.SymphaseError):
        srv.release(t)                       # not finished yet
    st = srv.wait(t, timeout_ms=60_000)
    assert st["state"] == "done"
    srv.release(t)
    with pytest.raises(sp.SymphaseError):
        srv.status(t)
    srv.close()


def test_serves_row_tiled_models_in_a_mix():
    """Row-tiled models (surface d=5 in 64-row tiles, the last one partial;
    25,000 rows in automatic 3,840-row tiles) served together with one-tile
    models, with a small tick budget so that requests are split over many
    ticks: every output equals sp_sample's for the request alone, and one
    tiled request equals the oracle's."""
    text = surface_memory(5, 5, "0.004").text()
    m = sp.Model(text)
    tiled = sp.DeviceModel(m, tile_rows=64)
    assert tiled.n_tiles == 3
    big_text = "\n".join(["H 0", "CX 0 1"] + [l for k in range(5000) for l in
                          (["X_ERROR(0.05) 0"] if k % 100 == 0 else []) +
                          ["DEPOLARIZE1(0.002) 1 2 3 4", "CX 1 2", "M 0", "MR 1 2 3 4"]]) + "\n"
    big = sp.DeviceModel(sp.Model(big_text))
    assert big.n_tiles == 7
    _, one = _model(surface_memory(3, 3, "0.01").text())
    srv = sp.Server(arena_bytes=256 << 20, max_active=3, tick_cost=1 << 16)
    reqs = []
    rng = np.random.default_rng(4)
    for i in range(12):
        dm = (tiled, big, one)[i % 3]
        shots = int(rng.integers(1, 40_000))
        first = int(rng.integers(0, 1 << 36))
        _say(f"server tiled mix request {i} tiles={dm.n_tiles} shots={shots}")
        reqs.append((srv.submit(dm, shots, seed=100 + i, first_shot=first), dm, shots, 100 + i, first))
    for t, dm, shots, seed, first in reqs:
        st = srv.wait(t, timeout_ms=60_000)
        assert st["state"] == "done"
        assert st["n_meas"] == dm.n_meas
        got = srv.output(st).clone()
        if dm is tiled and seed == 100:
            want = oracle.Circuit(text).sample(seed=seed, first_shot=first, shots=shots)
            assert np.array_equal(sp.to_numpy_bits(got), want)
        srv.release(t)
        assert torch.equal(got, _alone(dm, shots, seed, first)), (seed, shots, dm.n_tiles)
    assert srv.stats()["ticks"] > 12
    srv.close()
