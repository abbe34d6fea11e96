#!/usr/bin/env python3
"""Throughput of the sampling hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one pass of the whole path -- keyed Philox draws, threshold
select, 64-shot packing, out = M s + c over GF(2), store -- over one batch
of 10^6 shots of the rotated surface-code memory experiment, distance 5,
5 rounds (49 qubits, 145 measurements), circuit-level noise p = 1e-3.  Each
step samples the next 10^6 shots (first_shot advances), with the model
resident in HBM.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "measurement bits sampled/s (shots×meas), batched vs plain; p50/p99 latency"
PEAK_VALU = 256 * 4 * 16 * 2.4e9      # int32 lane-ops/s: CUs x SIMDs x lanes x clock
PHILOX_OPS = 40                         # 20 products 32x32->64 + 20 three-input XORs per block
KERNEL_SRC = os.path.join(ROOT, "paper_2311_03906_amd", "csrc", "sample.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sample_kernel_surface_d5_traffic.json")


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (profiling runs)")
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (counter calibration) and exit")
    return ap.parse_args()


def model_draw_work(m) -> tuple:
    """(Philox blocks per shot, drawn locations per shot): one block per l/4
    holding a drawn location, one threshold compare per drawn location."""
    return int(m.dims.n_draw_blocks), int(m.dims.n_drawn)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def time_steps(fn, steps: int, warmup: int, torch):
    """Runs fn(i) warmup + steps times; returns (wall seconds of the timed
    steps, per-step device milliseconds from events on the current stream)."""
    for i in range(warmup):
        fn(i)
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record()
        fn(warmup + i)
        ends[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, [s.elapsed_time(e) for s, e in zip(starts, ends)]


def pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(math.ceil(q / 100 * len(xs))) - 1)]


def cpu_baseline(text: str, n_meas: int) -> dict:
    import oracle
    oracle.build(force=False)
    c = oracle.Circuit(text)
    cores = os.cpu_count() or 1
    shots = 64 * 2048
    t0 = time.perf_counter()
    c.sample(seed=0, first_shot=0, shots=shots, n_threads=cores)
    dt = time.perf_counter() - t0
    return {"value": shots * n_meas / dt, "unit": "bits/s", "cores": cores, "kind": "oracle",
            "sample": f"{shots} shots of the same circuit (seed 0), concrete A-G tableau per shot, "
                      f"{cores} threads, {dt:.2f} s"}


def main():
    args = parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the sampler shards by shot range with no exchange, "
              "and only the one-GPU path is built and measured (see DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n}))
        return

    import paper_2311_03906_amd as sp
    from workloads import surface_memory, repetition_memory

    shots = 1_000_000
    text = surface_memory(5, 5, "0.001").text()
    model = sp.Model(text)
    dm = sp.DeviceModel(model, path="sparse")
    n_meas = model.n_meas
    n_blocks, n_drawn = model_draw_work(model)
    out = torch.empty((n_meas, (shots + 63) // 64), dtype=torch.int64, device="cuda")

    def step(i):
        dm.sample(shots, seed=0, first_shot=i * shots, out=out)

    wall, lat = time_steps(step, args.steps, args.warmup, torch)
    value = shots * n_meas * args.steps / wall
    avg_ms = sum(lat) / len(lat)
    ops = shots * (PHILOX_OPS * n_blocks + n_drawn)
    achieved = ops / (avg_ms * 1e-3)

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        t = json.load(open(TRAFFIC_FILE))
        if t.get("kernel_sha256_16") == kernel_hash():
            traffic = t.get("hbm_bytes_per_launch")

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "bits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "rotated surface-code memory-Z, d=5, 5 rounds, p=1e-3 circuit-level noise, "
                               "10^6 shots per step", "n_qubits": model.dims.n_qubits, "n_meas": n_meas,
                   "n_vars": model.n_vars, "drawn_locations": n_drawn, "philox_blocks": n_blocks,
                   "shots_per_step": shots, "path": "sparse", "launch": list(dm.launch), "seed": 0},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "mean": avg_ms},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU / 1e12, "unit": "Tops/s",
                     "frac": achieved / PEAK_VALU, "traffic": traffic,
                     "kernel": "sample_kernel<1 or 2 words, sparse>",
                     "ops_per_launch": ops},
    }

    if not args.no_extra:
        rec["extra"] = extra_workloads(sp, torch, surface_memory, repetition_memory)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(text, n_meas)
    print(json.dumps(rec))


def extra_workloads(sp, torch, surface_memory, repetition_memory) -> dict:
    """Other configurations, each timed over a few repetitions."""
    res = {}
    # Distance-3 repetition code, 3 rounds, 10^4 shots (launch-latency bound).
    m = sp.Model(repetition_memory(3, 3, "0.001").text())
    dm = sp.DeviceModel(m)
    out = torch.empty((m.n_meas, 157), dtype=torch.int64, device="cuda")
    wall, lat = time_steps(lambda i: dm.sample(10_000, seed=0, first_shot=i * 10_000, out=out), 200, 10, torch)
    res["repetition_d3_r3_1e4_shots"] = {"bits_per_s": 10_000 * m.n_meas * 200 / wall, "ms_per_call": wall / 200 * 1e3,
                                         "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99)}
    # Distance-15 surface code, 15 rounds, 10^7 shots in 2^20-shot batches.
    for p in ("0.001", "0.005"):
        m = sp.Model(surface_memory(15, 15, p).text())
        dm = sp.DeviceModel(m, path="sparse")
        total, batch = 10_000_000, 1 << 20
        out = torch.empty((m.n_meas, batch // 64), dtype=torch.int64, device="cuda")
        starts = list(range(0, total, batch))

        def one(i):
            f = starts[i % len(starts)]
            dm.sample(min(batch, total - f), seed=0, first_shot=f, out=out)

        one(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(len(starts)):
            one(i)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[f"surface_d15_r15_p{p}_1e7_shots"] = {"bits_per_s": total * m.n_meas / dt, "seconds": dt,
                                                   "batches": len(starts), "launch": list(dm.launch)}
    return res


if __name__ == "__main__":
    main()
