#!/usr/bin/env python3
"""Throughput of the sampling hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

The workload is the rotated surface-code memory experiment at distance 15,
15 rounds (449 qubits, 3,585 measurements, about 10^5 fault variables),
circuit-level noise at p = 1e-3 and at p = 5e-3, 10^7 shots per noise rate
sampled in batches of 2^20 shots (nine full batches and one of 562,816).
A step is one pass of the whole path -- keyed Philox draws, threshold
select, 64-shot packing, out = M s + c over GF(2), store -- over one batch
at both noise rates (two launches, models resident in HBM, outputs into a
resident buffer); step i samples batch i mod 10, so ten steps cover the
10^7 shots of both rates.  Prints one JSON line.
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
PEAK_HBM = 8.0e12                      # bytes/s, MI355X HBM3E
# Per-lane ALU work of one Philox4x32-10 block.  The counter is (l/4, shot
# lo, shot hi, 0) and a wave of 64 shots shares l/4, the key and (almost
# always) the high word, so round 1 and half of rounds 2-4 are wave-uniform
# or independent of the block: what is left for each shot is 15 products
# 32x32->64 and 17 three-input XORs.
WORK_PER_BLOCK = 32
KERNEL_SRC = os.path.join(ROOT, "paper_2311_03906_amd", "csrc", "sample.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sample_kernel_surface_d15_traffic.json")
D15_TOTAL, D15_BATCH = 10_000_000, 1 << 20
D15_PS = ("0.001", "0.005")


def parse_args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU legs (profiling runs)")
    ap.add_argument("--no-extra", action="store_true", help="skip the other workloads")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving sweep")
    ap.add_argument("--legs", default="rep,d5,draw,dense15,outputs,init,fig3,mix,small,serving",
                    help="comma list of the other workloads to run "
                         "(rep, d5, draw, dense15, outputs, init, fig3, mix, small, serving)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (counter calibration) and exit")
    return ap.parse_args()


def work_ops(m, shots: int) -> int:
    """Algorithmic ALU work of sampling `shots` shots of model m: per shot,
    WORK_PER_BLOCK per Philox block and one threshold compare per drawn
    location."""
    return shots * (WORK_PER_BLOCK * int(m.dims.n_draw_blocks) + int(m.dims.n_drawn))


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


def host_threads() -> int:
    """Host threads the CPU legs use: the CPUs this process may run on,
    at most 16 (one GPU's share of a shared host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(text: str, n_meas: int) -> dict:
    """The oracle (a concrete Aaronson-Gottesman tableau run per shot) on a
    fixed 2^12-shot subset of the workload: shots 0..4095 at p = 1e-3."""
    import oracle
    oracle.build(force=False)
    c = oracle.Circuit(text)
    cores = host_threads()
    shots = 1 << 12
    t0 = time.perf_counter()
    c.sample(seed=0, first_shot=0, shots=shots, n_threads=cores)
    dt = time.perf_counter() - t0
    return {"value": shots * n_meas / dt, "unit": "bits/s", "cores": cores, "kind": "oracle",
            "sample": f"subset: shots 0..{shots - 1} (2^12) of the d=15, p=1e-3 circuit, seed 0, concrete "
                      f"A-G tableau per shot, {cores} threads, {dt:.2f} s", "cpu": _cpu_model()}


def cpu_host_sampler(model, n_meas: int) -> dict:
    """The paper's method on the host CPU (sp_sample_host: the same keyed
    draws and the sparse product out = M s + c), one thread and all threads."""
    cores = host_threads()
    res = {"unit": "bits/s", "cpu": _cpu_model()}
    for key, threads, shots in (("one_core", 1, 1 << 14), ("all_cores", cores, 1 << 18)):
        model.sample_host(64, seed=0, first_shot=0, n_threads=threads)   # warm
        t0 = time.perf_counter()
        model.sample_host(shots, seed=0, first_shot=0, n_threads=threads)
        dt = time.perf_counter() - t0
        res[key] = {"value": shots * n_meas / dt, "threads": threads, "shots": shots, "seconds": dt}
    return res


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def padded_ld(words: int) -> int:
    """Row stride (in words) for rows of `words` 64-shot words: an odd number
    of 128-byte lines.  A workgroup writes one word of every row, so with a
    stride of a large power of two (2^20 shots put rows 128 KiB apart) the
    lines it and its neighbours write fall into a few L2 sets, which evict
    them half-written and write each back several times."""
    ld = -(-words // 16) * 16
    return ld + 16 if (ld // 16) % 2 == 0 else ld


def packed_out(torch, n_meas: int, words: int):
    """Measurement-major output of n_meas rows of `words` words, row stride
    padded_ld(words)."""
    return torch.empty((n_meas, padded_ld(words)), dtype=torch.int64, device="cuda")[:, :words]


def traffic_per_launch():
    """Scaled HBM bytes (FETCH_SIZE + WRITE_SIZE) per full-batch launch from
    the committed counter profile, when it was taken of this sample.hip and
    this output row stride."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    t = json.load(open(TRAFFIC_FILE))
    if t.get("kernel_sha256_16") != kernel_hash() or t.get("out_ld_words") != padded_ld(D15_BATCH // 64):
        return None
    return t.get("hbm_bytes_per_launch")


def main():
    args = parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the sampler shards by shot range with no exchange, "
              "and only the one-GPU path is built and measured.", file=sys.stderr)
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

    texts = {p: surface_memory(15, 15, p).text() for p in D15_PS}
    models = {p: sp.Model(texts[p]) for p in D15_PS}
    dms = {p: sp.DeviceModel(models[p], path="sparse") for p in D15_PS}
    n_meas = models[D15_PS[0]].n_meas
    out = packed_out(torch, n_meas, D15_BATCH // 64)
    batches = [(f, min(D15_BATCH, D15_TOTAL - f)) for f in range(0, D15_TOTAL, D15_BATCH)]
    # per-launch events on the stream the kernels run on (torch's current stream)
    launches = []   # (p, shots, start event, end event) of the timed steps
    timing = [False]

    def step(i):
        first, shots = batches[i % len(batches)]
        for p in D15_PS:
            if timing[0]:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                dms[p].sample(shots, seed=0, first_shot=first, out=out)
                b.record()
                launches.append((p, shots, a, b))
            else:
                dms[p].sample(shots, seed=0, first_shot=first, out=out)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    timing[0] = True
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.warmup + i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    bits = sum(shots * n_meas for _, shots, _, _ in launches)
    per_p = {}
    for p in D15_PS:
        ls = [(shots, a.elapsed_time(b)) for q, shots, a, b in launches if q == p]
        ms = [t for _, t in ls]
        ops = sum(work_ops(models[p], shots) for shots, _ in ls)
        full = [t for shots, t in ls if shots == D15_BATCH]
        per_p[p] = {"ms_per_launch_mean": sum(ms) / len(ms), "ms_full_batch_p50": pct(full, 50) if full else None,
                    "ms_full_batch_p99": pct(full, 99) if full else None, "launches": len(ls),
                    "bits_per_s_kernel": sum(s for s, _ in ls) * n_meas / (sum(ms) * 1e-3),
                    "valu_frac": ops / (sum(ms) * 1e-3) / PEAK_VALU, "ops": ops}
    kernel_ms = sum(v["ms_per_launch_mean"] * v["launches"] for v in per_p.values())
    ops_total = sum(v["ops"] for v in per_p.values())
    achieved = ops_total / (kernel_ms * 1e-3)
    m0 = models[D15_PS[0]]
    # HBM bytes per full launch (counter profile) over the full launches' mean duration
    traffic = traffic_per_launch()
    full_ms = sum(v["ms_full_batch_p50"] for v in per_p.values()) / len(per_p)
    hbm_rate = traffic / (full_ms * 1e-3) if traffic else 0.0
    rec = {
        "metric": METRIC,
        "value": bits / wall,
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
        "config": {"workload": "rotated surface-code memory-Z, d=15, 15 rounds, circuit-level noise p=1e-3 and "
                               "p=5e-3, 10^7 shots per rate in 2^20-shot batches; one step = one batch at both rates",
                   "n_qubits": m0.dims.n_qubits, "n_meas": n_meas,
                   "n_vars": {p: models[p].n_vars for p in D15_PS}, "drawn_locations": int(m0.dims.n_drawn),
                   "philox_blocks": int(m0.dims.n_draw_blocks), "shots_per_rate": D15_TOTAL,
                   "batch_shots": D15_BATCH, "out_ld_words": padded_ld(D15_BATCH // 64), "path": "sparse",
                   "launch": list(dms[D15_PS[0]].launch), "seed": 0},
        "latency_ms": {"per_rate": per_p},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU / 1e12, "unit": "Tops/s",
                     "frac": achieved / PEAK_VALU, "traffic": traffic,
                     "hbm_GB_per_s": hbm_rate / 1e9 if traffic else None,
                     "hbm_frac_of_8TB_per_s": hbm_rate / PEAK_HBM if traffic else None,
                     "kernel": "sample_kernel<1, 0>", "ops_per_full_launch": work_ops(m0, D15_BATCH),
                     "work_model": f"{WORK_PER_BLOCK} lane-ops per (shot, Philox block) + 1 per (shot, drawn location)",
                     "kernel_ms_mean": kernel_ms / len(launches),
                     "per_rate": {p: {"frac": v["valu_frac"], "ms_full_batch_p50": v["ms_full_batch_p50"],
                                      "bits_per_s_kernel": v["bits_per_s_kernel"]} for p, v in per_p.items()}},
    }
    step_ms = [sum(a.elapsed_time(b) for _, _, a, b in launches[k:k + len(D15_PS)])
               for k in range(0, len(launches), len(D15_PS))]
    rec["latency_ms"]["step_p50"] = pct(step_ms, 50)
    rec["latency_ms"]["step_p99"] = pct(step_ms, 99)
    del out

    legs = set() if args.no_extra else {x.strip() for x in args.legs.split(",") if x.strip()}
    if args.no_serving:
        legs.discard("serving")
    known = {"rep", "d5", "draw", "dense15", "outputs", "init", "fig3", "mix", "small", "serving"}
    unknown = legs - known
    if unknown:
        print(f"unknown legs: {sorted(unknown)}", file=sys.stderr)
        sys.exit(2)
    if legs:
        rec["extra"] = extra_workloads(sp, torch, surface_memory, repetition_memory, legs, texts)
        if "init" in legs:
            rec["extra"]["initialization_d15"] = init_leg(sp, torch, surface_memory)
        if "fig3" in legs:
            rec["extra"]["paper_fig3_layered_random"] = fig3_leg(sp, torch)
        if "mix" in legs:
            rec["extra"]["batched_mix_64"] = batched_mix_leg(sp, torch)
        if "small" in legs:
            rec["extra"]["batched_small_jobs_256"] = small_jobs_leg(sp, torch, surface_memory, repetition_memory)
        if "serving" in legs:
            rec["extra"]["serving_d15_pool16"] = serving_leg(sp, torch)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(texts["0.001"], n_meas)
        # the paper's method on the host CPU, beside the oracle
        rec["cpu_baseline"]["host_sampler"] = cpu_host_sampler(models["0.001"], n_meas)
    print(json.dumps(rec))


def extra_workloads(sp, torch, surface_memory, repetition_memory, legs, d15_texts) -> dict:
    """Other configurations, each timed over a few repetitions."""
    res = {}
    if "rep" in legs:
        res.update(_repetition_leg(sp, torch, repetition_memory))
    if "d5" in legs:
        res.update(_d5_leg(sp, torch, surface_memory))
    if "draw" in legs:
        res.update(_draw_only_leg(sp, torch, surface_memory))
    if "dense15" in legs:
        res.update(_dense15_leg(sp, torch, d15_texts))
    if "outputs" in legs:
        res.update(_outputs_leg(sp, torch, surface_memory))
    return res


def _repetition_leg(sp, torch, repetition_memory) -> dict:
    """Distance-3 repetition code, 3 rounds, 10^4 shots (launch-latency bound)."""
    res = {}
    m = sp.Model(repetition_memory(3, 3, "0.001").text())
    dm = sp.DeviceModel(m)
    out = torch.empty((m.n_meas, 157), dtype=torch.int64, device="cuda")
    wall, lat = time_steps(lambda i: dm.sample(10_000, seed=0, first_shot=i * 10_000, out=out), 200, 10, torch)
    res["repetition_d3_r3_1e4_shots"] = {"bits_per_s": 10_000 * m.n_meas * 200 / wall, "ms_per_call": wall / 200 * 1e3,
                                         "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99)}
    return res


def _d5_leg(sp, torch, surface_memory) -> dict:
    """Rotated surface code d=5, 5 rounds (49 qubits, 145 measurements),
    p = 1e-3, 10^6 shots per launch, 200 launches advancing first_shot."""
    m = sp.Model(surface_memory(5, 5, "0.001").text())
    dm = sp.DeviceModel(m, path="sparse")
    shots = 1_000_000
    out = torch.empty((m.n_meas, (shots + 63) // 64), dtype=torch.int64, device="cuda")
    wall, lat = time_steps(lambda i: dm.sample(shots, seed=0, first_shot=i * shots, out=out), 200, 10, torch)
    mean = sum(lat) / len(lat)
    return {"surface_d5_r5_p0.001_1e6_shots": {
        "bits_per_s": shots * m.n_meas * 200 / wall, "ms_per_call": wall / 200 * 1e3, "p50_ms": pct(lat, 50),
        "p99_ms": pct(lat, 99), "launch": list(dm.launch),
        "valu_frac": work_ops(m, shots) / (mean * 1e-3) / PEAK_VALU}}


def _d15_run(sp, torch, text, outputs="measurements") -> dict:
    """10^7 shots of one d=15 model in 2^20-shot launches."""
    m = sp.Model(text, outputs=outputs)
    dm = sp.DeviceModel(m, path="sparse")
    total, batch = D15_TOTAL, D15_BATCH
    out = packed_out(torch, m.n_meas, batch // 64)
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
    return {"bits_per_s": total * m.n_meas / dt, "rows": m.n_meas, "seconds": dt, "batches": len(starts),
            "launch": list(dm.launch), "valu_frac": work_ops(m, total) / dt / PEAK_VALU, "nnz": int(m.dims.nnz)}


def _draw_only_leg(sp, torch, surface_memory) -> dict:
    """The draw's own ceiling: the d=15 circuit at p = 1e-9 has the same
    Philox blocks, drawn locations and threshold compares as the headline,
    but next to nothing fires (the random first-round measurements still do),
    so five 2^20-shot launches time the draw and select alone."""
    m = sp.Model(surface_memory(15, 15, "1e-9").text())
    dm = sp.DeviceModel(m, path="sparse")
    out = packed_out(torch, m.n_meas, D15_BATCH // 64)
    lat = _event_ms(lambda: dm.sample(D15_BATCH, seed=0, first_shot=0, out=out), 5, torch)
    ms = pct(lat, 50)
    res = {"surface_d15_r15_p1e-9_draw_only_2^20_shots": {
        "ms_per_launch": ms, "bits_per_s": D15_BATCH * m.n_meas / (ms * 1e-3),
        "valu_frac": work_ops(m, D15_BATCH) / (ms * 1e-3) / PEAK_VALU,
        "philox_blocks": int(m.dims.n_draw_blocks), "drawn_locations": int(m.dims.n_drawn)}}
    del out, dm
    return res


def _dense15_leg(sp, torch, d15_texts) -> dict:
    """The d=15 workload's dense form of M (per fired variable, XOR into
    the rows set in its 3,585-bit column mask): three 2^20-shot launches
    per noise rate.  Its work grows with the rows per fired variable, so it
    is not the algorithmic path at this size; its own figure is the mask
    words it reads per launch."""
    res = {}
    for p, text in d15_texts.items():
        m = sp.Model(text)
        dm = sp.DeviceModel(m, path="dense")
        out = packed_out(torch, m.n_meas, D15_BATCH // 64)
        lat = _event_ms(lambda: dm.sample(D15_BATCH, seed=0, first_shot=0, out=out), 3, torch)
        ms = pct(lat, 50)
        res[f"surface_d15_r15_p{p}_dense_2^20_shots"] = {
            "ms_per_launch": ms, "bits_per_s": D15_BATCH * m.n_meas / (ms * 1e-3),
            "valu_frac_vs_sparse_work": work_ops(m, D15_BATCH) / (ms * 1e-3) / PEAK_VALU,
            "launch": list(dm.launch), "mask_words_per_variable": (m.n_meas + 63) // 64}
        del out, dm
        from paper_2311_03906_amd import autotune
        tuned, times = autotune.tune_path(m, shots=1 << 18, reps=2, cache=None)
        res[f"surface_d15_r15_p{p}_tuned"] = {"path": tuned.path, "launch": list(tuned.launch),
                                              "ms_2^18_shots": times}
        del tuned
    return res


def _outputs_leg(sp, torch, surface_memory) -> dict:
    """The same d=15 workload with detector outputs (each row a detector or
    the observable: sums of measurement rows, so M is sparser), and as a
    dynamic circuit whose ancillas are reset by X controlled by their last
    outcome (measurement outputs)."""
    res = {}
    for p in ("0.001", "0.005"):
        res[f"surface_d15_r15_p{p}_detectors_1e7_shots"] = _d15_run(
            sp, torch, surface_memory(15, 15, p, detectors=True).text(), outputs="detectors")
        res[f"surface_d15_r15_p{p}_feedback_reset_1e7_shots"] = _d15_run(
            sp, torch, surface_memory(15, 15, p, reset="feedback").text())
    return res


def fig3_leg(sp, torch) -> dict:
    """The paper's own benchmark family (Fig. 3): layered random interaction
    circuits, n qubits x n layers; each layer H/S/nothing per qubit, CNOTs
    on 5 (3a) or floor(n/2) (3b, 3c) random disjoint pairs, single-qubit
    depolarizing noise on every qubit (3c, p = 1e-3), then a Z measurement
    of 5% of the qubits; all qubits measured at the end.  Reported:
    Initialization time on the GPU, and on the host where it takes seconds
    (the host pass grows about as n^3.5 on 3b/3c), then GPU time to generate
    10^4 samples (the paper's sampling metric) and 10^6 samples; circuits
    of more than 9,216 rows are sampled in row tiles.  n = 1000 is the
    paper's largest size (3c: 2,000,000 fault variables)."""
    from workloads import random_layered_circuit
    res = {}
    sizes = [(100, ("3a", "3b", "3c")), (200, ("3a", "3b", "3c")), (400, ("3a", "3b", "3c")),
             (700, ("3a", "3b", "3c")), (1000, ("3a", "3b", "3c"))]
    for n, figs in sizes:
        for fig in figs:
            res[f"fig{fig}_n{n}"] = _fig3_case(sp, torch, random_layered_circuit, fig, n)
    return res


_FIG3_KW = {"3a": {"cnot_pairs": 5}, "3b": {}, "3c": {"p_dep": "0.001"}}
# host Initialization is timed where it takes seconds
_FIG3_HOST_MAX_N = {"3a": 1000, "3b": 400, "3c": 200}


def _fig3_case(sp, torch, random_layered_circuit, fig, n) -> dict:
    print(f"fig{fig} n={n}", file=sys.stderr, flush=True)
    circ = sp.Circuit(random_layered_circuit(n, seed=0, **_FIG3_KW[fig]).text())
    t_host = None
    if n <= _FIG3_HOST_MAX_N[fig]:
        t0 = time.perf_counter()
        sp.Model(circ)
        t_host = time.perf_counter() - t0
    t_dev = _device_init_s(sp, torch, circ, "measurements", reps=3 if n <= 200 else 1, warm=n <= 200)
    m = sp.Model(circ, init="device")
    dm = sp.DeviceModel(m)
    r = {"n_meas": m.n_meas, "n_vars": m.n_vars, "nnz": int(m.dims.nnz), "drawn": int(m.dims.n_drawn),
         "path": dm.path, "row_tiles": dm.n_tiles, "init_s": t_host, "init_device_s": t_dev}
    for shots in (10_000, 1_000_000):
        out = torch.empty((m.n_meas, (shots + 63) // 64), dtype=torch.int64, device="cuda")
        lat = _event_ms(lambda: dm.sample(shots, seed=0, out=out), 10 if n <= 400 else 3, torch)
        ms = pct(lat, 50)
        r[f"ms_{shots}"] = ms
        r[f"bits_per_s_{shots}"] = shots * m.n_meas / (ms * 1e-3)
        del out
    return r


def _device_init_s(sp, torch, circ, outputs, reps=3, warm=True) -> float:
    """Median wall time of Initialization on the GPU (sp_symbolize_device,
    synchronous: instruction upload, kernel, copy-back, host assembly)."""
    if warm:
        sp.Model(circ, outputs=outputs, init="device")
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sp.Model(circ, outputs=outputs, init="device")
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2]


def init_leg(sp, torch, surface_memory) -> dict:
    """Initialization (the symbolic-phase tableau pass) of the d=15 surface
    code, 15 rounds (449 qubits, about 10^5 fault variables), on the host
    and on the GPU; the model is the same bit for bit."""
    res = {}
    for p, outputs in (("0.001", "measurements"), ("0.005", "detectors")):
        circ = sp.Circuit(surface_memory(15, 15, p, detectors=outputs == "detectors").text())
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            m = sp.Model(circ, outputs=outputs)
            ts.append(time.perf_counter() - t0)
        host = sorted(ts)[1]
        dev = _device_init_s(sp, torch, circ, outputs)
        res[f"surface_d15_r15_p{p}_{outputs}"] = {"n_vars": m.n_vars, "nnz": int(m.dims.nnz), "host_s": host,
                                                  "device_s": dev, "speedup": host / dev}
    return res


def _event_ms(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    lat = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        lat.append(a.elapsed_time(b))
    return lat


def _plain_vs_batched(sp, torch, jobs, reps=10) -> dict:
    """Times the same jobs as one sp_sample launch each (plain), the plain
    sequence replayed from a graph, the batched launch (autotuned shape and
    schedule) and its graph replay."""
    from paper_2311_03906_amd import autotune
    bits = sum(j.shots * j.model.n_meas for j in jobs)
    ops = sum(j.shots * (WORK_PER_BLOCK * j.model.dims.n_draw_blocks + j.model.dims.n_drawn) for j in jobs)

    def plain():
        for j in jobs:
            j.model.sample(j.shots, seed=j.seed, first_shot=j.first_shot, out=j.out)

    res = {"jobs": len(jobs), "bits": bits}
    lat = _event_ms(plain, reps, torch)
    res["plain"] = {"ms_p50": pct(lat, 50), "ms_p99": pct(lat, 99)}
    g = sp.Graph.capture_plain(jobs)
    lat = _event_ms(g.launch, reps, torch)
    res["plain_graph"] = {"ms_p50": pct(lat, 50), "ms_p99": pct(lat, 99)}
    b, shape, sched, _ = autotune.tune_batch(jobs, reps=3)
    lat = _event_ms(b.launch, reps, torch)
    res["batched"] = {"ms_p50": pct(lat, 50), "ms_p99": pct(lat, 99), "launch": list(shape), "schedule": sched}
    gb = sp.Graph.capture_batch(b)
    lat = _event_ms(gb.launch, reps, torch)
    res["batched_graph"] = {"ms_p50": pct(lat, 50), "ms_p99": pct(lat, 99)}
    for k in ("plain", "plain_graph", "batched", "batched_graph"):
        ms = res[k]["ms_p50"]
        res[k]["bits_per_s"] = bits / (ms * 1e-3)
        res[k]["valu_frac"] = ops / (ms * 1e-3) / PEAK_VALU
    res["gain_batched_over_plain"] = res["plain"]["ms_p50"] / res["batched"]["ms_p50"]
    res["gain_batched_graph_over_plain"] = res["plain"]["ms_p50"] / res["batched_graph"]["ms_p50"]
    return res


def batched_mix_leg(sp, torch) -> dict:
    """64 circuits: repetition d 3..25 and rotated surface d 3..11 (odd),
    rounds = d, p log-uniform in [1e-4, 1e-2], shots log-uniform in
    [1e4, 1e6], sampling seed = circuit index (the mix is seeded, seed 0).
    Each model's evaluation path and launch shape come from the autotuner
    (tune_path: both paths timed on 2^18 shots, cached per circuit class)."""
    from paper_2311_03906_amd import autotune
    from workloads.circuits import batched_mix
    jobs, models, classes = [], {}, {}
    cache = autotune.Cache(path=None)
    t0 = time.perf_counter()
    for m in batched_mix(0):
        text = m["circuit"].text()
        if text not in models:
            mod = sp.Model(text)
            dm, times = autotune.tune_path(mod, shots=1 << 18, reps=2, cache=cache)
            models[text] = dm
            classes[autotune.path_class(mod)] = {"path": dm.path, "launch": list(dm.launch),
                                                 "ms_2^18_shots": times}
        jobs.append(sp.Job(models[text], m["shots"], seed=m["seed"]))
    res = _plain_vs_batched(sp, torch, jobs)
    res["tuning_s"] = time.perf_counter() - t0
    res["paths"] = {p: sum(1 for j in jobs if j.model.path == p) for p in ("sparse", "dense")}
    res["tuned_classes"] = len(classes)
    res["dense_classes"] = sorted(c for c, v in classes.items() if v["path"] == "dense")
    return res


def small_jobs_leg(sp, torch, surface_memory, repetition_memory) -> dict:
    """256 small jobs (repetition d 3/5/7/9 and surface d 3, d rounds,
    p = 1e-3, 10^4 shots each): the plain path is launch-bound here."""
    texts = [repetition_memory(d, d, "0.001").text() for d in (3, 5, 7, 9)] + [surface_memory(3, 3, "0.001").text()]
    dms = [sp.DeviceModel(sp.Model(t)) for t in texts]
    jobs = [sp.Job(dms[i % len(dms)], 10_000, seed=i) for i in range(256)]
    return _plain_vs_batched(sp, torch, jobs)


def serving_leg(sp, torch) -> dict:
    """Serving over a resident pool of 16 rotated-surface d=15, 15-round
    circuits (p log-uniform in [1e-3, 5e-3], the first two 1e-3 and 5e-3):
    Poisson arrivals, circuit uniform over the pool, shots log-uniform in
    [1e3, 1e6], seed = request id, outputs in a 16 GiB HBM arena.  The
    saturation rate is measured with a burst of 1,024 requests; the
    open-loop sweep runs at 0.25 .. 1.2 of it, per rate two seeds of at
    least 2,000 requests and 10 s of offered load each, reported over the
    middle 80% of completions (sustained bits/s, p50, p99) with the spread
    over the seeds."""
    from paper_2311_03906_amd import loadgen
    from workloads.circuits import serving_pool
    pool = serving_pool(0)
    models = [sp.DeviceModel(sp.Model(c["circuit"].text()), path="sparse") for c in pool]
    srv = sp.Server(arena_bytes=16 << 30, max_active=16)
    mean_bits = (1e6 - 1e3) / math.log(1e3) * models[0].n_meas
    burst = loadgen.poisson_plan(1024, 1e9, len(models), 1_000, 1_000_000, seed=1)
    sat = loadgen.run(srv, models, burst, first_id=1_000_000)
    cap = sat["steady"]["bits_per_s"]
    mu = cap / mean_bits
    out = {"saturation": {"bits_per_s": cap, "requests_per_s": mu, "requests": sat["requests"],
                          "p50_ms": sat["steady"]["p50_ms"], "p99_ms": sat["steady"]["p99_ms"]},
           "arena_bytes": 16 << 30, "max_active": 16, "sweep": []}
    for k, f in enumerate((0.25, 0.5, 0.75, 0.9, 1.0, 1.2)):
        n = int(max(2000, 10.0 * f * mu))
        runs = []
        for seed in (100 + k, 200 + k):
            print(f"serving steady f={f} seed={seed} n={n}", file=sys.stderr, flush=True)
            r = loadgen.run(srv, models, loadgen.poisson_plan(n, f * mu, len(models), 1_000, 1_000_000, seed=seed),
                            first_id=seed * 100_000)
            runs.append({"seed": seed, "requests": r["requests"], "offered_s": n / (f * mu), **r["steady"]})
        row = {"rate_factor": f, "offered_requests_per_s": f * mu, "offered_bits_per_s": f * cap, "runs": runs}
        for key in ("bits_per_s", "p50_ms", "p99_ms"):
            v = [x[key] for x in runs]
            row[key] = sum(v) / len(v)
            row[key + "_spread"] = max(v) - min(v)
        out["sweep"].append(row)
    srv.close()
    return out


if __name__ == "__main__":
    main()
