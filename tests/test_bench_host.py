"""Host-side pieces of bench.py (no GPU): the output row stride and the
committed counter profile it reads."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_padded_ld_is_an_odd_number_of_lines():
    for words in list(range(1, 4200)) + [15625, 16384, 1 << 15, 1 << 16]:
        ld = bench.padded_ld(words)
        assert words <= ld < words + 32
        assert ld % 16 == 0 and (ld // 16) % 2 == 1, (words, ld)
    assert bench.padded_ld(16384) == 16400


def test_traffic_profile_fields():
    t = json.load(open(bench.TRAFFIC_FILE))
    assert t["out_ld_words"] == bench.padded_ld(bench.D15_BATCH // 64)
    assert t["hbm_bytes_per_launch"] > t["algorithmic_output_bytes"] > 0
    for v in t["per_rate"].values():
        assert v["fetch_size_kib_per_dispatch"] > 0 and v["write_size_kib_per_dispatch"] > 0


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr) or "1 GPU" in (p.stdout + p.stderr)
