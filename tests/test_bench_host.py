"""Host-side parts of bench.py (no GPU): the line-granular traffic figure of
the split, the source digest that keys the committed counter summaries, and
the one-GPU guard."""
import json
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_las_touched_bytes_by_hand():
    # rows 0, 11, 63 of 64: means / log-scales (12 B rows) touch lines 0, 1, 5
    # (read and written back), quats (16 B) lines 0, 1, 7 (read), opacity
    # (4 B) lines 0, 1 (read and written back); mask 64 B; children 3 x 48 B
    m = np.zeros(64, np.uint8)
    m[[0, 11, 63]] = 1
    assert bench.las_touched_bytes(m, 3) == 64 + 2 * 384 + 2 * 384 + 384 + 2 * 256 + 3 * 48
    # row 10 of 16: its 12-byte rows straddle lines 0 and 1 (bytes 120..131)
    m = np.zeros(16, np.uint8)
    m[10] = 1
    assert bench.las_touched_bytes(m, 1) == 16 + 2 * 256 + 2 * 256 + 128 + 2 * 128 + 48
    # nothing selected: the mask alone
    assert bench.las_touched_bytes(np.zeros(1000, np.uint8), 0) == 1000


def test_source_digest_and_profile_keys():
    d = bench.kernel_source_digest()
    assert len(d) == 64 and int(d, 16) >= 0
    # a summary taken on another tile shape is not used
    assert bench.profile_facts("edge_fused", "bf16", "no such workload", 128, 4) == {}
    assert bench.cpu_model()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True, text=True)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["n_gpus"] == 2 and "one GPU" in out["error"]
