"""Host-side checks of bench.py: the one-GPU guard and the committed HBM
traffic record it reads."""
from __future__ import annotations

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_traffic_record_is_consistent():
    """The counter record of the dominant pass: its bytes per launch lie
    within a few percent of the algorithmic 16 G bytes per column of the
    recorded batch (the state read once and written once), and the record
    names the sources it was taken with."""
    t = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic.json")))
    assert t["stage"] == "s2_row" and t["column_batch"] > 0
    G = 256 * 256
    n_cols = 2233 / -(-2233 // t["column_batch"])  # mean columns per launch of the S2 sweep
    alg = 16.0 * G * n_cols
    assert abs(t["bytes_per_launch"] / alg - 1.0) < 0.05
    for src in t["sources_sha256"]:
        assert os.path.exists(os.path.join(ROOT, src))
