"""Host-side checks of the benchmark contract (no GPU needed): more than one
GPU is refused with a message before any device work, and the committed
HBM-traffic summary holds, per stage kernel, the scaled bytes per launch
and the VALU instructions per zone that the JSON line reports."""
from __future__ import annotations

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_summary_has_the_reported_fields():
    tr = json.load(open(os.path.join(ROOT, "profiles", "traffic_box256.json")))
    assert len(tr["source_sha256"]) == 64
    assert tr["fetch_factor"] > 0 and tr["write_factor"] > 0
    kernels = [k for k in tr if k.startswith(("k_lagr<", "k_euler<"))]
    assert "k_lagr<float,3,32,8,6>" in kernels
    for k in kernels:
        e = tr[k]
        assert e["bytes"] > 0 and e["fetch_kib"] > 0 and e["write_kib"] > 0
        assert e["valu_lane_instr_per_zone"] > 0 and 0 < e["valu_busy_pct"] <= 100
