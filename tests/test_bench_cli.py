"""bench.py's command line on the host: one GPU only, and the traffic record
it reads is well formed (no GPU needed)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_record_names_existing_sources():
    rec = json.load(open(os.path.join(ROOT, "profiles", "aligned_kernel_fp32_droplet_2048x16384.json")))
    for src in rec["kernel_sources"]:
        assert os.path.exists(os.path.join(ROOT, src)), src
    assert os.path.exists(os.path.join(ROOT, "profiles", rec["summary"]))
    assert rec["traffic_bytes_per_launch"] > 0 and len(rec["kernel_sources_sha256"]) == 64
