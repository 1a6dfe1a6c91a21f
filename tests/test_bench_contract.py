"""bench.py's command-line contract that needs no GPU: a request for more
than one GPU exits non-zero with a message, and the committed traffic
summary names the sources it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_summary_records_its_sources():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_k_even_k_odd_urban_km_800x800x128.json")))
    for f in rec["sources"]:
        assert os.path.exists(os.path.join(ROOT, "paper_2607_04516_amd", "csrc", f))
    assert len(rec["sources_sha256"]) == 64
    for st in ("f32", "f16s"):
        alg = rec["algorithmic_bytes_per_launch"][st]
        # counted bytes are at least the algorithmic ones and within 25% of them
        for key in ("per_launch_bytes", "per_launch_bytes_request_sizes"):
            assert alg <= rec[key][st] <= 1.25 * alg
