"""bench.py's host-side contract (no GPU): one GPU only, and the kernel-source hash that
gates the stored HBM-traffic measurement."""
import json
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_source_hash_and_traffic_record():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--print-source-hash"],
                       capture_output=True, text=True, timeout=120, check=True)
    h = r.stdout.strip()
    assert re.fullmatch(r"[0-9a-f]{16}", h)
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_k_integrate_53sp_flame.json")))
    assert re.fullmatch(r"[0-9a-f]{16}", rec["source_hash"])
    # the record scales both counters by a plain copy and carries per-launch bytes
    assert abs(rec["hbm_bytes_per_launch"] - rec["fetch_bytes_per_launch"] - rec["write_bytes_per_launch"]) \
        <= 1e-6 * rec["hbm_bytes_per_launch"]
    assert 1.5 < rec["copy_scale_fetch"] < 2.5 and 0.5 < rec["copy_scale_write"] < 1.5
