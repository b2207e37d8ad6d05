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


def test_sample_parity_grades_count_matched_cells():
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    rng = np.random.default_rng(3)
    ns, n = 5, 40
    Y = rng.random((ns, n))
    T = 1000 + rng.random(n)
    acc = rng.integers(1, 9, n).astype(np.int32)
    rej = np.zeros(n, np.int32)
    idx = np.array([1, 4, 7, 30])
    Yo, To = Y[:, idx].copy(), T[idx].copy()
    ao, ro = acc[idx].copy(), rej[idx].copy()
    Yo[2, 1] *= 1 + 3e-10          # graded, above the bar
    Yo[0, 2] *= 1 + 5e-11
    ao[3] += 1                     # a different step sequence: not graded
    Yo[1, 3] *= 1 + 1e-3
    gpu = {"final_state": (Y, T), "cell_counts": (acc, rej)}
    d = bench.sample_parity(gpu, (idx, Yo, To, ao, ro, np.zeros(4, np.int32)), 1e-6, 1e-12)
    assert d["cells"] == 4 and d["count_match_frac"] == 0.75
    assert abs(d["max_rel_err_count_matched"] - 3e-10) < 1e-12
    assert d["cells_above_bar"] == 1
    assert d["max_norm_err_count_mismatched"] > 100
