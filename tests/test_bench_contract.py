"""Host-side checks of bench.py's contract (no GPU): the multi-GPU refusal and
the HBM-traffic record that the roofline object reports."""
import hashlib
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_matches_the_m2l_source():
    """profiles/m2l_fp32_sphere5k_traffic.json names the SHA-256 of the M2L kernel
    text it was measured on; bench.py reports its bytes only while they match."""
    rec = json.load(open(os.path.join(ROOT, "profiles", "m2l_fp32_sphere5k_traffic.json")))
    src = bench.m2l_kernel_source()
    assert b"m2l_mfma_kernel" in src and b"m2l_direct_kernel" in src
    if rec["m2l_kernel_source_sha256"] == hashlib.sha256(src).hexdigest():
        assert bench.measured_traffic(1) == rec["hbm_bytes_per_launch"]
        parts = rec["hbm_bytes_read_per_launch"] + rec["hbm_bytes_written_per_launch"]
        assert abs(rec["hbm_bytes_per_launch"] - parts) <= 2  # rounded separately
    else:
        assert bench.measured_traffic(1) is None
    assert bench.measured_traffic(0) is None  # FP64 products: no counter record
