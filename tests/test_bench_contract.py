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


def oracle_dense(R, lev, o, gap):
    """A near-future block is a dense product when the oracle's interpolated operator (eq.
    Uabmn) is neither zero at every node pair (wavefront not yet there) nor free of the
    truncation everywhere (wavefront past: its polynomial form is applied instead)."""
    U = R.m2l_matrix(lev, o, gap=gap)
    return bool((U == 0).any() and (U > 0).any())


def test_m2l_flop_count_equals_the_dense_products_the_oracle_makes(monkeypatch):
    """The roofline's numerator: bench.py's algorithmic M2L flops of a march (2 P^2 per
    dense near-future block product, interval ends counted from the samples) equal the flops
    of the dense near-future matrix products (eq. m2l_near) the oracle's Algorithm 1 makes
    over the same march."""
    import synth
    from oracle import fmm as F
    xyz, tri = synth.icosphere(2)
    R = F.ReferenceFMM(xyz, tri, 1.0, 0.02, 2, 1, 3, 2, 2)
    made = []
    orig = F.ReferenceFMM.m2l_matrix

    def counted(self, lev, o, gap=None, deriv=0):
        if deriv == 0:
            made.append((lev, o, gap))
        return orig(self, lev, o, gap=gap, deriv=deriv)
    monkeypatch.setattr(F.ReferenceFMM, "m2l_matrix", counted)
    nt = 2 * R.M[2] + 3
    u = synth.random_history(R.geom.ns, nt, seed=1)
    q = synth.random_history(R.geom.ns, nt, seed=2)
    R.history_rhs(nt, u, q)       # samples 0 .. nt-2, as in a march of nt steps
    monkeypatch.setattr(F.ReferenceFMM, "m2l_matrix", orig)
    flops = sum(2 * R.P ** 2 * len(R.il_by_off[lev][o][0]) for lev, o, gap in made if oracle_dense(R, lev, o, gap))
    dense = [0] * (R.D + 1)
    for lev in range(2, R.D + 1):
        for o, (oi, _) in R.il_by_off[lev].items():
            dense[lev] += len(oi) * sum(oracle_dense(R, lev, o, g) for g in range(1, R.mu + 2))
    want = 2 * R.P ** 2 * bench.m2l_dense_blocks({"m2l_dense_blocks": dense}, range(0, nt - 1), R.m_leaf, R.D)
    assert flops > 0 and flops == want, (flops, want)
