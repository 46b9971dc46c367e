"""Writes fmm_sphere5k_alpha64.txt: the oracle's reference FMM (Algorithm 1, FP64) history
sum b^{alpha-1} at alpha = 64 on the benchmarked workload (icosphere level 4, 5120 faces,
Burton-Miller d = 2, c dt = mean edge, octree depth 4, p_s = p_t = 4) for a seeded synthetic
history of u and q (63 rows each).  alpha = 64 closes an interval at every level, so every
level's M2L, M2M and L2L have run.  Calls only oracle/ and the input generators in synth/.

    python tests/golden/make_fmm_sphere5k.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fmm  # noqa: E402

ALPHA = 64
SEEDS = (11, 12)


def main():
    w = synth.workload("sphere5k")
    t0 = time.time()
    R = fmm.ReferenceFMM(w["xyz"], w["tri"], w["c"], w["dt"], w["d"], w["bie"], w["depth"], w["p_s"], w["p_t"])
    ns = R.geom.ns
    u = synth.random_history(ns, ALPHA - 1, seed=SEEDS[0])
    q = synth.random_history(ns, ALPHA - 1, seed=SEEDS[1])
    b = R.history_rhs(ALPHA, u, q)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fmm_sphere5k_alpha64.txt")
    ilp = " ".join(str(len(R.il[lev])) for lev in range(2, R.D + 1))
    with open(out, "w") as fh:
        fh.write("# Oracle reference FMM (Algorithm 1, FP64) history sum b^{alpha-1}, written by make_fmm_sphere5k.py\n")
        fh.write(f"# workload sphere5k  alpha {ALPHA}  history seeds u {SEEDS[0]} q {SEEDS[1]}  rows {ALPHA - 1}\n")
        fh.write(f"# mu {R.mu}  m_leaf {R.m_leaf}  near_pairs {R.near_pairs}  il_pairs(levels 2..{R.D}) {ilp}\n")
        np.savetxt(fh, b, fmt="%.17e")
    print(f"wrote {out} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
