"""ORACLE — test infrastructure, not product code.

A plain, slow FP64 CPU implementation of what the time-domain BEM hot path
computes, written from the paper (Takahashi, Tanigawa, Miyazawa, "An
enhancement of the fast time-domain boundary element method for the
three-dimensional wave equation"):

* ``bspline``  — B-spline temporal basis and its truncated-power weights (eqs. u_bspline, decompose, w; Table 1)
* ``elemint``  — closed-form element integrals U, W and their Burton-Miller versions (App. B, eq. U_W_BM), in plain C
* ``mot``      — direct marching-on-in-time with no FMM (eqs. bie_disc, linear, sigma_tau_tilde)
* ``fmm``      — a literal reference of the interpolation-based space-time FMM (Sections 3-4, Algorithm 1)

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the HIP library and never
imports it.
"""
