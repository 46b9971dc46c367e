"""Captured-march replay (opts.graph) and the multi-scatterer batch (tdbem_run_batch).

A replayed march must equal the eagerly issued march: bitwise when both use
the same kernels (single-workgroup solve, Ns <= 2048), to 1e-9 relative L2
when the eager march uses the cooperative multi-workgroup solver (different
summation order, GMRES to 1e-12).  Every replay is checked, with eager work and
synchronisations between replays.  A batch must reproduce each context's
stand-alone march.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _P():
    import paper_2111_05205_amd as P
    return P


def _rel(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


@pytest.mark.parametrize("case", ["direct_l2", "fmm_l3", "fmm_geo11", "fmm_l3_f32_direct"])
def test_graph_replay_matches_eager(case):
    P = _P()
    force = None
    if case == "fmm_l3_f32_direct":
        # FP32 products on an LDS-free tile (P = 256): the moment conversion and
        # the tile are captured too
        xyz, tri = synth.icosphere(3)
        kw, d, bc, nt = dict(use_fmm=1, depth=3, p_s=4, p_t=4, m2l_prec=P.M2L_FP32), 2, P.NEUMANN, 40
        force = 2 * 9
    elif case == "direct_l2":
        xyz, tri = synth.icosphere(2)
        kw, d, bc, nt = dict(use_fmm=0), 1, P.DIRICHLET, 40
    elif case == "fmm_l3":
        xyz, tri = synth.icosphere(3)
        kw, d, bc, nt = dict(use_fmm=1, depth=3, p_s=3, p_t=3), 2, P.NEUMANN, 48
    else:
        xyz, tri = synth.geodesic_sphere(11)  # 2420 faces: the eager march uses the cooperative solver
        kw, d, bc, nt = dict(use_fmm=1, depth=3, p_s=3, p_t=3), 2, P.NEUMANN, 40
    dt = synth.mean_edge_length(xyz, tri)
    inc = synth.incident_params(xyz, seed=4)
    eager = P.TDBEM(xyz, tri, 1.0, dt, d, P.BMBIE, bc, nt_max=nt, **kw)
    g = P.TDBEM(xyz, tri, 1.0, dt, d, P.BMBIE, bc, nt_max=nt, graph=True, stream=torch.cuda.Stream(), **kw)
    if force is not None:
        for n in (1, 2):
            eager.set_m2l_variant(n, force)
            g.set_m2l_variant(n, force)
    xe, re_ = eager.run(nt, inc=inc)
    tol = 1e-9 if case == "fmm_geo11" else 0.0
    for rep in range(3):
        g.reset()
        xg, rg = g.run(nt, inc=inc)
        torch.cuda.synchronize()
        err = _rel(xg, xe)
        assert err <= tol, (rep, err)
        assert rg["steps"] == nt - 1 and rg["max_resid"] <= 1e-12
        # eager work on the default stream between replays
        eager.reset()
        eager.run(nt, inc=inc)
        torch.cuda.synchronize()
    # the stored history after a replay is the march's
    u, q = g.get_history(nt - 1)
    assert _rel(u if bc == P.NEUMANN else q, xe) <= tol


def test_graph_with_learned_guess_and_fallback_paths():
    P = _P()
    from paper_2111_05205_amd import mlp
    xyz, tri = synth.icosphere(2)
    dt = synth.mean_edge_length(xyz, tri)
    inc = synth.incident_params(xyz, seed=2)
    nt = 30
    params = mlp.init_params(5)
    a = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=nt, guess=P.GUESS_MLP)
    a.mlp_load(params)
    xa, ra = a.run(nt, inc=inc)
    b = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=nt, guess=P.GUESS_MLP, graph=True,
                stream=torch.cuda.Stream())
    b.mlp_load(params)
    for _ in range(2):
        b.reset()
        xb, rb = b.run(nt, inc=inc)
        assert torch.equal(xa, xb) and rb["total_iters"] == ra["total_iters"]
    # profiling switches the graph off for that run; the result is the same
    b.reset()
    b.profile(True)
    xc, _ = b.run(nt, inc=inc)
    b.profile(False)
    assert torch.equal(xa, xc)
    # a different nt captures a new graph
    b.reset()
    xd, rd = b.run(20, inc=inc)
    assert rd["steps"] == 19 and torch.equal(xd, xa[:19])


def _batch_case(P, k, graph):
    """Small scatterers of different shape, size, order and length."""
    rng = np.random.default_rng(100 + k)
    freq = int(rng.integers(5, 9))
    if k % 2:
        xyz, tri = synth.rounded_cube(freq, half=float(rng.uniform(0.5, 1.0)))
    else:
        xyz, tri = synth.ellipsoid(freq, rng.uniform(0.5, 1.5, size=3))
    d = 1 + k % 2
    nt = int(rng.integers(24, 48))
    dt = synth.mean_edge_length(xyz, tri)
    inc = synth.incident_params(xyz, seed=k)
    args = (xyz, tri, 1.0, dt, d, P.BMBIE, P.NEUMANN)
    s = P.TDBEM(*args, nt_max=nt, use_fmm=0, graph=graph, stream=torch.cuda.Stream())
    return s, nt, inc, args


@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_standalone(graph):
    P = _P()
    cases = [_batch_case(P, k, graph) for k in range(5)]
    solvers = [c[0] for c in cases]
    nts = [c[1] for c in cases]
    incs = [c[2] for c in cases]
    for rep in range(2):
        for s in solvers:
            s.reset()
        outs, infos, wall = P.run_batch(solvers, nts, incs)
        assert wall > 0.0
        for (s, nt, inc, args), x, ri in zip(cases, outs, infos):
            ref = P.TDBEM(*args, nt_max=nt, use_fmm=0)
            xr, rr = ref.run(nt, inc=inc)
            assert ri["steps"] == nt - 1 and ri["total_iters"] == rr["total_iters"]
            assert torch.equal(x, xr)  # same kernels in the same order (Ns <= 2048: one solver)
            ref.close()


def test_batch_errors():
    P = _P()
    xyz, tri = synth.icosphere(1)
    dt = synth.mean_edge_length(xyz, tri)
    s = P.TDBEM(xyz, tri, 1.0, dt, 1, P.BMBIE, P.NEUMANN, nt_max=10)
    with pytest.raises(P.TDBEMError):
        P.run_batch([s], [11], None)  # beyond nt_max


def test_graph_rerecorded_after_network_reload():
    """A march captured with network A, then network B loaded into the same
    context: the next graph run equals an eager march with B (bitwise: same
    kernels), so the replay cannot read A's freed or stale parameters."""
    P = _P()
    from paper_2111_05205_amd import mlp
    xyz, tri = synth.icosphere(2)
    dt = synth.mean_edge_length(xyz, tri)
    inc = synth.incident_params(xyz, seed=5)
    nt = 30
    pa = mlp.init_params(1)
    pb = mlp.init_params(2)
    eager = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=nt, guess=P.GUESS_MLP_ONLY)
    eager.mlp_load(pb)
    xe, re_ = eager.run(nt, inc=inc)
    g = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=nt, guess=P.GUESS_MLP_ONLY, graph=True,
                stream=torch.cuda.Stream())
    g.mlp_load(pa)
    xa, ra = g.run(nt, inc=inc)
    for rep in range(2):
        g.mlp_load(pb)
        g.reset()
        xg, rg = g.run(nt, inc=inc)
        torch.cuda.synchronize()
        assert rg["total_iters"] == re_["total_iters"], (rep, rg["total_iters"], re_["total_iters"], ra["total_iters"])
        assert torch.equal(xg, xe), rep
