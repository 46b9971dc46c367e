"""GPU space-time FMM through the C ABI against the oracle's reference FMM at identical
parameters (tree, hierarchy, mu, Chebyshev nodes, near/far split): relative L2 <= 1e-10."""
import numpy as np
import pytest

import synth
from oracle import fmm as F
from oracle import mot

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _P():
    import paper_2111_05205_amd as P
    return P


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def s3():
    xyz, tri = synth.icosphere(3)
    return xyz, tri, synth.mean_edge_length(xyz, tri)


@pytest.mark.parametrize("d,bie,bc", [(2, 1, 1), (1, 1, 0)])
def test_fmm_history_sum_matches_oracle(s3, d, bie, bc):
    P = _P()
    xyz, tri, dt = s3
    g = P.TDBEM(xyz, tri, 1.0, dt, d, bie, bc, use_fmm=1, depth=3, p_s=3, p_t=3, nt_max=64)
    R = F.ReferenceFMM(xyz, tri, 1.0, dt, d, bie, 3, 3, 3)
    inf = g.info()
    assert inf["mu"] == R.mu and inf["m_leaf"] == R.m_leaf
    assert inf["near_pairs"] == R.near_pairs
    assert inf["il_pairs"][2] == len(R.il[2]) and inf["il_pairs"][3] == len(R.il[3])
    u = synth.random_history(g.ns, 30, seed=11)
    q = synth.random_history(g.ns, 30, seed=12)
    dev = torch.device("cuda")
    for nsteps in (1, 6, 27):
        g.set_history(torch.tensor(u[:nsteps], device=dev), torch.tensor(q[:nsteps], device=dev))
        got = g.fmm_eval(nsteps + 1).cpu().numpy()
        want = R.history_rhs(nsteps + 1, u, q)
        assert _rel(got, want) < 1e-10, (nsteps, _rel(got, want))


def test_fmm_history_sum_d3_matches_oracle(s3):
    """d = 3: the recurrence with c_0^3(k) = 6k, c_1^3 = -6 and three auxiliaries.
    Single-layer history only (the oracle's closed-form derivatives stop at d = 2)."""
    P = _P()
    xyz, tri, dt = s3
    g = P.TDBEM(xyz, tri, 1.0, dt, 3, P.OBIE, P.DIRICHLET, use_fmm=1, depth=3, p_s=3, p_t=4, nt_max=64)
    R = F.ReferenceFMM(xyz, tri, 1.0, dt, 3, 0, 3, 3, 4)
    assert g.info()["mu"] == R.mu
    q = synth.random_history(g.ns, 40, seed=21)
    u0 = np.zeros_like(q)
    dev = torch.device("cuda")
    for nsteps in (5, 18, 37):
        g.set_history(None, torch.tensor(q[:nsteps], device=dev))
        got = g.fmm_eval(nsteps + 1).cpu().numpy()
        want = R.history_rhs(nsteps + 1, u0, q)
        assert _rel(got, want) < 1e-10, (nsteps, _rel(got, want))


def test_fmm_single_level_p4_matches_oracle():
    P = _P()
    xyz, tri = synth.icosphere(2)
    dt = synth.mean_edge_length(xyz, tri)
    g = P.TDBEM(xyz, tri, 1.0, dt, 2, 1, 1, use_fmm=1, depth=2, p_s=4, p_t=4, nt_max=32)
    R = F.ReferenceFMM(xyz, tri, 1.0, dt, 2, 1, 2, 4, 4)
    u = synth.random_history(g.ns, 24, seed=3)
    dev = torch.device("cuda")
    g.set_history(torch.tensor(u[:20], device=dev), None)
    got = g.fmm_eval(21).cpu().numpy()
    want = R.history_rhs(21, u, np.zeros_like(u))
    assert _rel(got, want) < 1e-10


def test_fmm_march_matches_oracle(s3):
    P = _P()
    xyz, tri, dt = s3
    nt = 36
    inc = synth.incident_params(xyz, seed=0)
    g = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, use_fmm=1, depth=3, p_s=3, p_t=3, nt_max=nt)
    x, info = g.run(nt, inc=inc)
    R = F.ReferenceFMM(xyz, tri, 1.0, dt, 2, 1, 3, 3, 3, bc=mot.NEUMANN)
    u, q = R.run(nt, mot.incident(R.geom, inc, 1.0, dt, nt, 1))
    assert _rel(x.cpu().numpy(), u) < 1e-10


def test_fmm_rejects_bad_options(s3):
    P = _P()
    xyz, tri, dt = s3
    for kw in (dict(depth=6), dict(p_s=9), dict(p_t=2), dict(mu=2)):
        args = dict(use_fmm=1, depth=3, p_s=3, p_t=3)
        args.update(kw)
        with pytest.raises(P.TDBEMError):
            P.TDBEM(xyz, tri, 1.0, dt, 2, 1, 1, nt_max=8, **args)


def test_fmm_fp32_m2l_products(s3):
    """Mixed precision: M2L operators and products in FP32 (FP32 accumulation), everything else
    FP64.  The history sum stays within FP32 rounding of the FP64 oracle FMM."""
    P = _P()
    xyz, tri, dt = s3
    g = P.TDBEM(xyz, tri, 1.0, dt, 2, 1, 1, use_fmm=1, depth=3, p_s=3, p_t=3, m2l_prec=P.M2L_FP32, nt_max=64)
    R = F.ReferenceFMM(xyz, tri, 1.0, dt, 2, 1, 3, 3, 3)
    u = synth.random_history(g.ns, 30, seed=13)
    dev = torch.device("cuda")
    g.set_history(torch.tensor(u[:25], device=dev), None)
    got = g.fmm_eval(26).cpu().numpy()
    want = R.history_rhs(26, u, np.zeros_like(u))
    e = _rel(got, want)
    assert 1e-12 < e < 1e-4, e


@pytest.mark.parametrize("pp", [3, 4])
def test_fmm_bf16_m2l_products(pp):
    """BF16 near-future products (operators and moments rounded to bf16, FP32 accumulation on
    v_mfma_f32_16x16x32_bf16), derivative products and everything else FP64: every BF16 tile
    shape (moments read per lane, or staged through LDS), one item per workgroup and persistent,
    against the FP64 oracle FMM.  p = 3 gives
    P = 81 (K padded to 96), p = 4 P = 256."""
    P = _P()
    xyz, tri = synth.icosphere(2)
    dt = synth.mean_edge_length(xyz, tri)
    R = F.ReferenceFMM(xyz, tri, 1.0, dt, 2, 1, 2, pp, pp)
    ns = tri.shape[0]
    u = synth.random_history(ns, 24, seed=5)
    q = synth.random_history(ns, 24, seed=6)
    want = R.history_rhs(21, u, q)
    # the oracle with both factors of the dense near-future products (the blocks the
    # wavefront crosses) rounded to bf16, as the BF16 path forms them (products then
    # exact, sums in FP64 here and FP32 there); the other blocks are exact on both sides
    from oracle import mlp as OM
    Rb = F.ReferenceFMM(xyz, tri, 1.0, dt, 2, 1, 2, pp, pp, near_round=OM.bf16)
    want_b = Rb.history_rhs(21, u, q)
    dev = torch.device("cuda")
    g = P.TDBEM(xyz, tri, 1.0, dt, 2, 1, 1, use_fmm=1, depth=2, p_s=pp, p_t=pp, m2l_prec=P.M2L_BF16, nt_max=32)
    errs, errs_b = {}, {}
    for choice in range(16, 36):  # BF16 tiles 8..11, their LDS-staged forms 12..15, and 16..17
        g.set_m2l_variant(1, choice)
        g.set_history(torch.tensor(u[:20], device=dev), torch.tensor(q[:20], device=dev))
        got = g.fmm_eval(21).cpu().numpy()
        errs[choice] = _rel(got, want)
        errs_b[choice] = _rel(got, want_b)
    print("BF16 history sum vs FP64 oracle FMM:", errs, "vs the bf16-rounded oracle:", errs_b,
          "rounding effect in the oracle:", _rel(want_b, want))
    # the rounding of the factors is the whole difference: the bf16 path reproduces the
    # rounded oracle to well under the rounding effect itself
    assert all(e < 0.02 * _rel(want_b, want) for e in errs_b.values()), errs_b
    with pytest.raises(P.TDBEMError):
        g.set_m2l_variant(1, 2)  # the LDS tiles are FP32 / FP64 only
    g.close()


@pytest.mark.parametrize("pp", [3, 4])
def test_fmm_bf16x3_m2l_products(pp):
    """Split BF16 products: both factors of a dense near-future product as x = hi + lo in bf16,
    products hi*hi + hi*lo + lo*hi with FP32 accumulation, every BF16 tile shape, one item per
    workgroup and persistent.  Against the oracle forming the same three products (in FP64), and
    against the exact FP64 oracle FMM, which it must approach to FP32-like accuracy."""
    from oracle import mlp as OM

    def prod3(X, U):
        Xh, Uh = OM.bf16(X), OM.bf16(U)
        Xl, Ul = OM.bf16(X - Xh), OM.bf16(U - Uh)
        return Xh @ Uh.T + Xh @ Ul.T + Xl @ Uh.T
    P = _P()
    xyz, tri = synth.icosphere(2)
    dt = synth.mean_edge_length(xyz, tri)
    R = F.ReferenceFMM(xyz, tri, 1.0, dt, 2, 1, 2, pp, pp)
    ns = tri.shape[0]
    u = synth.random_history(ns, 24, seed=5)
    q = synth.random_history(ns, 24, seed=6)
    want = R.history_rhs(21, u, q)
    Rb = F.ReferenceFMM(xyz, tri, 1.0, dt, 2, 1, 2, pp, pp, near_product=prod3)
    want_b = Rb.history_rhs(21, u, q)
    dev = torch.device("cuda")
    g = P.TDBEM(xyz, tri, 1.0, dt, 2, 1, 1, use_fmm=1, depth=2, p_s=pp, p_t=pp, m2l_prec=P.M2L_BF16X3, nt_max=32)
    errs, errs_b = {}, {}
    for choice in range(16, 36):  # BF16 tiles 8..11, their LDS-staged forms 12..15, and 16..17
        g.set_m2l_variant(1, choice)
        g.set_history(torch.tensor(u[:20], device=dev), torch.tensor(q[:20], device=dev))
        got = g.fmm_eval(21).cpu().numpy()
        errs[choice] = _rel(got, want)
        errs_b[choice] = _rel(got, want_b)
    eff = _rel(want_b, want)
    print("BF16X3 history sum vs FP64 oracle FMM:", errs, "vs the split-product oracle:", errs_b,
          "split effect in the oracle:", eff)
    assert eff < 1e-4
    assert all(e < 0.2 * eff for e in errs_b.values()), errs_b
    assert all(e < 1e-4 for e in errs.values()), errs
    g.close()


def test_fmm_padded_row_pitch_matches_oracle():
    """p_s = 3, p_t = 7 (P = 189): each gap's operator rows and each pair's staged products sit at a
    pitch of 192 rows, the zero-padded layout the benchmarked order (P = 625 at a pitch of 640) uses.
    History sums against the oracle's FMM: FP64 products to 1e-10 (autotuned tile and two forced
    ones), split BF16 against the oracle forming the same three products."""
    from oracle import mlp as OM

    def prod3(X, U):
        Xh, Uh = OM.bf16(X), OM.bf16(U)
        Xl, Ul = OM.bf16(X - Xh), OM.bf16(U - Uh)
        return Xh @ Uh.T + Xh @ Ul.T + Xl @ Uh.T
    P = _P()
    xyz, tri = synth.icosphere(2)
    dt = synth.mean_edge_length(xyz, tri)
    ns = tri.shape[0]
    u = synth.random_history(ns, 24, seed=15)
    q = synth.random_history(ns, 24, seed=16)
    want = F.ReferenceFMM(xyz, tri, 1.0, dt, 2, 1, 2, 3, 7).history_rhs(21, u, q)
    want_b = F.ReferenceFMM(xyz, tri, 1.0, dt, 2, 1, 2, 3, 7, near_product=prod3).history_rhs(21, u, q)
    dev = torch.device("cuda")
    for prec, choices in ((P.M2L_FP64, [None, 2 * 6, 2 * 3 + 1]), (P.M2L_BF16X3, [None, 2 * 17, 2 * 12])):
        g = P.TDBEM(xyz, tri, 1.0, dt, 2, 1, 1, use_fmm=1, depth=2, p_s=3, p_t=7, m2l_prec=prec, nt_max=32)
        for ch in choices:
            if ch is not None:
                g.set_m2l_variant(1, ch)
            g.set_history(torch.tensor(u[:20], device=dev), torch.tensor(q[:20], device=dev))
            got = g.fmm_eval(21).cpu().numpy()
            if prec == P.M2L_FP64:
                assert _rel(got, want) < 1e-10, (ch, _rel(got, want))
            else:
                eff = _rel(want_b, want)
                print(f"split BF16 tile {ch}: vs split oracle {_rel(got, want_b):.2e}, vs FP64 oracle "
                      f"{_rel(got, want):.2e}, split effect {eff:.2e}")
                assert _rel(got, want_b) < 0.2 * eff and _rel(got, want) < 1e-4
        g.close()


def test_fmm_bf16x3_every_tile_at_p5():
    """p_s = p_t = 5 (P = 625, each gap's rows at a pitch of 640), the benchmarked order, where the
    oracle's FMM is too slow for a test: every BF16 tile, one item per workgroup and persistent,
    gives the same sums bit for bit (the same products in the same K order), and the split-BF16
    sums stay within the split-product error of the FP64 products (pinned to the oracle's FMM at
    other orders, the 640-row pitch at P = 189)."""
    P = _P()
    xyz, tri = synth.icosphere(2)
    dt = synth.mean_edge_length(xyz, tri)
    ns = tri.shape[0]
    u = synth.random_history(ns, 24, seed=25)
    q = synth.random_history(ns, 24, seed=26)
    dev = torch.device("cuda")

    def sums(g):
        g.set_history(torch.tensor(u[:20], device=dev), torch.tensor(q[:20], device=dev))
        return g.fmm_eval(21).cpu().numpy()
    g64 = P.TDBEM(xyz, tri, 1.0, dt, 2, 1, 1, use_fmm=1, depth=2, p_s=5, p_t=5, m2l_prec=P.M2L_FP64, nt_max=32)
    want = sums(g64)
    g64.close()
    g = P.TDBEM(xyz, tri, 1.0, dt, 2, 1, 1, use_fmm=1, depth=2, p_s=5, p_t=5, m2l_prec=P.M2L_BF16X3, nt_max=32)
    got = {}
    for choice in range(16, 36):
        g.set_m2l_variant(1, choice)
        got[choice] = sums(g)
    g.close()
    ref = got[16]  # 32 columns x 128 rows, no LDS stage, every K step multiplied
    assert all(np.array_equal(v, ref) for v in got.values()), [c for c, v in got.items() if not np.array_equal(v, ref)]
    e = _rel(ref, want)
    print(f"split BF16 vs FP64 products at P = 625: {e:.2e}")
    assert 1e-8 < e < 2e-4, e


@pytest.mark.parametrize("depth,pp", [(3, 3), (3, 4)])
def test_dense_block_count_matches_the_oracle_operators(depth, pp):
    """The library evaluates a near-future block (eq. Uabmn) as a dense product only where the
    wavefront crosses the offset's node set; elsewhere the oracle's interpolated operator is
    zero at every node pair or free of the truncation.  Per level, the number of dense
    (pair, gap) products equals the count from the oracle's own operator matrices."""
    P = _P()
    xyz, tri = synth.icosphere(3)
    dt = synth.mean_edge_length(xyz, tri)
    R = F.ReferenceFMM(xyz, tri, 1.0, dt, 2, 1, depth, pp, pp)
    g = P.TDBEM(xyz, tri, 1.0, dt, 2, 1, 1, use_fmm=1, depth=depth, p_s=pp, p_t=pp, nt_max=8)
    info = g.info()
    assert info["mu"] == R.mu
    for lev in range(2, depth + 1):
        want = 0
        for o, (oi, _) in R.il_by_off[lev].items():
            for gap in range(1, R.mu + 2):
                U = R.m2l_matrix(lev, o, gap=gap)
                want += len(oi) * int(bool((U == 0).any() and (U > 0).any()))
        assert info["m2l_dense_blocks"][lev] == want, (lev, info["m2l_dense_blocks"][lev], want)
        assert 0 < want < (R.mu + 1) * len(R.il[lev])
    g.close()


N_M2L_TILES = 12  # tdbem_info.m2l_variant: choice = 2 * tile + persistent


def test_fmm_every_m2l_variant_matches_oracle():
    """Every M2L tile shape, one item per workgroup and persistent, FP64 and FP32,
    forced with tdbem_set_m2l_variant: the history sum against the oracle's FMM
    (P = 256, so the LDS-free tiles 8..11 are eligible)."""
    P = _P()
    xyz, tri = synth.icosphere(2)
    dt = synth.mean_edge_length(xyz, tri)
    R = F.ReferenceFMM(xyz, tri, 1.0, dt, 2, 1, 2, 4, 4)
    ns = tri.shape[0]
    u = synth.random_history(ns, 24, seed=3)
    q = synth.random_history(ns, 24, seed=4)
    want = R.history_rhs(21, u, q)
    dev = torch.device("cuda")
    for prec, tol in ((P.M2L_FP64, 1e-10), (P.M2L_FP32, 1e-4)):
        g = P.TDBEM(xyz, tri, 1.0, dt, 2, 1, 1, use_fmm=1, depth=2, p_s=4, p_t=4, m2l_prec=prec, nt_max=32)
        for choice in range(2 * N_M2L_TILES):
            g.set_m2l_variant(1, choice)
            assert g.info()["m2l_variant"][1] == choice
            g.set_history(torch.tensor(u[:20], device=dev), torch.tensor(q[:20], device=dev))
            e = _rel(g.fmm_eval(21).cpu().numpy(), want)
            assert e < tol, (prec, choice, e)
        with pytest.raises(P.TDBEMError):
            g.set_m2l_variant(1, 2 * N_M2L_TILES)
        with pytest.raises(P.TDBEMError):
            g.set_m2l_variant(2, 0)  # depth 2: only n = 1
        g.close()


def test_fmm_m2l_variants_agree_across_levels(s3):
    """Launches covering two levels at once (depth 3): every variant gives the
    autotuned variant's history sum (FP64 1e-12, FP32 1e-5 relative)."""
    P = _P()
    xyz, tri, dt = s3
    u = synth.random_history(tri.shape[0], 30, seed=5)
    dev = torch.device("cuda")
    for prec, tol in ((P.M2L_FP64, 1e-12), (P.M2L_FP32, 1e-5)):
        g = P.TDBEM(xyz, tri, 1.0, dt, 2, 1, 1, use_fmm=1, depth=3, p_s=4, p_t=4, m2l_prec=prec, nt_max=40)
        g.set_history(torch.tensor(u[:27], device=dev), None)
        ref = g.fmm_eval(28).cpu().numpy()
        for choice in range(2 * N_M2L_TILES):
            for n in (1, 2):
                g.set_m2l_variant(n, choice)
            g.set_history(torch.tensor(u[:27], device=dev), None)
            e = _rel(g.fmm_eval(28).cpu().numpy(), ref)
            assert e < tol, (prec, choice, e)
        g.close()


def test_fmm_direct_tiles_need_p_multiple_of_4(s3):
    P = _P()
    xyz, tri, dt = s3
    g = P.TDBEM(xyz, tri, 1.0, dt, 2, 1, 1, use_fmm=1, depth=3, p_s=3, p_t=3, nt_max=8)  # P = 81
    g.set_m2l_variant(1, 2 * 7)
    with pytest.raises(P.TDBEMError):
        g.set_m2l_variant(1, 2 * 8)
    g.close()


@pytest.mark.parametrize("d,bie,bc,p,level,depth", [(2, 1, 1, 3, 3, 3), (1, 1, 0, 4, 2, 2)])
def test_fmm_hermite_interpolation_matches_oracle(d, bie, bc, p, level, depth):
    """The paper's interpolation (cubic Hermite with finite-difference slopes, equispaced
    nodes): same parity bar as the Lagrange basis against the oracle's Hermite FMM."""
    P = _P()
    xyz, tri = synth.icosphere(level)
    dt = synth.mean_edge_length(xyz, tri)
    g = P.TDBEM(xyz, tri, 1.0, dt, d, bie, bc, use_fmm=1, depth=depth, p_s=p, p_t=p, nt_max=64,
                interp=P.INTERP_HERMITE)
    R = F.ReferenceFMM(xyz, tri, 1.0, dt, d, bie, depth, p, p, interp="hermite")
    assert g.info()["mu"] == R.mu and g.info()["m_leaf"] == R.m_leaf
    u = synth.random_history(g.ns, 30, seed=13)
    q = synth.random_history(g.ns, 30, seed=14)
    dev = torch.device("cuda")
    for nsteps in (2, 23):
        g.set_history(torch.tensor(u[:nsteps], device=dev), torch.tensor(q[:nsteps], device=dev))
        got = g.fmm_eval(nsteps + 1).cpu().numpy()
        want = R.history_rhs(nsteps + 1, u, q)
        assert _rel(got, want) < 1e-10, (nsteps, _rel(got, want))


def test_hermite_needs_three_nodes(s3):
    P = _P()
    xyz, tri, dt = s3
    with pytest.raises(P.TDBEMError) as e:
        P.TDBEM(xyz, tri, 1.0, dt, 1, 1, 1, use_fmm=1, depth=3, p_s=2, p_t=3, nt_max=8, interp=P.INTERP_HERMITE)
    assert e.value.code == P._native.E_INVAL
