"""GPU parity of the learned-guess network kernels and of the guess inside the march.

Tolerances, derived from the arithmetic: both sides round weights and layer
inputs to bfloat16 at the same points; the library accumulates in FP32, the
oracle in FP64, so pre-activations differ by ~1e-6 relative.  A hidden value
that lies within that distance of a bfloat16 rounding boundary rounds to the
neighbouring value (one bf16 ulp, 2^-8 relative) and, rarely, a ReLU mask
flips.  Outputs: relative L2 <= 2e-4; gradients: relative L2 <= 1e-3 (the bound
the network's gradient check asks for with bf16 weights); loss, dy and Adam
(pure FP32 element-wise on identical inputs): 1e-6 relative.
"""
import ctypes

import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from oracle import mot

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _P():
    import paper_2111_05205_amd as P
    return P


def _M():
    from paper_2111_05205_amd import mlp
    return mlp


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _params(seed, bias=0.1):
    p = omlp.init_params(seed).astype(np.float64)
    P = omlp.unpack(p)
    rng = np.random.default_rng(seed + 11)
    for k in ("b1", "b2", "b3", "b4"):
        P[k][...] = rng.normal(size=P[k].shape) * bias
    return omlp.pack(P).astype(np.float32)


def _feat(n, seed):
    f = np.random.default_rng(seed).normal(size=(n, 16)).astype(np.float32)
    f[:, 12:] = 0.0
    return f


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("n", [1, 64, 64 * 5 + 37])
def test_forward_matches_oracle(n):
    M = _M()
    p, f = _params(1), _feat(n, 2)
    y, act = M.forward(_dev(p), _dev(f), act=True)
    yr, cache = omlp.forward(p.astype(np.float64), f.astype(np.float64))
    assert _rel(y.cpu().numpy(), yr) < 2e-4
    # hidden activations: bf16 values, equal to the oracle's except for rare one-ulp boundary cases
    a = act.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    a = a.view(np.float32).astype(np.float64)
    for k, name in enumerate(("h1", "h2", "h3")):
        ref = cache[name]
        diff = a[k] != ref
        assert diff.mean() < 2e-3, (name, diff.mean())
        assert np.all(np.abs(a[k] - ref)[diff] <= 2.0 ** -7 * np.abs(ref)[diff] + 1e-30)


@pytest.mark.parametrize("n", [1, 300, 5120])
def test_loaded_forward_equals_api_forward(n):
    """The march's forward (hidden-layer weights pre-packed as bf16 fragments at
    mlp_load) gives the API forward's outputs bit for bit."""
    M = _M()
    P = _P()
    xyz, tri = synth.icosphere(1)
    s = P.TDBEM(xyz, tri, 1.0, synth.mean_edge_length(xyz, tri), 2, P.BMBIE, P.NEUMANN, nt_max=8,
                guess=P.GUESS_MLP)
    p, f = _params(7), _feat(n, 8)
    with pytest.raises(P.TDBEMError):
        s.mlp_forward_loaded(_dev(f))  # nothing installed yet
    s.mlp_load(_dev(p))
    y_api = M.forward(_dev(p), _dev(f))
    y_loaded = s.mlp_forward_loaded(_dev(f))
    assert torch.equal(y_api, y_loaded)
    s.close()


def test_forward_ragged_rows_only_written():
    M = _M()
    n = 100
    p, f = _params(3), _feat(n, 4)
    y = M.forward(_dev(p), _dev(f))
    y2 = M.forward(_dev(p), _dev(f[:37]))
    assert torch.equal(y[:37], y2)  # each row depends on its own features only


@pytest.mark.parametrize("n", [64 * 3 + 5, 1000])
def test_backward_matches_oracle(n):
    M = _M()
    p, f = _params(5), _feat(n, 6)
    dy = np.random.default_rng(7).normal(size=n).astype(np.float32)
    y, act = M.forward(_dev(p), _dev(f), act=True)
    g = M.backward(_dev(p), _dev(f), act, _dev(dy)).cpu().numpy()
    _, cache = omlp.forward(p.astype(np.float64), f.astype(np.float64))
    gr = omlp.backward(cache, dy.astype(np.float64))
    assert _rel(g, gr) < 1e-3
    Gb, Rb = omlp.unpack(g), omlp.unpack(gr)
    for name, _ in omlp.layout():
        assert _rel(Gb[name], Rb[name]) < 3e-3, name
    assert np.all(Gb["W1"][:, 12:] == 0.0)
    # deterministic
    g2 = M.backward(_dev(p), _dev(f), act, _dev(dy)).cpu().numpy()
    assert np.array_equal(g, g2)


def test_backward_empty_batch_gives_zero():
    M = _M()
    p = _dev(_params(8))
    f = torch.zeros(0, 16, dtype=torch.float32, device="cuda")
    y, act = M.forward(p, f, act=True)
    g = M.backward(p, f, act, torch.zeros(0, dtype=torch.float32, device="cuda"))
    assert y.numel() == 0 and float(g.abs().max()) == 0.0


def test_mse_and_adam_match_oracle():
    M = _M()
    rng = np.random.default_rng(9)
    y, t = rng.normal(size=777).astype(np.float32), rng.normal(size=777).astype(np.float32)
    loss, dy = M.mse(_dev(y), _dev(t))
    lr_, dyr = omlp.mse(y.astype(np.float64), t.astype(np.float64))
    assert abs(float(loss) - lr_) <= 1e-6 * lr_
    assert _rel(dy.cpu().numpy(), dyr) < 1e-6
    n = omlp.nparams()
    p0 = rng.normal(size=n).astype(np.float32)
    opt = M.Adam(_dev(p0), lr=1e-2)
    pd = _dev(p0)
    pr, m, v = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    for t_ in range(1, 4):
        g = rng.normal(size=n).astype(np.float32)
        opt.step(pd, _dev(g))
        pr, m, v = omlp.adam(pr, g.astype(np.float64), m, v, t_, lr=1e-2)
    assert _rel(pd.cpu().numpy() - p0, pr - p0) < 1e-5


def test_argument_errors():
    P, M = _P(), _M()
    L = P._native.lib()
    p = _dev(_params(1))
    f = torch.zeros(64 * 16 + 1, dtype=torch.float32, device="cuda")
    y = torch.zeros(64, dtype=torch.float32, device="cuda")
    # misaligned features
    rc = L.tdbem_mlp_forward(ctypes.c_void_p(p.data_ptr()), 64, ctypes.c_void_p(f.data_ptr() + 4),
                             ctypes.c_void_p(y.data_ptr()), None, None)
    assert rc == P._native.E_INVAL
    # workspace too small
    act = torch.zeros(3 * 64 * 256, dtype=torch.int16, device="cuda")
    w = torch.zeros(10, dtype=torch.float32, device="cuda")
    rc = L.tdbem_mlp_backward(ctypes.c_void_p(p.data_ptr()), 64, ctypes.c_void_p(f.data_ptr()),
                              ctypes.c_void_p(act.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                              ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(w.data_ptr()), 10, None)
    assert rc == P._native.E_INVAL
    # step number 0 (Adam counts from 1)
    q = p.clone()
    rc = L.tdbem_mlp_adam_step(ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(q.data_ptr()),
                               ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(q.data_ptr()), 0, 1e-3, 0.9, 0.999,
                               1e-8, None)
    assert rc == P._native.E_INVAL and torch.equal(q, p)
    assert "Adam" in L.tdbem_last_error(None).decode() or "adam" in L.tdbem_last_error(None).decode()
    xyz, tri = synth.icosphere(1)
    with pytest.raises(P.TDBEMError):
        P.TDBEM(xyz, tri, 1.0, synth.mean_edge_length(xyz, tri), 1, 1, 1, guess=7)


@pytest.fixture(scope="module")
def march_case():
    """Icosphere level 2, BMBIE d=2 Neumann, direct; oracle march for b and A."""
    xyz, tri = synth.icosphere(2)
    dt = synth.mean_edge_length(xyz, tri)
    inc = synth.incident_params(xyz, seed=3)
    nt = 40
    ref = mot.DirectMOT(xyz, tri, 1.0, dt, 2, mot.BMBIE, mot.NEUMANN)
    return xyz, tri, dt, inc, nt, ref


def test_recorded_features_and_targets_match_oracle(march_case):
    P = _P()
    xyz, tri, dt, inc, nt, ref = march_case
    s = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=nt)
    fb = torch.zeros(nt * s.ns * 16, dtype=torch.float32, device="cuda")
    tb = torch.zeros(nt * s.ns, dtype=torch.float32, device="cuda")
    s.mlp_record(fb, tb)
    s.run(nt, inc=inc)
    u, _ = s.get_history(nt - 1)
    u = u.cpu().numpy()
    q = np.zeros_like(u)
    forc = mot.incident(ref.geom, inc, 1.0, dt, nt, mot.BMBIE)
    diag = np.diag(ref.A)
    fg = fb.view(nt, s.ns, 16).cpu().numpy()
    tg = tb.view(nt, s.ns).cpu().numpy()
    assert np.all(fg[:4] == 0.0) and np.all(tg[:4] == 0.0)
    for beta in (4, 9, 17, 30, nt - 2):
        b = forc[beta] + ref.history_rhs(beta + 1, u, q)
        f, sc = omlp.features(u, beta, b, diag, xyz, tri)
        assert sc > 0.0
        assert np.max(np.abs(fg[beta] - f)) < 2e-6 * max(1.0, np.abs(f).max()), beta
        t = omlp.target(u[beta], omlp.extrapolate(u, beta), sc)
        assert np.max(np.abs(tg[beta] - t)) < 2e-6 * max(1.0, np.abs(t).max()), beta


@pytest.mark.parametrize("mode", ["ZERO", "PREV", "MLP"])
def test_solution_does_not_depend_on_guess(march_case, mode):
    P, M = _P(), _M()
    xyz, tri, dt, inc, nt, _ = march_case
    base = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=nt)
    x0, r0 = base.run(nt, inc=inc)
    s = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=nt, guess=getattr(P, "GUESS_" + mode))
    if mode == "MLP":
        s.mlp_load(M.init_params(3))
    x1, r1 = s.run(nt, inc=inc)
    assert _rel(x1.cpu().numpy(), x0.cpu().numpy()) < 1e-9
    assert r1["max_resid"] <= 1e-12 and r1["steps"] == nt - 1
    if mode == "ZERO":
        assert r1["guesses_rejected"] == 0  # zero is never worse than zero


def test_garbage_network_falls_back(march_case):
    P, M = _P(), _M()
    xyz, tri, dt, inc, nt, _ = march_case
    base = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=nt)
    x0, _ = base.run(nt, inc=inc)
    s = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=nt, guess=P.GUESS_MLP)
    p = M.init_params(4)
    p[-1] = 1e30  # output bias: every proposal is enormous
    s.mlp_load(p)
    x1, r1 = s.run(nt, inc=inc)
    # every step with a network proposal starts from the extrapolation (or zero) instead
    assert r1["guesses_replaced"] + r1["guesses_rejected"] >= nt - 1 - 4 and r1["guesses_replaced"] >= 1
    assert _rel(x1.cpu().numpy(), x0.cpu().numpy()) < 1e-9
    p[-1] = float("nan")
    s2 = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=nt, guess=P.GUESS_MLP)
    s2.mlp_load(p)
    x2, _ = s2.run(nt, inc=inc)
    assert _rel(x2.cpu().numpy(), x0.cpu().numpy()) < 1e-9


def test_training_reduces_loss(march_case):
    """Library kernels only: record a march, train a few hundred Adam steps."""
    P, M = _P(), _M()
    xyz, tri, dt, inc, nt, _ = march_case
    s = P.TDBEM(xyz, tri, 1.0, dt, 2, P.BMBIE, P.NEUMANN, nt_max=nt)
    fb = torch.zeros(nt * s.ns * 16, dtype=torch.float32, device="cuda")
    tb = torch.zeros(nt * s.ns, dtype=torch.float32, device="cuda")
    s.mlp_record(fb, tb)
    s.run(nt, inc=inc)
    f = fb.view(nt, s.ns, 16)[4:nt - 1].reshape(-1, 16).contiguous()
    t = tb.view(nt, s.ns)[4:nt - 1].reshape(-1).contiguous()
    p0 = M.init_params(0)
    l0 = float(M.mse(M.forward(p0, f), t)[0])
    p, _ = M.train(f, t, steps=300, batch=2048, lr=1e-3, lr_final=1e-4, params=p0)
    l1 = float(M.mse(M.forward(p, f), t)[0])
    assert l1 < 0.2 * l0, (l0, l1)


def test_trained_network_saves_iterations():
    """The committed network (trained on solver-generated ellipsoid runs by the
    library's kernels) against zero, previous-row and extrapolated starting points
    on icosphere level 4 (Ns = 5120), Nt = 256, Burton-Miller d = 2 Neumann, FMM
    depth 4, GMRES to 1e-8: it saves iterations, the solution is unchanged."""
    import os
    P, M = _P(), _M()
    path = os.path.join(os.path.dirname(P.__file__), "data", "mlp_guess.npy")
    params = M.load(path)
    xyz, tri = synth.icosphere(4)
    inc = synth.incident_params(xyz, seed=0)
    res = M.evaluate(params, xyz, tri, 256, inc, modes=("ZERO", "PREV", "EXTRAP", "MLP_ONLY", "MLP"),
                     gmres_tol=1e-8)
    it = {k: v["total"] for k, v in res.items()}
    ms = {k: v["march_ms"] for k, v in res.items()}
    print("GMRES iterations per march:", it, "march ms:", ms)
    # the network's own proposal (no comparison with the extrapolation) against
    # zero and previous-row starts, and the guarded start against all three
    assert it["MLP_ONLY"] < 0.97 * min(it["ZERO"], it["PREV"])
    assert it["MLP"] < 0.97 * min(it["ZERO"], it["PREV"])
    assert it["MLP"] < it["EXTRAP"]
    assert all(v.get("rel_diff_vs_first", 0.0) < 1e-6 for v in res.values())
