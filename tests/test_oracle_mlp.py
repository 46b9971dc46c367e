"""Pins of the oracle's learned-guess network: bfloat16 rounding against torch's
conversion, backpropagation against finite differences, Adam's closed-form first
step, ReLU homogeneity, a one-hidden-layer special case computed by brute force,
and the feature/target definition against invariants."""
import numpy as np
import pytest
import torch

from oracle import mlp


def _rand_params(seed, bias=0.1):
    p = mlp.init_params(seed).astype(np.float64)
    P = mlp.unpack(p)
    rng = np.random.default_rng(seed + 7)
    for k in ("b1", "b2", "b3", "b4"):
        P[k][...] = rng.normal(size=P[k].shape) * bias
    return mlp.pack(P)


def test_layout_size():
    assert mlp.nparams() == 256 * 16 + 256 + 2 * (256 * 256 + 256) + 256 + 1 == 136193


def test_bf16_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.uniform(-20, 20, size=20000),
                        rng.uniform(-3, 3, size=5000)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x.astype(np.float64)), ref)


def test_bf16_ties_to_even():
    e = 2.0 ** -8
    assert mlp.bf16(1.0 + e) == 1.0                    # halfway, even neighbour is 1
    assert mlp.bf16(1.0 + 3 * e) == 1.0 + 4 * e        # halfway, even neighbour is 1 + 2^-6
    assert mlp.bf16(-(1.0 + 3 * e)) == -(1.0 + 4 * e)
    assert mlp.bf16(1.0 + 1.5 * e) == 1.0 + 2 * e
    assert mlp.bf16(0.0) == 0.0
    assert mlp.bf16(3.0) == 3.0


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = _rand_params(3)
    feat = rng.normal(size=(7, 16))
    dy = rng.normal(size=7)
    y, cache = mlp.forward(p, feat, rounding=False)
    g = mlp.backward(cache, dy)
    # indices in every block, including a padding column of W1 (gradient 0)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.layout()])
    idx = [offs[0] + 5 * 16 + 3, offs[0] + 9 * 16 + 13]
    for b in range(len(offs) - 1):
        idx += list(rng.integers(offs[b], offs[b + 1], size=6))
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (dy @ mlp.forward(pp, feat, rounding=False)[0] - dy @ mlp.forward(pm, feat, rounding=False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    assert g[offs[0] + 9 * 16 + 13] == 0.0


def test_rounded_gradient_close_to_exact():
    rng = np.random.default_rng(2)
    p = _rand_params(4)
    feat = rng.normal(size=(64, 16))
    dy = rng.normal(size=64)
    g0 = mlp.backward(mlp.forward(p, feat, rounding=False)[1], dy)
    g1 = mlp.backward(mlp.forward(p, feat, rounding=True)[1], dy)
    # rounding moves pre-activations by ~2^-9 of their size; the few ReLU masks
    # that flip change whole gradient entries, so the norm moves by a few percent
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 0.1
    assert not np.array_equal(g0, g1)


def test_relu_network_positively_homogeneous():
    rng = np.random.default_rng(3)
    P = mlp.unpack(mlp.init_params(5).astype(np.float64))
    feat = rng.normal(size=(9, 16))
    p = mlp.pack(P)  # biases are zero after init
    y1 = mlp.forward(p, feat, rounding=False)[0]
    y2 = mlp.forward(p, 2.5 * feat, rounding=False)[0]
    assert np.allclose(y2, 2.5 * y1, rtol=1e-13, atol=1e-13)


def test_one_hidden_layer_special_case_by_loops():
    """W2 = W3 = identity and b2 = b3 = 0 leave relu(W1 x + b1); compare with loops."""
    rng = np.random.default_rng(4)
    P = mlp.unpack(_rand_params(6))
    P["W2"][...] = np.eye(256)
    P["W3"][...] = np.eye(256)
    P["b2"][...] = 0.0
    P["b3"][...] = 0.0
    feat = rng.normal(size=(3, 16))
    y = mlp.forward(mlp.pack(P), feat, rounding=False)[0]
    for r in range(3):
        acc = P["b4"][0]
        for o in range(256):
            z = P["b1"][o]
            for i in range(12):
                z += P["W1"][o, i] * feat[r, i]
            acc += P["W4"][o] * (z if z > 0 else 0.0)
        assert abs(acc - y[r]) < 1e-12 * max(1.0, abs(acc))


def test_mse_derivative():
    rng = np.random.default_rng(5)
    y, t = rng.normal(size=11), rng.normal(size=11)
    loss, dy = mlp.mse(y, t)
    assert abs(loss - np.mean((y - t) ** 2)) < 1e-15
    h = 1e-6
    for i in range(11):
        yp, ym = y.copy(), y.copy()
        yp[i] += h
        ym[i] -= h
        assert abs((mlp.mse(yp, t)[0] - mlp.mse(ym, t)[0]) / (2 * h) - dy[i]) < 1e-8


def test_adam_first_step_closed_form_and_convergence():
    rng = np.random.default_rng(6)
    g = rng.normal(size=50)
    p0 = rng.normal(size=50)
    p1, m, v = mlp.adam(p0, g, np.zeros(50), np.zeros(50), 1, lr=1e-2, eps=1e-8)
    # with zero moments the bias-corrected step is lr * g / (|g| + eps)
    assert np.allclose(p1, p0 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # minimise 0.5 (p - 3)^2
    p, m, v = np.array([0.0]), np.zeros(1), np.zeros(1)
    for t in range(1, 3001):
        p, m, v = mlp.adam(p, p - 3.0, m, v, t, lr=0.05)
    assert abs(p[0] - 3.0) < 1e-3


def test_features_invariants():
    import synth
    xyz, tri = synth.icosphere(2)
    ns = tri.shape[0]
    rng = np.random.default_rng(7)
    hist = rng.normal(size=(8, ns))
    b = rng.normal(size=ns)
    diag = rng.uniform(0.5, 2.0, size=ns)
    f, s = mlp.features(hist, 6, b, diag, xyz, tri)
    assert f.shape == (ns, 16) and np.all(f[:, 12:] == 0.0)
    # s is the RMS of the last four rows and of b / diag together
    assert abs(s - np.sqrt((np.sum(hist[2:6] ** 2) + np.sum((b / diag) ** 2)) / (5 * ns))) < 1e-14 * s
    # densities and rhs scale together; geometry does not
    f2, s2 = mlp.features(3.0 * hist, 6, 3.0 * b, diag, xyz, tri)
    assert abs(s2 - 3.0 * s) < 1e-12 * s and np.allclose(f2, f, rtol=1e-13, atol=1e-13)
    # backward differences: a quadratic history has zero third difference and its
    # extrapolation is exact, so b / diag - e is b / diag - (the next quadratic value)
    t = np.arange(8, dtype=np.float64)[:, None]
    quad = (1.0 + 0.5 * t - 0.25 * t * t) * rng.normal(size=ns)
    fq, sq = mlp.features(quad, 6, b, diag, xyz, tri)
    assert np.allclose(fq[:, 0] * sq, quad[5]) and np.allclose(fq[:, 1] * sq, quad[5] - quad[4])
    assert np.allclose(fq[:, 2] * sq, quad[5] - 2 * quad[4] + quad[3])
    assert np.allclose(fq[:, 3], 0.0, atol=1e-12)
    assert np.allclose(fq[:, 4] * sq, b / diag - quad[6])
    # outward unit normals on a sphere, areas near the equilateral value, centroids inside
    n = f[:, 5:8]
    xc = f[:, 9:12]
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0) and np.all(np.sum(n * xc, axis=1) > 0)
    assert 0.3 < np.mean(f[:, 8]) < 0.5 and np.all(np.linalg.norm(xc, axis=1) <= 1.0)
    # zero history and rhs: all density inputs vanish
    fz, sz = mlp.features(0 * hist, 6, 0 * b, diag, xyz, tri)
    assert sz == 0.0 and np.all(fz[:, :5] == 0.0)


def test_guess_inverts_target():
    rng = np.random.default_rng(8)
    xp, xn = rng.normal(size=20), rng.normal(size=20)
    t = mlp.target(xn, xp, 0.7)
    assert np.allclose(mlp.guess(xp, 0.7, t), xn, rtol=1e-15, atol=1e-15)
    y = t.copy()
    y[3] = np.nan
    g = mlp.guess(xp, 0.7, y)
    assert g[3] == xp[3]


def test_extrapolation_exact_on_quadratics_only():
    t = np.arange(10, dtype=np.float64)[:, None]
    rng = np.random.default_rng(9)
    a, b, c = rng.normal(size=(3, 5))
    q = a + b * t + c * t * t
    for beta in range(3, 10):
        assert np.allclose(mlp.extrapolate(q, beta), q[beta], rtol=1e-13, atol=1e-12)
    cub = t ** 3 * np.ones(5)
    # third difference of t^3 is 6: the parabola through three points misses by exactly 6
    assert np.allclose(cub[6] - mlp.extrapolate(cub, 6), 6.0)


# Planted mistakes: each must make one of the pins above fail.
def _plant_bf16_truncates(mp):
    def trunc(x):
        m, e = np.frexp(np.asarray(x, dtype=np.float64))
        return np.ldexp(np.trunc(m * 256.0), e - 8)
    mp.setattr(mlp, "bf16", trunc)


def _plant_bf16_ties_away(mp):
    def away(x):
        m, e = np.frexp(np.asarray(x, dtype=np.float64))
        return np.ldexp(np.sign(m) * np.floor(np.abs(m) * 256.0 + 0.5), e - 8)
    mp.setattr(mlp, "bf16", away)


def _plant_backward_untransposed(mp):
    orig = mlp.backward

    def bwd(cache, dy):
        r = cache["r"]
        flip = lambda v: r(v).T if np.ndim(v) == 2 and v.shape[0] == v.shape[1] else r(v)
        return orig({**cache, "r": flip}, dy)
    mp.setattr(mlp, "backward", bwd)


def _plant_backward_without_relu_masks(mp):
    orig = mlp.backward

    def bwd(cache, dy):
        return orig({**cache, **{k: np.ones_like(cache[k]) for k in ("z1", "z2", "z3")}}, dy)
    mp.setattr(mlp, "backward", bwd)


def _plant_output_bias_dropped(mp):
    orig = mlp.forward

    def fwd(p, feat, rounding=True):
        y, cache = orig(p, feat, rounding)
        return y - mlp.unpack(np.asarray(p, dtype=np.float64))["b4"][0], cache
    mp.setattr(mlp, "forward", fwd)


def _plant_mse_half_derivative(mp):
    orig = mlp.mse
    mp.setattr(mlp, "mse", lambda y, t: (orig(y, t)[0], orig(y, t)[1] / 2))


def _plant_adam_without_bias_correction(mp):
    orig = mlp.adam
    mp.setattr(mlp, "adam", lambda p, g, m, v, t, lr, **kw: orig(p, g, m, v, 10 ** 9, lr, **kw))


@pytest.mark.parametrize("plant,pin", [
    (_plant_bf16_truncates, test_bf16_matches_torch_conversion),
    (_plant_bf16_ties_away, test_bf16_ties_to_even),
    (_plant_backward_untransposed, test_backward_matches_finite_differences),
    (_plant_backward_without_relu_masks, test_backward_matches_finite_differences),
    (_plant_output_bias_dropped, test_one_hidden_layer_special_case_by_loops),
    (_plant_mse_half_derivative, test_mse_derivative),
    (_plant_adam_without_bias_correction, test_adam_first_step_closed_form_and_convergence),
])
def test_planted_mistakes_fail_a_pin(monkeypatch, plant, pin):
    pin()
    plant(monkeypatch)
    with pytest.raises(AssertionError):
        pin()
