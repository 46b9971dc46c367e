"""ORACLE (test infrastructure): the learned initial guess of the per-step solve, in FP64.

The paper solves one sparse system A x^{alpha-1} = b^{alpha-1} per step (eq.
linear) and names no solver.  The GPU path solves it by GMRES; this module is
the plain definition of the small per-element network that proposes the
starting point of that solve, of its training gradients and of the optimiser,
so that the library's kernels can be compared with it:

* ``bf16``      round-to-nearest-even to bfloat16 (8 significant bits), the
                rounding applied to every weight and every layer input before
                it enters a product;
* ``forward``   12 features -> 3 hidden ReLU layers of width 256 -> 1 output,
                products of bf16-rounded operands summed exactly (FP64);
* ``backward``  reverse-mode derivative of ``forward`` with the rounding
                treated as the identity (straight-through);
* ``mse``       mean squared error and its derivative;
* ``adam``      one step of Adam (Kingma and Ba, 2015) with bias correction;
* ``features``  the per-element inputs and the normalisation of the target;
* ``extrapolate``, ``target``, ``guess``  the network output y corrects the
                quadratic extrapolation of the last three rows: the proposal is
                extrapolation + s y, so y = 0 reproduces the extrapolation.

Parameter vector (FP32 master copy, packed, the layout the C ABI states):
W1 [256][16] (input columns 12..15 are padding), b1 [256], W2 [256][256],
b2 [256], W3 [256][256], b3 [256], W4 [256], b4 [1]; W[o][i] maps input i to
output o.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the HIP library.
"""
import numpy as np

N_IN = 12
N_IN_PAD = 16
WIDTH = 256


def layout():
    """(name, shape) of each parameter block in order."""
    return [("W1", (WIDTH, N_IN_PAD)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
            ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("W4", (WIDTH,)), ("b4", (1,))]


def nparams():
    return sum(int(np.prod(s)) for _, s in layout())


def unpack(p):
    """Views of the packed vector p by block name."""
    out, o = {}, 0
    for name, shape in layout():
        n = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + n]).reshape(shape)
        o += n
    return out


def pack(blocks):
    return np.concatenate([np.asarray(blocks[name], dtype=np.float64).ravel() for name, _ in layout()])


def bf16(x):
    """Round to the nearest bfloat16 value (8 significant bits, ties to even),
    returned in float64.  Normal range only (no subnormal or overflow handling)."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                  # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0), e - 8)


def forward(p, feat, rounding=True):
    """Network output y (n,) for features feat (n, 12 or 16) and the values
    backward needs.  rounding=False gives the same network without bf16
    rounding (used to check the derivative by finite differences)."""
    r = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    P = unpack(np.asarray(p, dtype=np.float64))
    h0 = r(np.asarray(feat, dtype=np.float64)[:, :N_IN])
    z1 = h0 @ r(P["W1"][:, :N_IN]).T + P["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ r(P["W2"]).T + P["b2"]
    h2 = r(np.maximum(z2, 0.0))
    z3 = h2 @ r(P["W3"]).T + P["b3"]
    h3 = r(np.maximum(z3, 0.0))
    y = h3 @ r(P["W4"]) + P["b4"][0]
    cache = {"h0": h0, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "z3": z3, "h3": h3, "P": P, "r": r}
    return y, cache


def backward(cache, dy):
    """Gradient of sum_r dy_r y_r with respect to the packed parameters."""
    P, r = cache["P"], cache["r"]
    dy = np.asarray(dy, dtype=np.float64)
    g = {}
    g["W4"] = cache["h3"].T @ dy
    g["b4"] = np.array([dy.sum()])
    dz3 = np.outer(dy, r(P["W4"])) * (cache["z3"] > 0.0)
    g["W3"] = dz3.T @ cache["h2"]
    g["b3"] = dz3.sum(axis=0)
    dz2 = (dz3 @ r(P["W3"])) * (cache["z2"] > 0.0)
    g["W2"] = dz2.T @ cache["h1"]
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ r(P["W2"])) * (cache["z1"] > 0.0)
    gw1 = np.zeros((WIDTH, N_IN_PAD))
    gw1[:, :N_IN] = dz1.T @ cache["h0"]
    g["W1"] = gw1
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def mse(y, t):
    """Loss (1/n) sum (y - t)^2 and its derivative 2 (y - t) / n."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = max(len(y), 1)
    e = y - t
    return float(e @ e) / n, 2.0 * e / n


def adam(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step number t >= 1; returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed):
    """He-normal weights, zero biases, zero padding columns (FP32 values)."""
    rng = np.random.default_rng(seed)
    b = {}
    b["W1"] = np.zeros((WIDTH, N_IN_PAD))
    b["W1"][:, :N_IN] = rng.normal(size=(WIDTH, N_IN)) * np.sqrt(2.0 / N_IN)
    b["W2"] = rng.normal(size=(WIDTH, WIDTH)) * np.sqrt(2.0 / WIDTH)
    b["W3"] = rng.normal(size=(WIDTH, WIDTH)) * np.sqrt(2.0 / WIDTH)
    b["W4"] = rng.normal(size=WIDTH) * np.sqrt(1.0 / WIDTH)
    for k in ("b1", "b2", "b3"):
        b[k] = np.zeros(WIDTH)
    b["b4"] = np.zeros(1)
    return pack(b).astype(np.float32)


def mesh_scales(xyz, tri):
    """Geometry normalisation: mean edge length h, bounding-box centre and the
    largest vertex distance R from that centre."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(tri)
    e = np.concatenate([np.linalg.norm(xyz[tri[:, a]] - xyz[tri[:, b]], axis=1) for a, b in ((0, 1), (1, 2), (2, 0))])
    cen = 0.5 * (xyz.min(axis=0) + xyz.max(axis=0))
    rad = np.linalg.norm(xyz - cen, axis=1).max()
    return float(e.mean()), cen, float(rad)


def features(hist, beta, b, diag, xyz, tri):
    """Inputs of the guess for unknown row beta (>= 4) and the scale s.

    hist: solved rows (>= beta, ns) of the unknown (u on Neumann faces, q on
    Dirichlet faces); b: right-hand side of step beta; diag: the diagonal of
    the per-step matrix.  With x1..x4 the rows beta-1..beta-4, e the quadratic
    extrapolation 3 x1 - 3 x2 + x3 and s the root mean square of x1..x4 and
    b/diag, the density inputs are the backward differences of the history
    x1, x1 - x2, x1 - 2 x2 + x3, x1 - 3 x2 + 3 x3 - x4 and the Jacobi-scaled
    right-hand side relative to the extrapolation b/diag - e, each divided by
    s; geometry: outward unit normal, area / h^2, (centroid - centre) / R."""
    hist = np.asarray(hist, dtype=np.float64)
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(tri)
    ns = tri.shape[0]
    bj = np.asarray(b, dtype=np.float64) / np.asarray(diag, dtype=np.float64)
    x1, x2, x3, x4 = (hist[beta - k] for k in range(1, 5))
    ssq = sum(float(x @ x) for x in (x1, x2, x3, x4)) + float(bj @ bj)
    s = np.sqrt(ssq / (5.0 * ns))
    inv = 1.0 / s if s > 0.0 else 0.0
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    cr = np.cross(p1 - p0, p2 - p0)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    nout = cr / (2.0 * area[:, None])
    xc = (p0 + p1 + p2) / 3.0
    h, cen, rad = mesh_scales(xyz, tri)
    e = 3.0 * x1 - 3.0 * x2 + x3
    f = np.zeros((ns, N_IN_PAD))
    f[:, 0] = x1 * inv
    f[:, 1] = (x1 - x2) * inv
    f[:, 2] = (x1 - 2.0 * x2 + x3) * inv
    f[:, 3] = (x1 - 3.0 * x2 + 3.0 * x3 - x4) * inv
    f[:, 4] = (bj - e) * inv
    f[:, 5:8] = nout
    f[:, 8] = area / (h * h)
    f[:, 9:12] = (xc - cen) / rad
    return f, s


def extrapolate(hist, beta):
    """Quadratic extrapolation of row beta from rows beta-1, beta-2, beta-3:
    the value at beta of the parabola through them, 3 x1 - 3 x2 + x3."""
    hist = np.asarray(hist, dtype=np.float64)
    return 3.0 * hist[beta - 1] - 3.0 * hist[beta - 2] + hist[beta - 3]


def target(x_new, base, s):
    """Training target: what the extrapolation base misses, divided by s."""
    inv = 1.0 / s if s > 0.0 else 0.0
    return (np.asarray(x_new, dtype=np.float64) - np.asarray(base, dtype=np.float64)) * inv


def guess(base, s, y):
    """Proposed starting point base + s y (base where y is not finite)."""
    y = np.asarray(y, dtype=np.float64)
    return np.where(np.isfinite(y), np.asarray(base, dtype=np.float64) + s * y, base)
