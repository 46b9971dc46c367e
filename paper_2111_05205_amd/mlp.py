"""Learned initial guess of the per-step solve: Python side of the library's
network kernels (argument marshalling) and the training harness.

The network, its parameter layout and features are described in
include/tdbem.h.  All arithmetic (forward, backward, loss, optimiser, features,
targets) runs in libtdbem.so; this module allocates device buffers, draws the
training batches and loops.

    params = init_params(seed)
    feat, target = generate(runs)           # solver-generated (features, targets)
    params, losses = train(feat, target, steps=..., batch=...)
    tdbem.mlp_load(params); TDBEM(..., guess=GUESS_MLP)
"""
import ctypes
import math

import numpy as np

from . import _native as N

NPARAM = N.MLP_NPARAM
IN_PAD = N.MLP_IN_PAD
WIDTH = N.MLP_WIDTH


def _torch():
    import torch
    return torch


def _fptr(t, n=None, name="array", dtype=None):
    """Device pointer of a contiguous float32 (or dtype) CUDA tensor; None -> NULL."""
    if t is None:
        return None
    torch = _torch()
    dt = torch.float32 if dtype is None else dtype
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dt or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dt} CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(t):
    return ctypes.c_void_p(_torch().cuda.current_stream(t.device).cuda_stream)


def _check(rc):
    if rc < 0:
        from . import TDBEMError
        raise TDBEMError(rc, N.lib().tdbem_last_error(None).decode())


def init_params(seed=0, device="cuda"):
    """He-normal weights, zero biases and padding (packed FP32 vector on the device)."""
    torch = _torch()
    g = torch.Generator().manual_seed(int(seed))
    blocks = [torch.zeros(WIDTH, IN_PAD)]
    blocks[0][:, :N.MLP_IN] = torch.randn(WIDTH, N.MLP_IN, generator=g, dtype=torch.float64) * math.sqrt(2.0 / N.MLP_IN)
    blocks.append(torch.zeros(WIDTH))
    for _ in range(2):
        blocks.append(torch.randn(WIDTH, WIDTH, generator=g, dtype=torch.float64) * math.sqrt(2.0 / WIDTH))
        blocks.append(torch.zeros(WIDTH))
    blocks.append(torch.randn(WIDTH, generator=g, dtype=torch.float64) * math.sqrt(1.0 / WIDTH))
    blocks.append(torch.zeros(1))
    p = torch.cat([b.reshape(-1).float() for b in blocks])
    assert p.numel() == NPARAM
    return p.to(device)


def forward(params, feat, act=None):
    """y (n) for feat (n x 16); act: None, True (allocate) or a 3 x n x 256 int16 tensor."""
    torch = _torch()
    n = feat.shape[0]
    y = torch.empty(n, dtype=torch.float32, device=feat.device)
    if act is True:
        act = torch.empty(3, n, WIDTH, dtype=torch.int16, device=feat.device)
    _check(N.lib().tdbem_mlp_forward(_fptr(params, NPARAM, "params"), int(n), _fptr(feat, n * IN_PAD, "feat"),
                                     _fptr(y), _fptr(act, 3 * n * WIDTH, "act", torch.int16), _stream(feat)))
    return (y, act) if act is not None else y


def backward(params, feat, act, dy, work=None):
    """Gradient (NPARAM floats) of sum dy * y."""
    torch = _torch()
    n = feat.shape[0]
    need = int(N.lib().tdbem_mlp_workspace_floats(int(n)))
    if work is None or work.numel() < need:
        work = torch.empty(need, dtype=torch.float32, device=feat.device)
    grad = torch.empty(NPARAM, dtype=torch.float32, device=feat.device)
    _check(N.lib().tdbem_mlp_backward(_fptr(params, NPARAM, "params"), int(n), _fptr(feat, n * IN_PAD, "feat"),
                                      _fptr(act, 3 * n * WIDTH, "act", torch.int16), _fptr(dy, n, "dy"),
                                      _fptr(grad), _fptr(work), ctypes.c_size_t(work.numel()), _stream(feat)))
    return grad


def backward_noalloc(params, feat, act, dy, grad=None):
    """The same gradient through the entry point that allocates nothing (library scratch)."""
    torch = _torch()
    n = feat.shape[0]
    if grad is None:
        grad = torch.empty(NPARAM, dtype=torch.float32, device=feat.device)
    _check(N.lib().tdbem_mlp_backward_noalloc(_fptr(params, NPARAM, "params"), int(n),
                                              _fptr(feat, n * IN_PAD, "feat"),
                                              _fptr(act, 3 * n * WIDTH, "act", torch.int16), _fptr(dy, n, "dy"),
                                              _fptr(grad, NPARAM, "grad"), _stream(feat)))
    return grad


def mse(y, t):
    """(loss tensor of 1 element, dy)."""
    torch = _torch()
    n = y.numel()
    dy = torch.empty_like(y)
    loss = torch.empty(1, dtype=torch.float32, device=y.device)
    _check(N.lib().tdbem_mlp_mse(int(n), _fptr(y), _fptr(t, n, "t"), _fptr(dy), _fptr(loss), _stream(y)))
    return loss, dy


class Adam:
    """Adam state (first/second moments) of one packed parameter vector."""

    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        torch = _torch()
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.t = 0
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps

    def step(self, params, grad, lr=None):
        self.t += 1
        _check(N.lib().tdbem_mlp_adam_step(_fptr(params, NPARAM, "params"), _fptr(grad, NPARAM, "grad"),
                                           _fptr(self.m), _fptr(self.v), int(self.t),
                                           float(self.lr if lr is None else lr), float(self.beta1),
                                           float(self.beta2), float(self.eps), _stream(params)))


# ---------------------------------------------------------------------------
# Training data and training loop


def training_shapes(n_runs, seed=1000, freq_range=(10, 31)):
    """Seeded random ellipsoids: geodesic frequency uniform in freq_range
    (Ns = 20 freq^2), semi-axes uniform in [0.5, 2], incident direction per run."""
    import synth
    out = []
    for r in range(n_runs):
        rng = np.random.default_rng(seed + r)
        freq = int(rng.integers(freq_range[0], freq_range[1] + 1))
        axes = rng.uniform(0.5, 2.0, size=3)
        xyz, tri = synth.ellipsoid(freq, axes)
        out.append({"xyz": xyz, "tri": tri, "seed": seed + r, "freq": freq, "axes": axes})
    return out


def make_solver(xyz, tri, d=2, bie=1, bc=1, nt=256, p=4, guess=N.GUESS_EXTRAP, gmres_tol=1e-8, m2l_prec=0):
    """FMM context with the deepest octree the time step allows (dt = mean edge / c, c = 1)."""
    import synth
    from . import create_fmm
    dt = synth.mean_edge_length(xyz, tri)
    return create_fmm(xyz, tri, 1.0, dt, d, bie, bc, p_s=p, p_t=p, nt_max=nt, gmres_tol=gmres_tol, guess=guess,
                      m2l_prec=m2l_prec), dt


def generate(shapes, nt=256, rows_per_run=None, seed=0, verbose=False, **solver_kw):
    """March each shape under its incident pulse while recording features and
    targets; returns (feat (N x 16), target (N)) float32 device tensors, with
    rows_per_run seeded rows kept per run (all when None)."""
    import synth
    torch = _torch()
    feats, targets = [], []
    for k, s in enumerate(shapes):
        solver, dt = make_solver(s["xyz"], s["tri"], nt=nt, **solver_kw)
        ns = solver.ns
        fb = torch.zeros(nt * ns * IN_PAD, dtype=torch.float32, device="cuda")
        tb = torch.zeros(nt * ns, dtype=torch.float32, device="cuda")
        solver.mlp_record(fb, tb)
        inc = synth.incident_params(s["xyz"], seed=s["seed"])
        solver.run(nt, inc=inc)
        solver.mlp_record()
        f = fb.view(nt, ns, IN_PAD)[4:nt - 1].reshape(-1, IN_PAD)
        t = tb.view(nt, ns)[4:nt - 1].reshape(-1)
        if rows_per_run is not None and rows_per_run < t.numel():
            g = torch.Generator(device="cpu").manual_seed(seed + k)
            idx = torch.randperm(t.numel(), generator=g)[:rows_per_run].to(f.device)
            f, t = f[idx], t[idx]
        feats.append(f.contiguous())
        targets.append(t.contiguous())
        if verbose:
            print(f"run {k}: ns={ns} depth={solver.info()['depth']} rows={t.numel()}", flush=True)
        solver.close()
        del fb, tb
    return torch.cat(feats).contiguous(), torch.cat(targets).contiguous()


def train(feat, target, steps=2000, batch=8192, lr=1e-3, lr_final=1e-4, seed=0, params=None, log_every=0):
    """Adam on the mean squared error of seeded mini-batches, learning rate
    decayed geometrically from lr to lr_final.  Returns (params, losses)."""
    torch = _torch()
    params = init_params(seed) if params is None else params.clone()
    opt = Adam(params, lr=lr)
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = target.numel()
    work = None
    losses = []
    for it in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=g).to(feat.device)
        fb, tb = feat[idx].contiguous(), target[idx].contiguous()
        y, act = forward(params, fb, act=True)
        loss, dy = mse(y, tb)
        if work is None:
            work = torch.empty(int(N.lib().tdbem_mlp_workspace_floats(int(fb.shape[0]))), dtype=torch.float32,
                               device=feat.device)
        grad = backward(params, fb, act, dy, work)
        opt.step(params, grad, lr * (lr_final / lr) ** (it / max(steps - 1, 1)))
        losses.append(float(loss.item()) if (log_every and it % log_every == 0) or it == steps - 1 else None)
    return params, losses


def evaluate(params, xyz, tri, nt, inc, modes=("ZERO", "PREV", "EXTRAP", "MLP"), **solver_kw):
    """GMRES iterations of one march per starting-point mode (same solution for
    every mode): {mode: {total, per_step_mean, per_step_max, rejected, march_ms}}."""
    torch = _torch()
    out = {}
    ref = None
    for mode in modes:
        solver, _ = make_solver(xyz, tri, nt=nt, guess=getattr(N, "GUESS_" + mode), **solver_kw)
        if mode in ("MLP", "MLP_ONLY"):
            solver.mlp_load(params)
        x, ri = solver.run(nt, inc=inc)
        it = ri["total_iters"]
        out[mode] = {"total": it, "per_step_mean": it / ri["steps"], "per_step_max": ri["max_iters"],
                     "rejected": ri["guesses_rejected"], "replaced": ri["guesses_replaced"],
                     "march_ms": round(ri["march_ms"], 1),
                     "ns": solver.ns, "depth": solver.info()["depth"]}
        if ref is None:
            ref = x
        else:
            out[mode]["rel_diff_vs_first"] = float(torch.linalg.norm(x - ref) / torch.linalg.norm(ref))
        solver.close()
    return out


def save(params, path):
    np.save(path, params.detach().cpu().numpy().astype(np.float32))


def load(path, device="cuda"):
    torch = _torch()
    a = np.load(path, allow_pickle=False)
    if a.dtype != np.float32 or a.size != NPARAM:
        raise ValueError(f"{path}: expected {NPARAM} float32 parameters")
    return torch.from_numpy(a).to(device)


def main():
    """Train the guess network on solver-generated runs and write its parameters.

        python -m paper_2111_05205_amd.mlp --runs 40 --steps 3000 --out weights.npy
    """
    import argparse
    import json
    import time
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", type=int, default=40)
    ap.add_argument("--freq-min", type=int, default=10)
    ap.add_argument("--freq-max", type=int, default=31)
    ap.add_argument("--nt", type=int, default=256)
    ap.add_argument("--rows-per-run", type=int, default=200000)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=1e-5)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--out", default="")
    ap.add_argument("--params", default="", help="evaluate these parameters (.npy) instead of training")
    ap.add_argument("--eval", default="", help="comma list of evaluation meshes: icoL<level>:<nt>")
    ap.add_argument("--gmres-tol", type=float, default=1e-8)
    a = ap.parse_args()
    if a.params:
        params = load(a.params)
    else:
        t0 = time.time()
        shapes = training_shapes(a.runs, seed=a.seed, freq_range=(a.freq_min, a.freq_max))
        feat, target = generate(shapes, nt=a.nt, rows_per_run=a.rows_per_run, verbose=True, gmres_tol=a.gmres_tol)
        t1 = time.time()
        print(json.dumps({"runs": a.runs, "rows": int(target.numel()), "generate_s": round(t1 - t0, 1)}), flush=True)
        params, losses = train(feat, target, steps=a.steps, batch=a.batch, lr=a.lr, lr_final=a.lr_final,
                               log_every=max(a.steps // 20, 1))
        del feat, target
        t2 = time.time()
        print(json.dumps({"train_s": round(t2 - t1, 1), "loss": [x for x in losses if x is not None]}), flush=True)
        save(params, a.out)
    import synth
    for spec in filter(None, a.eval.split(",")):
        mesh, nt = spec.split(":")
        xyz, tri = synth.icosphere(int(mesh[4:]))
        inc = synth.incident_params(xyz, seed=0)
        t3 = time.time()
        res = evaluate(params, xyz, tri, int(nt), inc, gmres_tol=a.gmres_tol)
        print(json.dumps({"eval": spec, "gmres_tol": a.gmres_tol, "seconds": round(time.time() - t3, 1),
                          "iterations": res}), flush=True)


if __name__ == "__main__":
    main()
