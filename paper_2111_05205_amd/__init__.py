"""MI355X time-domain boundary element method (Burton-Miller / ordinary BIE,
B-spline time basis, interpolation-based space-time FMM) — Python binding.

Every computation runs in the HIP library libtdbem.so behind the C ABI of
include/tdbem.h; this module only marshals arguments.  Device arrays are
torch float64 CUDA (HIP) tensors; the library works on the current torch
stream of the tensors' device.
"""
import ctypes
import sys

import numpy as np

from . import _native as N
from ._native import (BMBIE, DIRICHLET, MIXED, GUESS_EXTRAP, GUESS_MLP, GUESS_MLP_ONLY, GUESS_PREV, GUESS_ZERO, INC_GAUSS_MOD,
                      INC_RAISED_COS, INTERP_HERMITE, INTERP_LAGRANGE, M2L_BF16, M2L_BF16X3, M2L_FP32, M2L_FP64, NEUMANN,
                      OBIE)

__all__ = ["TDBEM", "TDBEMError", "incident", "run_batch", "create_fmm", "BMBIE", "OBIE", "DIRICHLET", "NEUMANN", "MIXED", "M2L_FP64", "M2L_FP32", "M2L_BF16", "M2L_BF16X3",
           "INC_GAUSS_MOD", "INC_RAISED_COS", "GUESS_EXTRAP", "GUESS_ZERO", "GUESS_PREV", "GUESS_MLP", "GUESS_MLP_ONLY",
           "INTERP_LAGRANGE", "INTERP_HERMITE"]


class TDBEMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tdbem error {code}: {msg}")
        self.code = code


def _torch():
    import torch
    return torch


def _dptr(t, n=None, name="array"):
    """Device pointer of a contiguous float64 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def incident(inc: dict):
    """tdbem_incident from a dict with keys kind ('gauss_mod'|'raised_cos'), dir, f0, sigma, t0, rb."""
    s = N.Incident()
    s.kind = INC_GAUSS_MOD if inc["kind"] == "gauss_mod" else INC_RAISED_COS
    for k in range(3):
        s.dir[k] = float(inc["dir"][k])
    s.f0, s.sigma, s.t0, s.rb = float(inc.get("f0", 1.0)), float(inc["sigma"]), float(inc.get("t0", 0.0)), \
        float(inc.get("rb", 0.0))
    return s


def create_fmm(xyz, tri, c, dt, d, bie=BMBIE, bc=NEUMANN, max_depth=7, **kw):
    """FMM context with the deepest octree (<= max_depth) whose leaves are wide
    enough for the time step (M_leaf >= 1); other options as for TDBEM."""
    last = None
    for depth in range(max_depth, 1, -1):
        try:
            return TDBEM(xyz, tri, c, dt, d, bie, bc, use_fmm=1, depth=depth, **kw)
        except TDBEMError as e:
            if e.code != N.E_INVAL:
                raise
            last = e
    raise last


def run_batch(solvers, nts, incs=None, out=True):
    """March several contexts together (tdbem_run_batch).  nts: steps per context;
    incs: incident dicts (or None for zero forcing).  Returns (histories or None,
    per-context run info dicts, wall milliseconds)."""
    torch = _torch()
    n = len(solvers)
    L = N.lib()
    ctxs = (ctypes.c_void_p * n)(*[s._h for s in solvers])
    nt_arr = (ctypes.c_int * n)(*[int(x) for x in nts])
    inc_arr = None
    if incs is not None:
        inc_arr = (N.Incident * n)(*[incident(x) for x in incs])
    outs = None
    out_arr = None
    if out:
        outs = [torch.empty(int(nts[i]) - 1, s.ns, dtype=torch.float64, device=s.device) for i, s in enumerate(solvers)]
        out_arr = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
    infos = (N.RunInfo * n)()
    wall = ctypes.c_double(0.0)
    rc = L.tdbem_run_batch(ctxs, n, nt_arr, inc_arr, out_arr, infos, ctypes.byref(wall))
    if rc < 0:
        msgs = [L.tdbem_last_error(s._h).decode() for s in solvers]
        raise TDBEMError(rc, "; ".join(m for m in msgs if m) or L.tdbem_last_error(None).decode())
    return outs, [{k: getattr(r, k) for k, _ in N.RunInfo._fields_} for r in infos], wall.value


class TDBEM:
    """One scatterer: a context of the HIP library (tdbem_create ... tdbem_destroy)."""

    def __init__(self, xyz, tri, c, dt, d, bie=BMBIE, bc=NEUMANN, *, use_fmm=0, depth=4, p_s=4, p_t=4, mu=0,
                 m2l_prec=M2L_FP64, gmres_tol=1e-12, gmres_restart=30, gmres_maxiter=300, nt_max=4096,
                 guess=GUESS_EXTRAP, graph=False, stream=None, device=None, face_bc=None, near_form=0,
                 near_prec=0, interp=0, growth_limit=0.0, growth_lag=1, leaf_ratio=0.0):
        """face_bc: None, or per face 1 (q given, u unknown) / 0 (u given, q unknown): a mixed
        boundary condition (tdbem_create_mixed; bc is then ignored)."""
        torch = _torch()
        self._L = N.lib()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        mesh = N.Mesh(xyz.shape[0], tri.shape[0], xyz.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      tri.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        o = N.Opts(int(use_fmm), int(depth), int(p_s), int(p_t), int(mu), int(m2l_prec), float(gmres_tol),
                   int(gmres_restart), int(gmres_maxiter), int(nt_max), int(guess), int(bool(graph)),
                   int(near_form), int(near_prec), int(interp), float(growth_limit), int(growth_lag),
                   float(leaf_ratio))
        self.stream = stream  # a torch.cuda.Stream the context works on (kept alive), or None
        if stream is not None:
            stream = stream.cuda_stream
        else:
            with torch.cuda.device(self.device):
                stream = torch.cuda.current_stream(self.device).cuda_stream
        h = ctypes.c_void_p()
        if face_bc is not None:
            fb = np.ascontiguousarray(face_bc, dtype=np.int8)
            if fb.shape != (tri.shape[0],):
                raise ValueError("face_bc must have one value per triangle")
            rc = self._L.tdbem_create_mixed(ctypes.byref(mesh), float(c), float(dt), int(d), int(bie),
                                            fb.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), ctypes.byref(o),
                                            ctypes.c_void_p(stream), ctypes.byref(h))
        else:
            rc = self._L.tdbem_create(ctypes.byref(mesh), float(c), float(dt), int(d), int(bie), int(bc),
                                      ctypes.byref(o), ctypes.c_void_p(stream), ctypes.byref(h))
        if rc != N.OK:
            raise TDBEMError(rc, self._L.tdbem_last_error(None).decode())
        self._h = h
        inf = self.info()
        self.ns = inf["ns"]
        self.nt_max = int(nt_max)

    def close(self):
        if getattr(self, "_h", None):
            self._L.tdbem_destroy(self._h)
            self._h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter shutdown the HIP runtime may already be finalising: leave the
        # device memory to the process exit instead of calling into it
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        """Message of the context's last failed call (tdbem_last_error)."""
        return self._L.tdbem_last_error(self._h).decode()

    def _check(self, rc):
        if rc < 0:
            raise TDBEMError(rc, self._L.tdbem_last_error(self._h).decode())
        return rc

    def _empty(self, *shape):
        torch = _torch()
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def info(self):
        i = N.Info()
        self._check(self._L.tdbem_get_info(self._h, ctypes.byref(i)))
        out = {k: getattr(i, k) for k, _ in N.Info._fields_}
        out["il_pairs"] = list(i.il_pairs)
        out["m2l_variant"] = list(i.m2l_variant)
        out["m2l_dense_blocks"] = list(i.m2l_dense_blocks)
        out["m2l_ops_users"] = list(i.m2l_ops_users)
        return out

    def reset(self):
        self._check(self._L.tdbem_reset(self._h))

    def set_history(self, u=None, q=None):
        nsteps = 0 if u is None and q is None else (u if u is not None else q).shape[0]
        self._check(self._L.tdbem_set_history(self._h, nsteps, _dptr(u, nsteps * self.ns, "u"),
                                              _dptr(q, nsteps * self.ns, "q")))

    def get_history(self, nsteps):
        u, q = self._empty(nsteps, self.ns), self._empty(nsteps, self.ns)
        self._check(self._L.tdbem_get_history(self._h, nsteps, _dptr(u), _dptr(q)))
        return u, q

    def fmm_eval(self, alpha, out=None):
        out = self._empty(self.ns) if out is None else out
        self._check(self._L.tdbem_fmm_eval(self._h, int(alpha), _dptr(out, self.ns, "out")))
        return out

    def step(self, forcing=None, bc_values=None, out=None, check=True):
        out = self._empty(self.ns) if out is None else out
        si = N.StepInfo()
        rc = self._L.tdbem_step(self._h, _dptr(forcing, self.ns, "forcing"), _dptr(bc_values, self.ns, "bc_values"),
                                _dptr(out, self.ns, "out"), ctypes.byref(si))
        if check:
            self._check(rc)
        return out, {"alpha": si.alpha, "iters": si.iters, "resid": si.resid, "rc": rc}

    def run(self, nt, forcing=None, inc=None, out=None, check=True):
        out = self._empty(nt - 1, self.ns) if out is None else out
        ri = N.RunInfo()
        incs = incident(inc) if isinstance(inc, dict) else inc
        rc = self._L.tdbem_run(self._h, int(nt), _dptr(forcing, (nt - 1) * self.ns, "forcing"),
                               ctypes.byref(incs) if incs is not None else None, _dptr(out, (nt - 1) * self.ns, "out"),
                               ctypes.byref(ri))
        if check:
            self._check(rc)
        return out, {k: getattr(ri, k) for k, _ in N.RunInfo._fields_} | {"rc": rc}

    def field(self, pts, alpha):
        """Scattered field at off-surface points pts (n x 3) and time t_alpha (tdbem_field)."""
        p = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        out = self._empty(p.shape[0])
        self._check(self._L.tdbem_field(self._h, p.shape[0], p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        int(alpha), _dptr(out)))
        return out

    def direct_rows(self, rows, alpha):
        """Exact history part of b^{alpha-1} at the given collocation rows (tdbem_direct_rows)."""
        r = np.ascontiguousarray(rows, dtype=np.int32).reshape(-1)
        out = self._empty(r.shape[0])
        self._check(self._L.tdbem_direct_rows(self._h, r.shape[0], r.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                              int(alpha), _dptr(out)))
        return out

    def incident_forcing(self, inc, a0, n):
        out = self._empty(n, self.ns)
        incs = incident(inc) if isinstance(inc, dict) else inc
        self._check(self._L.tdbem_incident_forcing(self._h, ctypes.byref(incs), int(a0), int(n), _dptr(out)))
        return out

    def set_m2l_variant(self, n, choice):
        """Override the autotuned M2L launch for the n finest levels ending together
        (choice = 2 * tile + persistent, see tdbem_info.m2l_variant)."""
        self._check(self._L.tdbem_set_m2l_variant(self._h, int(n), int(choice)))

    def profile(self, enable=True, kinds=None):
        """Start (clear) or stop per-kernel timing of this context; kinds: None (all)
        or an iterable of category names (see PROF_KINDS) to bracket only those."""
        if kinds is None or not enable:
            self._check(self._L.tdbem_profile(self._h, int(bool(enable))))
        else:
            mask = 0
            for k in kinds:
                mask |= 1 << N.PROF_KINDS.index(k)
            self._check(self._L.tdbem_profile_mask(self._h, mask))

    def profile_read(self):
        """{category: (total ms, launches)} accumulated since profile(True)."""
        n = len(N.PROF_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int64 * n)()
        self._check(self._L.tdbem_profile_read(self._h, ms, cnt, n))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(N.PROF_KINDS)}

    def checkpoint(self):
        """State of the march as bytes (tdbem_checkpoint)."""
        n = ctypes.c_size_t(0)
        self._check(self._L.tdbem_checkpoint(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._check(self._L.tdbem_checkpoint(self._h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    def restore(self, data: bytes):
        """Continue from a checkpoint taken by checkpoint() (tdbem_restore)."""
        buf = ctypes.create_string_buffer(bytes(data), len(data))
        self._check(self._L.tdbem_restore(self._h, buf, len(data)))

    def mlp_load(self, params):
        """Use the network with these packed FP32 parameters (CUDA tensor) when guess=GUESS_MLP."""
        from .mlp import _fptr
        self._check(self._L.tdbem_mlp_load(self._h, _fptr(params, N.MLP_NPARAM, "params")))

    def mlp_forward_loaded(self, feat):
        """y (n) of the installed network for feat (n x 16 float32 CUDA tensor), through the
        march's kernel (pre-packed bf16 fragments); equals mlp.forward of the same parameters."""
        import torch
        from .mlp import _fptr
        n = feat.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=feat.device)
        torch.cuda.synchronize()
        self._check(self._L.tdbem_mlp_forward_loaded(self._h, int(n), _fptr(feat, n * N.MLP_IN_PAD, "feat"),
                                                     _fptr(y)))
        return y

    def mlp_record(self, feat=None, target=None):
        """Record features (nt_max x Ns x 16) and targets (nt_max x Ns), float32 CUDA tensors, during
        later steps (rows beta >= 4); no arguments stops recording."""
        from .mlp import _fptr
        self._rec = (feat, target)  # keep the buffers alive while recorded into
        self._check(self._L.tdbem_mlp_record(self._h, _fptr(feat, self.nt_max * self.ns * N.MLP_IN_PAD, "feat"),
                                             _fptr(target, self.nt_max * self.ns, "target")))

    def near_row(self, i):
        n = self._check(self._L.tdbem_near_row(self._h, int(i), 0, None, None, None, None))
        j = np.zeros(n, dtype=np.int32)
        g = np.zeros(n, dtype=np.int32)
        cu = np.zeros(n)
        cw = np.zeros(n)
        self._check(self._L.tdbem_near_row(self._h, int(i), n, j.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           g.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                           cu.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           cw.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return j, g, cu, cw
