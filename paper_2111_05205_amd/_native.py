"""ctypes declarations of the C ABI in include/tdbem.h (argument marshalling only)."""
import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtdbem.so")

OK, E_INVAL, E_NOMEM, E_DEVICE, E_NOT_CONVERGED, E_DIVERGED, E_STATE = 0, -1, -2, -3, -4, -5, -6
OBIE, BMBIE = 0, 1
DIRICHLET, NEUMANN, MIXED = 0, 1, 2
M2L_FP64, M2L_FP32, M2L_BF16, M2L_BF16X3 = 0, 1, 2, 3
INTERP_LAGRANGE, INTERP_HERMITE = 0, 1
INC_GAUSS_MOD, INC_RAISED_COS = 0, 1
GUESS_EXTRAP, GUESS_ZERO, GUESS_PREV, GUESS_MLP, GUESS_MLP_ONLY = 0, 1, 2, 3, 4
MLP_IN, MLP_IN_PAD, MLP_WIDTH, MLP_NPARAM = 12, 16, 256, 136193
MLP_NOALLOC_MAX_ROWS = 8192


class Mesh(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("xyz", ctypes.POINTER(ctypes.c_double)), ("tri", ctypes.POINTER(ctypes.c_int32))]


class Opts(ctypes.Structure):
    _fields_ = [("use_fmm", ctypes.c_int), ("depth", ctypes.c_int), ("p_s", ctypes.c_int), ("p_t", ctypes.c_int),
                ("mu", ctypes.c_int), ("m2l_prec", ctypes.c_int), ("gmres_tol", ctypes.c_double),
                ("gmres_restart", ctypes.c_int), ("gmres_maxiter", ctypes.c_int), ("nt_max", ctypes.c_int),
                ("guess", ctypes.c_int), ("graph", ctypes.c_int), ("near_form", ctypes.c_int),
                ("near_prec", ctypes.c_int), ("interp", ctypes.c_int), ("growth_limit", ctypes.c_double),
                ("growth_lag", ctypes.c_int), ("leaf_ratio", ctypes.c_double)]


class Incident(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("dir", ctypes.c_double * 3), ("f0", ctypes.c_double),
                ("sigma", ctypes.c_double), ("t0", ctypes.c_double), ("rb", ctypes.c_double)]


class StepInfo(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_int), ("iters", ctypes.c_int), ("resid", ctypes.c_double)]


class RunInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("total_iters", ctypes.c_int), ("max_iters", ctypes.c_int),
                ("max_resid", ctypes.c_double), ("march_ms", ctypes.c_double), ("guesses_rejected", ctypes.c_int),
                ("guesses_replaced", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("ns", ctypes.c_int), ("d", ctypes.c_int), ("bie", ctypes.c_int), ("bc", ctypes.c_int),
                ("c", ctypes.c_double), ("dt", ctypes.c_double), ("use_fmm", ctypes.c_int), ("depth", ctypes.c_int),
                ("p_s", ctypes.c_int), ("p_t", ctypes.c_int), ("mu", ctypes.c_int), ("m_leaf", ctypes.c_int),
                ("near_pairs", ctypes.c_int64), ("near_coefs", ctypes.c_int64), ("a_nnz", ctypes.c_int64),
                ("il_pairs", ctypes.c_int64 * 16), ("m2l_matrix_bytes", ctypes.c_int64), ("setup_ms", ctypes.c_double),
                ("m2l_variant", ctypes.c_int * 16), ("gmres_workgroups", ctypes.c_int),
                ("m2l_dense_blocks", ctypes.c_int64 * 16), ("m2l_ops_users", ctypes.c_int * 16)]


PROF_KINDS = ["near_history", "gmres", "l2p", "p2m", "m2l_gemm", "m2l_reduce", "m2m", "l2l", "other", "mlp",
              "m2l_deriv"]

_lib = None


def lib():
    """Load libtdbem.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc, gfx950); the library has no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
        L.tdbem_create.argtypes = [ctypes.POINTER(Mesh), ctypes.c_double, ctypes.c_double, ip, ip, ip,
                                   ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
        L.tdbem_create_mixed.argtypes = [ctypes.POINTER(Mesh), ctypes.c_double, ctypes.c_double, ip, ip,
                                         ctypes.POINTER(ctypes.c_int8), ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
        L.tdbem_field.argtypes = [vp, ip, dp, ip, vp]
        L.tdbem_direct_rows.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_int32), ip, vp]
        L.tdbem_destroy.argtypes = [vp]
        L.tdbem_destroy.restype = None
        L.tdbem_last_error.argtypes = [vp]
        L.tdbem_last_error.restype = ctypes.c_char_p
        L.tdbem_get_info.argtypes = [vp, ctypes.POINTER(Info)]
        L.tdbem_reset.argtypes = [vp]
        L.tdbem_set_history.argtypes = [vp, ip, vp, vp]
        L.tdbem_fmm_eval.argtypes = [vp, ip, vp]
        L.tdbem_step.argtypes = [vp, vp, vp, vp, ctypes.POINTER(StepInfo)]
        L.tdbem_run.argtypes = [vp, ip, vp, ctypes.POINTER(Incident), vp, ctypes.POINTER(RunInfo)]
        L.tdbem_get_history.argtypes = [vp, ip, vp, vp]
        L.tdbem_incident_forcing.argtypes = [vp, ctypes.POINTER(Incident), ip, ip, vp]
        L.tdbem_near_row.argtypes = [vp, ip, ip, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                     dp, dp]
        L.tdbem_profile.argtypes = [vp, ip]
        L.tdbem_profile_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int64), ip]
        L.tdbem_profile_mask.argtypes = [vp, ctypes.c_uint]
        L.tdbem_set_m2l_variant.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        L.tdbem_mlp_forward.argtypes = [vp, ip, vp, vp, vp, vp]
        L.tdbem_mlp_forward_loaded.argtypes = [vp, ip, vp, vp]
        L.tdbem_mlp_workspace_floats.argtypes = [ip]
        L.tdbem_mlp_workspace_floats.restype = ctypes.c_size_t
        L.tdbem_mlp_backward.argtypes = [vp, ip, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
        L.tdbem_mlp_backward_noalloc.argtypes = [vp, ip, vp, vp, vp, vp, vp]
        L.tdbem_mlp_mse.argtypes = [ip, vp, vp, vp, vp, vp]
        L.tdbem_mlp_adam_step.argtypes = [vp, vp, vp, vp, ip, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_float, vp]
        L.tdbem_run_batch.argtypes = [ctypes.POINTER(vp), ip, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(Incident),
                                      ctypes.POINTER(vp), ctypes.POINTER(RunInfo), dp]
        L.tdbem_checkpoint.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_size_t)]
        L.tdbem_restore.argtypes = [vp, vp, ctypes.c_size_t]
        L.tdbem_mlp_load.argtypes = [vp, vp]
        L.tdbem_mlp_record.argtypes = [vp, vp, vp]
        _lib = L
    return _lib
