"""ctypes binding of libspfas.so: the C structs of include/spfas.h and the
entry points under the same names.  Argument marshalling only; every step
of the method runs in the library."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspfas.so")

SPFAS_OK, SPFAS_NOT_CONVERGED = 0, 1
SPFAS_ERR_INVALID, SPFAS_ERR_OOM, SPFAS_ERR_DEVICE, SPFAS_ERR_NUMERIC = -1, -2, -3, -4
SPFAS_MEM_HOST, SPFAS_MEM_DEVICE = 0, 1
SPFAS_NEWTON, SPFAS_PICARD = 0, 1
SPFAS_PREC_FP64, SPFAS_PREC_MIXED = 0, 1
SPFAS_AGG_BOX, SPFAS_AGG_USER, SPFAS_AGG_GREEDY = 0, 1, 2
SPFAS_OP_EIGVALS, SPFAS_OP_PP, SPFAS_OP_PSIGMA, SPFAS_OP_MLOC, SPFAS_OP_DLOC, SPFAS_OP_W, SPFAS_OP_QSIGMA, SPFAS_OP_MCOUNT = range(8)

EXPORTED = ["spfas_default_solve_opts", "spfas_setup_hierarchy", "spfas_fas_solve", "spfas_cascadic_solve",
            "spfas_picard_solve", "spfas_newton_solve", "spfas_eval_residual", "spfas_eval_residual_noalloc",
            "spfas_level_sizes", "spfas_hierarchy_device_bytes", "spfas_hierarchy_reset_peak",
            "spfas_get_aggregation",
            "spfas_get_permutation", "spfas_get_level_operator", "spfas_destroy", "spfas_last_error",
            "spfas_version", "spfas_profile_enable", "spfas_profile_read",
            "spfas_server_create", "spfas_server_add_model", "spfas_server_submit", "spfas_server_wait",
            "spfas_server_counters_get", "spfas_server_destroy", "spfas_server_last_error"]
SPFAS_SOLVE_FAS, SPFAS_SOLVE_NEWTON, SPFAS_SOLVE_PICARD = 0, 1, 2
(SPFAS_PROF_FINE_RESID, SPFAS_PROF_FINE_LINEARIZE, SPFAS_PROF_FINE_SPMV, SPFAS_PROF_FINE_AMG_DOWN,
 SPFAS_PROF_FINE_AMG_RESTRICT, SPFAS_PROF_FINE_AMG_UP, SPFAS_PROF_FINE_SPMV2, SPFAS_PROF_FINE_RESID_TRIALS,
 SPFAS_PROF_AMG_TAIL_DOWN, SPFAS_PROF_AMG_TAIL_RESTRICT, SPFAS_PROF_AMG_TAIL_UP) = range(11)
# names match the kernels as a profiler reports them (classical finest AMG level)
PROF_NAMES = {SPFAS_PROF_FINE_RESID: "k_fine_resid", SPFAS_PROF_FINE_LINEARIZE: "k_fine_lin_cells",
              SPFAS_PROF_FINE_SPMV: "k_spmv_dot<true>", SPFAS_PROF_FINE_SPMV2: "k_spmv_dot2<true>",
              SPFAS_PROF_FINE_AMG_DOWN: "k_cyc<0, true>", SPFAS_PROF_FINE_AMG_RESTRICT: "k_cyc<1, true>",
              SPFAS_PROF_FINE_AMG_UP: "k_cyc<2, true>", SPFAS_PROF_FINE_RESID_TRIALS: "k_fine_resid_trials",
              SPFAS_PROF_AMG_TAIL_DOWN: "amg_tail_down", SPFAS_PROF_AMG_TAIL_RESTRICT: "amg_tail_restrict",
              SPFAS_PROF_AMG_TAIL_UP: "amg_tail_up"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class spfas_mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_cells", C.c_int64), ("n_faces", C.c_int64),
                ("cell_volume", _dp), ("cell_centroid", _dp), ("cell_k0", _dp),
                ("face_cells", _ip), ("face_area", _dp), ("face_normal", _dp),
                ("face_point", _dp), ("face_kind", C.POINTER(C.c_int8))]


class spfas_coarsen_opts(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("box", C.c_int32 * 3), ("m", C.c_int32), ("host_only", C.c_int32),
                ("agg_kind", C.c_int32), ("user_agg", _ip), ("user_agg_len", C.c_int64),
                ("greedy_size", C.c_int32), ("eig_threshold", C.c_double), ("m_min", C.c_int32),
                ("m_f", C.c_int32), ("greedy_size_coarse", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


class spfas_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


SPFAS_KAPPA_EXP, SPFAS_KAPPA_RICHARDS = 0, 1
KAPPA_KINDS = {"exp": SPFAS_KAPPA_EXP, "richards": SPFAS_KAPPA_RICHARDS}


class spfas_problem(C.Structure):
    _fields_ = [("alpha", C.c_double), ("source", C.c_void_p), ("g_dirichlet", C.c_void_p),
                ("g_neumann", C.c_void_p), ("mem", C.c_int32), ("kappa_kind", C.c_int32),
                ("kappa_a", C.c_double), ("kappa_beta", C.c_double), ("shift", C.c_void_p)]


class spfas_solve_opts(C.Structure):
    _fields_ = [("smoother", C.c_int32), ("rtol", C.c_double), ("atol", C.c_double), ("max_it", C.c_int32),
                ("bt_nmax", C.c_int32), ("bt_theta", C.c_double), ("dp_cap", C.c_double),
                ("coarsest_max_steps", C.c_int32), ("lin_rtol", C.c_double), ("lin_max_it", C.c_int32),
                ("x0_given", C.c_int32), ("lin_rtol_coarse", C.c_double), ("lin_target", C.c_double),
                ("newton_pcg", C.c_int32), ("amg_reuse", C.c_int32),
                ("lin_max_it_coarse", C.c_int32), ("coarsest_atol", C.c_double), ("precision", C.c_int32)]


class spfas_stats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("lin_iters", C.c_int32), ("bt_halvings", C.c_int32),
                ("smoothing_steps", C.c_int32), ("stopped_after_presmooth", C.c_int32),
                ("r0", C.c_double), ("r_final", C.c_double), ("solve_ms", C.c_double),
                ("rejected_steps", C.c_int32), ("refine_steps", C.c_int32)]


class spfas_server_opts(C.Structure):
    _fields_ = [("n_slots", C.c_int32), ("hbm_budget", C.c_int64), ("device", C.c_int32)]


class spfas_request_info(C.Structure):
    _fields_ = [("queue_ms", C.c_double), ("setup_ms", C.c_double), ("solve_ms", C.c_double),
                ("total_ms", C.c_double), ("cache_hit", C.c_int32)]


class spfas_server_counters(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("setups", C.c_int64),
                ("cache_hits", C.c_int64), ("evictions", C.c_int64), ("peak_bytes", C.c_int64),
                ("cached_bytes", C.c_int64), ("budget_bytes", C.c_int64)]


_lib = None


def lib():
    """Loads the in-tree library; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime under the same soname
    # (libamdhip64.so.7); loading torch first makes this library bind to
    # that one runtime instead of bringing a second copy into the process.
    try:
        import torch  # noqa: F401
    except Exception:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(paper_2005_01275_amd/build.py); there is no fallback path")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.spfas_default_solve_opts.argtypes = [C.POINTER(spfas_solve_opts)]
    L.spfas_default_solve_opts.restype = None
    L.spfas_setup_hierarchy.argtypes = [C.POINTER(spfas_mesh), C.POINTER(spfas_coarsen_opts),
                                        C.POINTER(spfas_allocator), vp, C.POINTER(vp)]
    L.spfas_setup_hierarchy.restype = C.c_int
    for nm in ("spfas_fas_solve", "spfas_picard_solve", "spfas_newton_solve"):
        f = getattr(L, nm)
        f.argtypes = [vp, C.POINTER(spfas_problem), C.POINTER(spfas_solve_opts), vp, vp, C.c_int32,
                      C.POINTER(spfas_stats), vp]
        f.restype = C.c_int
    L.spfas_cascadic_solve.argtypes = [vp, C.POINTER(spfas_problem), C.POINTER(spfas_solve_opts), vp, vp, C.c_int32,
                                       C.POINTER(spfas_stats), _ip, vp]
    L.spfas_cascadic_solve.restype = C.c_int
    L.spfas_eval_residual.argtypes = [vp, C.POINTER(spfas_problem), vp, vp, vp, vp, C.c_int32, vp]
    L.spfas_eval_residual.restype = C.c_int
    L.spfas_eval_residual_noalloc.argtypes = [vp, C.POINTER(spfas_problem), vp, vp, vp, vp, vp]
    L.spfas_eval_residual_noalloc.restype = C.c_int
    L.spfas_level_sizes.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int64)]
    L.spfas_level_sizes.restype = C.c_int
    L.spfas_hierarchy_device_bytes.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.spfas_hierarchy_device_bytes.restype = C.c_int
    L.spfas_hierarchy_reset_peak.argtypes = [vp]
    L.spfas_hierarchy_reset_peak.restype = C.c_int
    L.spfas_get_aggregation.argtypes = [vp, C.c_int32, _ip]
    L.spfas_get_aggregation.restype = C.c_int
    L.spfas_get_permutation.argtypes = [vp, C.c_int32, _ip, _ip]
    L.spfas_get_permutation.restype = C.c_int
    L.spfas_get_level_operator.argtypes = [vp, C.c_int32, C.c_int32, _dp, C.c_size_t]
    L.spfas_get_level_operator.restype = C.c_int
    L.spfas_destroy.argtypes = [vp]
    L.spfas_destroy.restype = None
    L.spfas_last_error.argtypes = []
    L.spfas_last_error.restype = C.c_char_p
    L.spfas_version.argtypes = []
    L.spfas_version.restype = C.c_int
    L.spfas_profile_enable.argtypes = [vp, C.c_int32]
    L.spfas_profile_enable.restype = C.c_int
    L.spfas_profile_read.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
    L.spfas_profile_read.restype = C.c_int
    L.spfas_server_create.argtypes = [C.POINTER(spfas_server_opts), C.POINTER(vp)]
    L.spfas_server_create.restype = C.c_int
    L.spfas_server_add_model.argtypes = [vp, C.POINTER(spfas_mesh), C.POINTER(spfas_coarsen_opts),
                                         C.POINTER(C.c_int64)]
    L.spfas_server_add_model.restype = C.c_int
    L.spfas_server_submit.argtypes = [vp, C.c_int64, C.POINTER(spfas_problem), C.POINTER(spfas_solve_opts),
                                      C.c_int32, C.POINTER(C.c_int64)]
    L.spfas_server_submit.restype = C.c_int
    L.spfas_server_wait.argtypes = [vp, C.c_int64, vp, vp, C.POINTER(spfas_stats), C.POINTER(spfas_request_info)]
    L.spfas_server_wait.restype = C.c_int
    L.spfas_server_counters_get.argtypes = [vp, C.POINTER(spfas_server_counters)]
    L.spfas_server_counters_get.restype = C.c_int
    L.spfas_server_destroy.argtypes = [vp]
    L.spfas_server_destroy.restype = None
    L.spfas_server_last_error.argtypes = []
    L.spfas_server_last_error.restype = C.c_char_p
    _lib = L
    return L


def _torch_alloc(nbytes, stream, ctx):
    import torch
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception:
        return None


def _torch_free(ptr, nbytes, stream, ctx):
    import torch
    torch.cuda.caching_allocator_delete(int(ptr))


# callbacks that hand the hierarchy's device memory to PyTorch's caching
# allocator (kept alive for the life of the process)
TORCH_ALLOCATOR = spfas_allocator(alloc=ALLOC_FN(_torch_alloc), free=FREE_FN(_torch_free), ctx=None)


class SpfasError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"spfas error {code}: {msg}")
        self.code = code


def check(rc):
    if rc < 0:
        raise SpfasError(rc, lib().spfas_last_error().decode())
    return rc
