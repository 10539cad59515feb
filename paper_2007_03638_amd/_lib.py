"""ctypes declarations of the C ABI in include/mera.h (argument marshalling only)."""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmera_hip.so")

c_int, c_double, c_void_p, c_size_t, c_uint64 = (ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t,
                                                 ctypes.c_uint64)


class MeraMat(ctypes.Structure):
    _fields_ = [("n", c_int), ("p", c_int), ("data", c_void_p)]


class MeraShape(ctypes.Structure):
    _fields_ = [("T", c_int), ("d", c_int), ("chi", c_int), ("geometry", c_int)]


class KrylovOpts(ctypes.Structure):
    _fields_ = [("krylov_dim", c_int), ("max_restarts", c_int), ("tol", c_double), ("extrapolate", c_int)]


class EvalInfo(ctypes.Structure):
    _fields_ = [("energy", c_double), ("applications_rho", c_int), ("applications_htilde", c_int),
                ("residual_rho", c_double), ("residual_htilde", c_double), ("macs", c_double)]


class Job(ctypes.Structure):
    _fields_ = [("shape", MeraShape), ("h3_host", ctypes.POINTER(c_double)),
                ("init_host", ctypes.POINTER(ctypes.POINTER(c_double))), ("prec", c_int), ("lbfgs_m", c_int),
                ("max_iter", c_int), ("grad_tol", c_double), ("polish_tol", c_double), ("precondition", c_int),
                ("max_ls_evals", c_int), ("krylov", KrylovOpts), ("method", c_int), ("retraction", c_int),
                ("grassmann_w", c_int), ("ev_gamma", c_double)]


class Result(ctypes.Structure):
    _fields_ = [("energy", c_double), ("gnorm", c_double), ("iterations", c_int), ("evaluations", c_int),
                ("status", c_int), ("polish_iter", c_int), ("seconds", c_double), ("macs", c_double),
                ("queued_seconds", c_double), ("krylov_applications", c_int)]


class ServerStats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_int64), ("grouped_batches", ctypes.c_int64), ("bindings", ctypes.c_int64),
                ("graph_launches", ctypes.c_int64), ("graph_captures", ctypes.c_int64),
                ("eager_runs", ctypes.c_int64)]


class IterLog(ctypes.Structure):
    _fields_ = [("iter", c_int), ("evals", c_int), ("energy", c_double), ("gnorm", c_double), ("alpha", c_double),
                ("prec", c_int)]


class KernelStat(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_char * 80), ("launches", c_int), ("seconds", c_double), ("flops", c_double),
                ("bytes", c_double)]


MAT_P = ctypes.POINTER(MeraMat)

# name -> (restype, argtypes)
SIGNATURES = {
    "mera_ctx_create": (c_int, [c_int, c_void_p, ctypes.POINTER(c_void_p)]),
    "mera_ctx_destroy": (None, [c_void_p]),
    "mera_last_error": (ctypes.c_char_p, [c_void_p]),
    "mera_ctx_trim": (c_int, [c_void_p]),
    "mera_ctx_macs": (c_double, [c_void_p]),
    "mera_ctx_set_intermediate_limit": (c_int, [c_void_p, c_size_t]),
    "mera_ctx_set_verbose": (c_int, [c_void_p, c_int]),
    "mera_layer_dims": (c_int, [ctypes.POINTER(MeraShape), ctypes.POINTER(c_int), ctypes.POINTER(c_int)]),
    "mera_h3_tfim": (c_int, [c_double, ctypes.POINTER(c_double)]),
    "mera_h3_xxz": (c_int, [c_double, ctypes.POINTER(c_double)]),
    "mera_h2_tfim": (c_int, [c_double, ctypes.POINTER(c_double)]),
    "mera_h2_xxz": (c_int, [c_double, ctypes.POINTER(c_double)]),
    "mera_warm_create": (c_int, [c_void_p, ctypes.POINTER(MeraShape), ctypes.POINTER(c_void_p)]),
    "mera_warm_destroy": (None, [c_void_p]),
    "mera_energy_grad": (c_int, [c_void_p, ctypes.POINTER(MeraShape), MAT_P, MAT_P, c_void_p, c_int, c_void_p,
                                 ctypes.POINTER(KrylovOpts), ctypes.POINTER(c_double), MAT_P, MAT_P, MAT_P, MAT_P,
                                 ctypes.POINTER(EvalInfo)]),
    "mera_ascend": (c_int, [c_void_p, ctypes.POINTER(MeraShape), c_int, MAT_P, MAT_P, c_int, c_void_p, c_void_p]),
    "mera_descend": (c_int, [c_void_p, ctypes.POINTER(MeraShape), c_int, MAT_P, MAT_P, c_int, c_void_p, c_void_p]),
    "mera_layer_grad": (c_int, [c_void_p, ctypes.POINTER(MeraShape), c_int, MAT_P, MAT_P, c_int, c_int, c_void_p,
                                c_void_p, c_void_p, MAT_P, MAT_P, c_void_p]),
    "stiefel_project": (c_int, [c_void_p, c_int, MAT_P, MAT_P, MAT_P]),
    "stiefel_project_noalloc": (c_int, [c_void_p, c_int, MAT_P, MAT_P, MAT_P]),
    "stiefel_retract": (c_int, [c_void_p, c_int, MAT_P, MAT_P, c_double, MAT_P, MAT_P]),
    "stiefel_transport": (c_int, [c_void_p, c_int, MAT_P, MAT_P, MAT_P]),
    "stiefel_retract_exp": (c_int, [c_void_p, c_int, MAT_P, MAT_P, c_double, MAT_P, MAT_P]),
    "stiefel_transport_exp": (c_int, [c_void_p, c_int, MAT_P, MAT_P, c_double, MAT_P, MAT_P]),
    "grassmann_project": (c_int, [c_void_p, c_int, MAT_P, MAT_P, MAT_P]),
    "mera_ev_update": (c_int, [c_void_p, c_int, MAT_P, MAT_P, MAT_P, c_double, MAT_P]),
    "stiefel_precondition": (c_int, [c_void_p, c_int, MAT_P, MAT_P, MAT_P, c_double, MAT_P]),
    "mera_inner": (c_int, [c_void_p, c_int, MAT_P, MAT_P, ctypes.POINTER(c_double)]),
    "lbfgs_create": (c_int, [c_void_p, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int), c_int,
                             ctypes.POINTER(c_void_p)]),
    "lbfgs_destroy": (None, [c_void_p]),
    "lbfgs_reset": (c_int, [c_void_p]),
    "lbfgs_size": (c_int, [c_void_p]),
    "lbfgs_step": (c_int, [c_void_p, c_void_p, MAT_P, MAT_P, MAT_P, MAT_P, ctypes.POINTER(c_double)]),
    "lbfgs_push": (c_int, [c_void_p, c_void_p, MAT_P, MAT_P, c_double, MAT_P, MAT_P, ctypes.POINTER(c_int)]),
    "run_optimize": (c_int, [c_void_p, ctypes.POINTER(Job), ctypes.POINTER(Result),
                             ctypes.POINTER(ctypes.POINTER(c_double)), ctypes.POINTER(IterLog), c_int,
                             ctypes.POINTER(c_int)]),
    "mera_ctx_profile": (c_int, [c_void_p, c_int]),
    "mera_ctx_kernel_stats": (c_int, [c_void_p, ctypes.POINTER(KernelStat), c_int]),
    "mera_opt_create": (c_int, [c_void_p, ctypes.POINTER(Job), ctypes.POINTER(c_void_p)]),
    "mera_opt_step": (c_int, [c_void_p, c_void_p, ctypes.POINTER(c_int), ctypes.POINTER(Result)]),
    "mera_opt_final": (c_int, [c_void_p, c_void_p, ctypes.POINTER(ctypes.POINTER(c_double))]),
    "mera_opt_destroy": (None, [c_void_p]),
    "mera_server_create": (c_int, [c_void_p, c_size_t, c_int, ctypes.POINTER(c_void_p)]),
    "mera_server_configure": (c_int, [c_void_p, c_int, c_int, c_double]),
    "mera_server_get_stats": (c_int, [c_void_p, ctypes.POINTER(ServerStats)]),
    "mera_server_submit": (c_int, [c_void_p, ctypes.POINTER(Job), ctypes.POINTER(c_uint64)]),
    "mera_server_poll": (c_int, [c_void_p, c_uint64, ctypes.POINTER(Result)]),
    "mera_job_footprint": (c_size_t, [ctypes.POINTER(MeraShape), c_int]),
    "mera_server_destroy": (None, [c_void_p]),
}

_lib = None


def load():
    """Load the built HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} (run paper_2007_03638_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
