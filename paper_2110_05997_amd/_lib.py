"""ctypes binding of libcpd (include/cpd.h).

Argument marshalling only: every step of the CPD path runs in the HIP library.  PyTorch supplies
device memory (``tensor.data_ptr()``) and the current HIP stream.  If the shared library is not
built the import of this module raises, on purpose: there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libcpd.so")

CPD_F64, CPD_F32, CPD_BF16 = 0, 1, 2
CPD_INIT_RANDOM, CPD_INIT_MLSVD, CPD_INIT_GIVEN = 0, 1, 2
STOP_NAMES = {0: "none", 1: "rel_err", 2: "step", 3: "improvement", 4: "grad", 5: "avg_err",
              6: "avg_impr", 7: "diverged", 8: "maxiter"}


class CpdError(RuntimeError):
    pass


class Params(ctypes.Structure):
    _fields_ = [
        ("maxiter", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("mlsvd_tol", ctypes.c_double),
        ("init_damp", ctypes.c_double),
        ("cg_tol", ctypes.c_double),
        ("cg_fixed", ctypes.c_int32),
        ("cg_uniforms", ctypes.POINTER(ctypes.c_double)),
        ("seed", ctypes.c_uint64),
        ("init", ctypes.c_int32),
        ("core_dims", ctypes.c_int32 * 3),
        ("compute_dtype", ctypes.c_int32),
        ("refine_iters", ctypes.c_int32),
        ("st_mlsvd", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("drawback", ctypes.c_int32),
    ]


class StepInfo(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int32),
        ("cg_iters", ctypes.c_int32),
        ("cg_cap", ctypes.c_int32),
        ("stop", ctypes.c_int32),
        ("rel_err", ctypes.c_double),
        ("step_norm", ctypes.c_double),
        ("grad_inf", ctypes.c_double),
        ("gain", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("cg_resid", ctypes.c_double),
        ("t_ns", ctypes.c_int64),
        ("drew_back", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class SolveInfo(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("stop_reason", ctypes.c_int32),
        ("core_dims", ctypes.c_int32 * 3),
        ("tol_iter", ctypes.c_int32),
        ("rel_err_core", ctypes.c_double),
        ("rel_err_full", ctypes.c_double),
        ("t_norm", ctypes.c_double),
        ("refine_iters", ctypes.c_int32),
        ("refine_stop", ctypes.c_int32),
        ("time_to_tol_ns", ctypes.c_int64),
    ]


class KernelTime(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class BatchItem(ctypes.Structure):
    _fields_ = [
        ("T", ctypes.c_void_p),
        ("dims", ctypes.c_int64 * 3),
        ("R", ctypes.c_int32),
        ("W0", ctypes.c_void_p * 3),
        ("W", ctypes.c_void_p * 3),
        ("lam", ctypes.c_void_p),
    ]


class Mlp(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_h1", ctypes.c_int32), ("n_h2", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("W", ctypes.c_void_p * 3), ("b", ctypes.c_void_p * 3)]


class MlpGrads(ctypes.Structure):
    _fields_ = [("dW", ctypes.c_void_p * 3), ("db", ctypes.c_void_p * 3)]


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("step", ctypes.c_int32), ("mW", ctypes.c_void_p * 3),
                ("mb", ctypes.c_void_p * 3), ("vW", ctypes.c_void_p * 3), ("vb", ctypes.c_void_p * 3)]


PROFILE_KERNELS = ["gram", "dgn", "project", "residual", "mttkrp", "eig"]

_P = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_I64x3 = ctypes.c_int64 * 3
_I32x3 = ctypes.c_int32 * 3
_Px3 = ctypes.c_void_p * 3

# (name, restype, argtypes) for every symbol declared in include/cpd.h
SIGNATURES = [
    ("cpd_last_error", ctypes.c_char_p, []),
    ("cpd_version", ctypes.c_char_p, []),
    ("cpd_default_params", None, [ctypes.POINTER(Params)]),
    ("cpd_workspace_bytes", ctypes.c_size_t, [_I64x3, ctypes.c_int32, ctypes.POINTER(Params)]),
    ("cpd_compress", ctypes.c_int, [_P, ctypes.c_int32, _I64x3, ctypes.c_int32, ctypes.POINTER(Params),
                                    _Px3, _Px3, _P, _I32x3, _P, ctypes.c_size_t, _P]),
    ("cpd_state_bytes", ctypes.c_size_t, [_I32x3, ctypes.c_int32, ctypes.POINTER(Params)]),
    ("cpd_state_init", ctypes.c_int, [_P, _P, _I32x3, ctypes.c_int32, _P, ctypes.c_double,
                                      ctypes.POINTER(Params), _P]),
    ("cpd_dgn_step", ctypes.c_int, [_P, _P, ctypes.POINTER(Params), ctypes.POINTER(StepInfo), _P]),
    ("cpd_dgn_run", ctypes.c_int, [_P, _P, ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(StepInfo), ctypes.c_int32, _P]),
    ("cpd_state_factors", ctypes.c_int, [_P, _P, ctypes.c_int32, _P]),
    ("cpd_solve", ctypes.c_int, [_P, ctypes.c_int32, _I64x3, ctypes.c_int32, ctypes.POINTER(Params), _P,
                                 _Px3, _P, ctypes.POINTER(SolveInfo), _P, ctypes.c_size_t, _P]),
    ("cpd_solve_mixed", ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_int32, _I64x3, ctypes.c_int32,
                                       ctypes.POINTER(Params), _P, _Px3, _P, ctypes.POINTER(SolveInfo), _P,
                                       ctypes.c_size_t, _P]),
    ("cpd_gram_workspace_bytes", ctypes.c_size_t, [_I64x3, ctypes.c_int32]),
    ("cpd_gram", ctypes.c_int, [_P, ctypes.c_int32, _I64x3, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                ctypes.c_size_t, _P]),
    ("cpd_eig_workspace_bytes", ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    ("cpd_eig_top", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, ctypes.c_size_t, _P]),
    ("cpd_mttkrp_workspace_bytes", ctypes.c_size_t, [_I64x3, ctypes.c_int32, ctypes.c_int32]),
    ("cpd_mttkrp", ctypes.c_int, [_P, ctypes.c_int32, _I64x3, _Px3, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, _P, _P, ctypes.c_size_t, _P]),
    ("cpd_residual_workspace_bytes", ctypes.c_size_t, [_I64x3]),
    ("cpd_residual_norm2", ctypes.c_int, [_P, ctypes.c_int32, _I64x3, _Px3, ctypes.c_int32, _P, _P,
                                          ctypes.c_size_t, _P]),
    ("cpd_tt_workspace_bytes", ctypes.c_size_t, [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                                                  ctypes.POINTER(Params)]),
    ("cpd_solve_tt", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32,
                                    ctypes.POINTER(Params), _P, ctypes.POINTER(ctypes.c_void_p), _P,
                                    ctypes.POINTER(SolveInfo), _P, ctypes.c_size_t, _P]),
    ("cpd_residual_norm2_noalloc", ctypes.c_int, [_P, ctypes.c_int32, _I64x3, _Px3, ctypes.c_int32, _P, _P]),
    ("cpd_jtj_v", ctypes.c_int, [_Px3, _Px3, _I32x3, ctypes.c_int32, _Px3, _P]),
    ("cpd_batch_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(BatchItem), ctypes.c_int32,
                                                     ctypes.POINTER(Params)]),
    ("cpd_solve_batched", ctypes.c_int, [ctypes.POINTER(BatchItem), ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(Params), ctypes.POINTER(SolveInfo), _P, ctypes.c_size_t,
                                         _P]),
    ("cpd_batch_plan_create", ctypes.c_int, [ctypes.POINTER(BatchItem), ctypes.c_int32, ctypes.c_int32,
                                             ctypes.POINTER(Params), _P, ctypes.c_size_t, _P,
                                             ctypes.POINTER(ctypes.c_void_p)]),
    ("cpd_batch_plan_run", ctypes.c_int, [_P, ctypes.POINTER(SolveInfo), _P]),
    ("cpd_batch_plan_variant", ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_float)]),
    ("cpd_batch_plan_destroy", None, [_P]),
    ("cpd_mlp_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(Mlp), ctypes.c_int32]),
    ("cpd_mlp_forward", ctypes.c_int, [ctypes.POINTER(Mlp), _P, _P, ctypes.c_int32, _P, ctypes.c_size_t, _P]),
    ("cpd_mlp_mse", ctypes.c_int, [_P, _P, ctypes.c_int64, _P, _P, _P, ctypes.c_size_t, _P]),
    ("cpd_mlp_backward", ctypes.c_int, [ctypes.POINTER(Mlp), _P, _P, ctypes.POINTER(MlpGrads), ctypes.c_int32, _P,
                                        ctypes.c_size_t, _P]),
    ("cpd_mlp_adam_step", ctypes.c_int, [ctypes.POINTER(Mlp), ctypes.POINTER(MlpGrads), ctypes.POINTER(Adam), _P]),
    ("cpd_learned_features", ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64, _P, _P, _P]),
    ("cpd_learned_target", ctypes.c_int, [_Px3, _P, _I32x3, ctypes.c_int32, ctypes.c_double, _P, _P]),
    ("cpd_learned_start_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(Mlp), _I32x3, ctypes.c_int32,
                                                            ctypes.c_int32]),
    ("cpd_learned_start", ctypes.c_int, [ctypes.POINTER(Mlp), _P, _I32x3, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_double, ctypes.POINTER(Params), _P, _P,
                                         ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_double), _P, ctypes.c_size_t, _P]),
    ("cpd_profile_enable", None, [ctypes.c_int32]),
    ("cpd_profile_select", None, [ctypes.c_uint32]),
    ("cpd_profile_reset", None, []),
    ("cpd_profile_read", ctypes.c_int, [ctypes.POINTER(KernelTime)]),
    ("cpd_profile_block_sum_ns", ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_size_t,
                                                ctypes.POINTER(ctypes.c_double), _P]),
]

_lib = None


def lib():
    """Load libcpd.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libcpd is not built ({LIB_PATH} missing); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, what):
    if status != 0:
        msg = lib().cpd_last_error().decode(errors="replace")
        raise CpdError(f"{what} failed with status {status}: {msg}")
