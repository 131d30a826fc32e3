"""ctypes declarations of include/mu.h and loading of libmu.so.

Argument marshalling only: every computation happens in the HIP library.
Loading fails loudly when the library has not been built; there is no CPU
fallback.
"""

from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmu.so")

MU_OK, MU_E_ARG, MU_E_NODEVICE, MU_E_NOMEM, MU_E_DEVICE, MU_E_UNSUPPORTED, MU_E_STATE = range(7)
MU_COST_CHI2, MU_COST_POISSON = 0, 1
MU_MEM_HOST, MU_MEM_DEVICE = 0, 1
MU_SE, MU_GE, MU_SG, MU_STG, MU_TF = range(5)
MU_REF_PAR, MU_REF_FUN, MU_REF_LIT = range(3)
MU_HESSE_GAUSS_NEWTON, MU_HESSE_DIFF = 0, 1
MU_MAX_TERMS = 4
MU_MAX_FACTORS_PER_TERM = 3
MU_MAX_PAR = 1024

PRIM_CODES = {"se": MU_SE, "ge": MU_GE, "sg": MU_SG, "stg": MU_STG, "tf": MU_TF}
COST_CODES = {"chi2": MU_COST_CHI2, "poisson": MU_COST_POISSON}

dp = C.POINTER(C.c_double)
vp = C.c_void_p


class MuError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mu status {status}: {msg}")
        self.status = status


class mu_histo(C.Structure):
    _fields_ = [("counts", vp), ("n_bins", C.c_int64), ("dt", C.c_double), ("t0_bin", C.c_double),
                ("first", C.c_int64), ("last", C.c_int64), ("map_row", C.c_int32), ("reserved", C.c_int32)]


class mu_ref(C.Structure):
    _fields_ = [("kind", C.c_int32), ("slot", C.c_int32), ("literal", C.c_double)]


class mu_factor(C.Structure):
    _fields_ = [("prim", C.c_int32), ("reserved", C.c_int32), ("arg", mu_ref * 2)]


class mu_term(C.Structure):
    _fields_ = [("coef", C.c_double), ("amp", mu_ref), ("first_factor", C.c_int32), ("n_factors", C.c_int32)]


class mu_theory_desc(C.Structure):
    _fields_ = [("tau_mu", C.c_double), ("n0", mu_ref), ("nbkg", mu_ref),
                ("terms", C.POINTER(mu_term)), ("n_terms", C.c_int32),
                ("factors", C.POINTER(mu_factor)), ("n_factors", C.c_int32),
                ("map", C.POINTER(C.c_int32)), ("n_rows", C.c_int32), ("n_slots", C.c_int32),
                ("F", dp), ("f0", dp), ("n_fun", C.c_int32), ("n_par", C.c_int32)]


class mu_expr_theory_desc(C.Structure):
    _fields_ = [("tau_mu", C.c_double), ("n0", mu_ref), ("nbkg", mu_ref), ("asymmetry", C.c_char_p),
                ("map", C.POINTER(C.c_int32)), ("n_rows", C.c_int32), ("n_slots", C.c_int32),
                ("F", dp), ("f0", dp), ("n_fun", C.c_int32), ("n_par", C.c_int32)]


class mu_fit_opts(C.Structure):
    _fields_ = [("max_fcn", C.c_int32), ("max_iter", C.c_int32), ("tol_edm", C.c_double),
                ("tol_step_rel", C.c_double), ("analytic_grad", C.c_int32), ("batched", C.c_int32),
                ("polish", C.c_int32), ("reserved", C.c_int32), ("fixed", C.c_void_p)]


class mu_fit_result(C.Structure):
    _fields_ = [("cost", C.c_double), ("edm", C.c_double), ("n_iter", C.c_int32), ("n_fcn", C.c_int32),
                ("n_grad", C.c_int32), ("status", C.c_int32)]


_lib = None


def lib():
    """The loaded libmu.so (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1604_02334_amd.build` "
                           "(there is no CPU fallback)")
    try:  # load torch's HIP runtime first so that both share one runtime
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    S = C.c_int
    sigs = {
        "mu_abi_version": (C.c_int, []),
        "mu_status_string": (C.c_char_p, [S]),
        "mu_ctx_create": (S, [C.c_int, vp, C.c_uint, C.POINTER(vp)]),
        "mu_ctx_destroy": (S, [vp]),
        "mu_ctx_last_error": (C.c_char_p, [vp]),
        "mu_ctx_synchronize": (S, [vp]),
        "mu_ctx_set_tile": (S, [vp, C.c_int32]),
        "mu_ctx_get_tile": (C.c_int32, [vp]),
        "mu_ctx_set_anchor": (S, [vp, C.c_int32]),
        "mu_ctx_get_anchor": (C.c_int32, [vp]),
        "mu_ctx_set_specialize": (S, [vp, C.c_int32]),
        "mu_ctx_timing": (S, [vp, C.c_int32]),
        "mu_ctx_timing_read": (S, [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
        "mu_autotune": (S, [vp, vp, vp, S, vp, C.c_int32, C.c_uint, C.c_int32, C.POINTER(C.c_int32),
                            C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
        "mu_autotune_set": (S, [vp, vp, vp, S, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
        "mu_autotune_batch": (S, [vp, C.c_int32, C.POINTER(vp), C.POINTER(vp), S, C.c_int32, vp, C.c_uint, C.c_int32,
                                  C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
        "mu_autotune_save": (S, [vp, C.c_char_p]),
        "mu_autotune_load": (S, [vp, C.c_char_p]),
        "mu_autotune_check_file": (S, [C.c_char_p, C.c_char_p, C.c_int32]),
        "mu_histo_check": (S, [C.POINTER(mu_histo), C.c_int32, C.c_char_p, C.c_int32]),
        "mu_data_create": (S, [vp, C.POINTER(mu_histo), C.c_int32, C.POINTER(vp)]),
        "mu_data_destroy": (S, [vp]),
        "mu_data_bins": (C.c_int64, [vp]),
        "mu_data_histos": (C.c_int32, [vp]),
        "mu_data_is_f64": (C.c_int32, [vp]),
        "mu_theory_check": (S, [C.POINTER(mu_theory_desc), C.c_char_p, C.c_int32]),
        "mu_theory_create": (S, [vp, C.POINTER(mu_theory_desc), C.POINTER(vp)]),
        "mu_theory_destroy": (S, [vp]),
        "mu_theory_npar": (C.c_int32, [vp]),
        "mu_theory_check_expr": (S, [C.POINTER(mu_expr_theory_desc), C.c_char_p, C.c_int32]),
        "mu_theory_expr_source": (S, [C.POINTER(mu_expr_theory_desc), C.c_char_p, C.c_int64,
                                      C.POINTER(C.c_int64)]),
        "mu_theory_compile_check": (S, [C.POINTER(mu_expr_theory_desc), C.c_char_p, C.c_int32]),
        "mu_theory_create_expr": (S, [vp, C.POINTER(mu_expr_theory_desc), C.POINTER(vp)]),
        "mu_chi2_eval": (S, [vp, vp, vp, S, vp, C.c_int32, C.c_uint, vp, vp]),
        "mu_chi2_grad": (S, [vp, vp, vp, S, vp, C.c_int32, C.c_uint, vp, vp]),
        "mu_chi2_eval_static": (S, [vp, vp, vp, S, vp, C.c_int32, vp, vp]),
        "mu_chi2_eval_grad": (S, [vp, vp, vp, S, vp, C.c_int32, vp, C.c_int32, C.c_uint, vp, vp, vp]),
        "mu_chi2_batch": (S, [vp, C.c_int32, C.POINTER(vp), C.POINTER(vp), S, C.c_int32, vp, C.c_uint, vp, vp]),
        "mu_model_eval": (S, [vp, vp, vp, vp, C.c_uint, vp]),
        "mu_hesse": (S, [vp, vp, vp, S, C.c_int32, vp, vp, vp, vp, C.POINTER(C.c_int32)]),
        "mu_profile": (S, [vp, vp, vp, S, vp, vp, C.c_int32, C.c_int32, vp, vp, vp, vp]),
        "mu_minos": (S, [vp, vp, vp, S, vp, vp, C.c_int32, C.c_double, C.POINTER(C.c_double),
                         C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
        "mu_fit_batch": (S, [vp, C.c_int32, C.POINTER(vp), C.POINTER(vp), S, C.c_int32, vp,
                             C.POINTER(mu_fit_opts), vp, vp, C.POINTER(mu_fit_result)]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols():
    """Names declared in include/mu.h that the binding expects."""
    return sorted(["mu_abi_version", "mu_status_string", "mu_ctx_create", "mu_ctx_destroy", "mu_ctx_last_error",
                   "mu_ctx_synchronize", "mu_ctx_set_tile", "mu_ctx_get_tile", "mu_ctx_set_anchor", "mu_ctx_get_anchor",
                   "mu_ctx_set_specialize", "mu_ctx_timing", "mu_ctx_timing_read", "mu_autotune", "mu_autotune_set",
                   "mu_autotune_batch", "mu_autotune_save", "mu_autotune_load", "mu_autotune_check_file",
                   "mu_histo_check", "mu_data_create",
                   "mu_data_destroy", "mu_data_bins", "mu_data_histos", "mu_data_is_f64", "mu_theory_check",
                   "mu_theory_create", "mu_theory_destroy", "mu_theory_npar", "mu_theory_check_expr",
                   "mu_theory_expr_source", "mu_theory_compile_check", "mu_theory_create_expr",
                   "mu_chi2_eval", "mu_chi2_grad",
                   "mu_chi2_eval_static",
                   "mu_chi2_eval_grad", "mu_chi2_batch", "mu_model_eval", "mu_fit_batch", "mu_hesse", "mu_profile",
                   "mu_minos",
                   "mu_seeder_param_count", "mu_seeder_create", "mu_seeder_destroy", "mu_seeder_get_params",
                   "mu_seeder_get_grads", "mu_seeder_steps", "mu_gen_histos", "mu_seeder_forward",
                   "mu_seeder_train_step", "mu_seeder_train", "mu_seed_infer", "mu_seeder_save", "mu_seeder_layer",
                   "mu_seeder_load"])
