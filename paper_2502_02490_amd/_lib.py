"""ctypes declarations of the C ABI in include/dirac.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdirac.so")

OK, EINVAL, ENOMEM, EHIP, ESINGULAR, ENOCONV, ENONFINITE, EUNSUPPORTED = range(8)
STATUS_NAMES = ["DIRAC_OK", "DIRAC_EINVAL", "DIRAC_ENOMEM", "DIRAC_EHIP", "DIRAC_ESINGULAR", "DIRAC_ENOCONV",
                "DIRAC_ENONFINITE", "DIRAC_EUNSUPPORTED"]
F64, F32, F16, BF16 = 0, 1, 2, 3
LEX, EO, NATIVE, OPENQXD = 0, 1, 2, 3
CGLS, GCR, MIXED_GCR, FGCR_PTC, FGCR_PTC_EO, FGCR_SAP = 0, 1, 2, 3, 4, 5

# every symbol declared in include/dirac.h
EXPORTS = ["dirac_create", "dirac_create_openqxd", "dirac_set_cache_block", "dirac_destroy", "dirac_load_clover", "dirac_get_clover", "clover_invert",
           "dirac_native_bytes", "dirac_import", "dirac_export", "dirac_apply", "dirac_apply_eo", "dirac_apply_eo_multi",
           "dirac_apply_eo_noalloc",
           "dirac_apply_hop", "dirac_apply_clover", "dirac_sap", "dirac_solve", "dirac_solve_batched", "dirac_last_error",
           "ptc_create", "ptc_destroy", "ptc_num_weights", "ptc_set_weights", "ptc_get_weights", "ptc_get_grad",
           "ptc_zero_grad", "ptc_forward", "ptc_forward_eo", "ptc_backward", "ptc_adam_step", "ptc_get_adam_state", "ptc_set_adam_state",
           "ptc_train_step", "ptc_loss", "dirac_residual", "dirac_lincomb", "dirac_dot"]


class Params(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("kappa", ctypes.c_double), ("csw", ctypes.c_double),
                ("csw_qed", ctypes.c_double), ("qhat", ctypes.c_int), ("bc_phase", ctypes.c_double * 4),
                ("cstar", ctypes.c_int)]


class SolverParams(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("tol", ctypes.c_double), ("inner_prec", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("x0_given", ctypes.c_int), ("precision", ctypes.c_int), ("ptc", ctypes.c_void_p),
                ("sap_ncy", ctypes.c_int), ("sap_nmr", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("restarts", ctypes.c_int), ("outer", ctypes.c_int),
                ("fell_back", ctypes.c_int), ("true_rel_res", ctypes.c_double), ("seconds", ctypes.c_double),
                ("host_syncs", ctypes.c_int)]


class DiracError(RuntimeError):
    def __init__(self, status: int, message: str):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libdirac.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2502_02490_amd.build` "
                           "(the library has no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i, st = ctypes.c_void_p, ctypes.c_int, ctypes.c_int
    lib.dirac_create.argtypes = [ctypes.POINTER(Params), vp, vp, vp, ctypes.POINTER(vp)]
    lib.dirac_destroy.argtypes = [vp]
    lib.dirac_create_openqxd.argtypes = [ctypes.POINTER(Params), vp, vp, vp, vp, ctypes.POINTER(vp)]
    lib.dirac_set_cache_block.argtypes = [vp, vp]
    lib.dirac_load_clover.argtypes = [vp, vp, i, vp]
    lib.dirac_get_clover.argtypes = [vp, vp, i, i, vp]
    lib.clover_invert.argtypes = [vp, i, vp]
    lib.dirac_native_bytes.argtypes = [vp, i, i]
    lib.dirac_native_bytes.restype = ctypes.c_size_t
    lib.dirac_import.argtypes = [vp, vp, vp, i, i, i, vp]
    lib.dirac_export.argtypes = [vp, vp, vp, i, i, i, vp]
    lib.dirac_apply.argtypes = [vp, vp, vp, i, i, i, vp]
    lib.dirac_apply_eo.argtypes = [vp, vp, vp, i, i, i, vp]
    lib.dirac_apply_eo_multi.argtypes = [vp, vp, vp, i, i, i, vp]
    lib.dirac_apply_eo_noalloc.argtypes = [vp, vp, vp, i, i, vp]
    lib.dirac_apply_hop.argtypes = [vp, vp, vp, i, i, i, vp]
    lib.dirac_apply_clover.argtypes = [vp, vp, vp, i, i, i, vp]
    lib.dirac_sap.argtypes = [vp, vp, vp, i, i, vp]
    lib.dirac_solve.argtypes = [vp, vp, vp, i, ctypes.POINTER(SolverParams), ctypes.POINTER(SolveInfo), vp]
    lib.dirac_solve_batched.argtypes = [vp, i, vp, vp, i, i, ctypes.POINTER(SolverParams), vp, vp]
    lib.dirac_last_error.restype = ctypes.c_char_p
    lib.ptc_create.argtypes = [vp, i, ctypes.POINTER(vp)]
    lib.ptc_destroy.argtypes = [vp]
    lib.ptc_num_weights.argtypes = [vp]
    lib.ptc_num_weights.restype = ctypes.c_size_t
    lib.ptc_set_weights.argtypes = [vp, vp, ctypes.c_size_t]
    lib.ptc_get_weights.argtypes = [vp, vp, ctypes.c_size_t]
    lib.ptc_get_grad.argtypes = [vp, vp, ctypes.c_size_t]
    lib.ptc_zero_grad.argtypes = [vp, vp]
    lib.ptc_forward.argtypes = [vp, vp, vp, vp, vp]
    lib.ptc_forward_eo.argtypes = [vp, vp, vp, vp, vp]
    lib.ptc_backward.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.ptc_adam_step.argtypes = [vp, ctypes.c_double, vp]
    lib.ptc_get_adam_state.argtypes = [vp, vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int)]
    lib.ptc_set_adam_state.argtypes = [vp, vp, vp, ctypes.c_size_t, i]
    lib.ptc_train_step.argtypes = [vp, vp, vp, vp, i, ctypes.c_double, ctypes.POINTER(ctypes.c_double), vp]
    lib.ptc_loss.argtypes = [vp, vp, vp, vp, i, ctypes.POINTER(ctypes.c_double), vp]
    dp = ctypes.POINTER(ctypes.c_double)
    lib.dirac_residual.argtypes = [vp, vp, vp, vp, i, dp, vp]
    lib.dirac_lincomb.argtypes = [vp, vp, i, ctypes.c_double, vp, ctypes.c_double, vp, i, i, dp, vp]
    lib.dirac_dot.argtypes = [vp, vp, vp, i, i, dp, vp]
    for name in EXPORTS:
        if name not in ("dirac_native_bytes", "dirac_last_error", "ptc_num_weights"):
            getattr(lib, name).restype = st
    _lib = lib
    return lib


def check(status: int) -> int:
    if status != OK:
        msg = _lib.dirac_last_error().decode() if _lib is not None else ""
        raise DiracError(status, msg)
    return status
