"""ctypes declarations of the C ABI in include/lq.h (liblq.so, built in-tree).

Loading fails loudly if the library has not been built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblq.so")

LQ_OK, LQ_NOT_CONVERGED = 0, 1
STATUS_NAMES = {0: "LQ_OK", 1: "LQ_NOT_CONVERGED", -1: "LQ_ERR_ARG", -2: "LQ_ERR_STATE", -3: "LQ_ERR_HIP",
                -4: "LQ_ERR_NOMEM", -5: "LQ_ERR_SINGULAR", -6: "LQ_ERR_NONFINITE", -7: "LQ_ERR_NODEVICE"}

F64, F32, F16 = 0, 1, 2
PREC = {"f64": F64, "f32": F32, "f16": F16}

KINDS = {"D": 0, "Ddag": 1, "DdagD": 2, "schur": 3, "schur_dag": 4, "schur_normal": 5, "hop_eo": 6,
         "hop_oe": 7, "hop_eo_dag": 8, "hop_oe_dag": 9, "clover_e": 10, "clover_o": 11, "clover_inv_o": 12,
         "schur_left": 13}
FULL_KINDS = ("D", "Ddag", "DdagD")

CGNE, BICGSTAB = 0, 1


class OpParams(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("kappa", ctypes.c_double), ("csw", ctypes.c_double),
                ("bc", (ctypes.c_double * 2) * 4), ("clover_traceless", ctypes.c_int), ("link_recon", ctypes.c_int),
                ("twist", ctypes.c_double)]


class SolverParams(ctypes.Structure):
    _fields_ = [("solver", ctypes.c_int), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int),
                ("inner", ctypes.c_int), ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int),
                ("check_every", ctypes.c_int), ("even_odd", ctypes.c_int), ("left_precond", ctypes.c_int),
                ("reliable", ctypes.c_int), ("deflate", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("nconv", ctypes.c_int), ("nouter", ctypes.c_int), ("restarts", ctypes.c_int),
                ("converged", ctypes.c_int), ("diff", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
                ("hop_bytes", ctypes.c_double), ("n_hop", ctypes.c_int)]


LEAPFROG, OMELYAN = 0, 1
INTEGRATORS = {"leapfrog": LEAPFROG, "omelyan": OMELYAN}


class MDParams(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("tau", ctypes.c_double), ("nsteps", ctypes.c_int),
                ("integrator", ctypes.c_int), ("lam", ctypes.c_double), ("fermion", ctypes.c_int),
                ("force_prec", ctypes.c_int), ("chrono", ctypes.c_int)]


class MDStats(ctypes.Structure):
    _fields_ = [("H0", ctypes.c_double), ("H1", ctypes.c_double), ("dH", ctypes.c_double),
                ("T0", ctypes.c_double), ("T1", ctypes.c_double), ("Sg0", ctypes.c_double),
                ("Sg1", ctypes.c_double), ("Sf0", ctypes.c_double), ("Sf1", ctypes.c_double),
                ("n_force", ctypes.c_int), ("converged", ctypes.c_int), ("iters", ctypes.c_long),
                ("t_ms", ctypes.c_double)]


class EigParams(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int), ("m", ctypes.c_int), ("max_restarts", ctypes.c_int),
                ("cheb_degree", ctypes.c_int), ("cheb_lo", ctypes.c_double), ("cheb_hi", ctypes.c_double),
                ("tol", ctypes.c_double)]


class EigStats(ctypes.Structure):
    _fields_ = [("nconv", ctypes.c_int), ("restarts", ctypes.c_int), ("applies", ctypes.c_long),
                ("cheb_lo", ctypes.c_double), ("cheb_hi", ctypes.c_double)]


class MGParams(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int * 4), ("nvec", ctypes.c_int), ("setup_iters", ctypes.c_int),
                ("setup_tol", ctypes.c_double), ("smooth_steps", ctypes.c_int), ("coarse_tol", ctypes.c_double),
                ("coarse_max_iter", ctypes.c_int), ("gcr_restart", ctypes.c_int)]


# name -> (restype, argtypes)
P = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double
SIGNATURES = {
    "lq_op_params_default": (None, [ctypes.POINTER(OpParams)]),
    "lq_solver_params_default": (None, [ctypes.POINTER(SolverParams)]),
    "lq_version": (ctypes.c_char_p, []),
    "lq_last_error": (ctypes.c_char_p, []),
    "lq_op_create": (I, [ctypes.POINTER(OpParams), ctypes.POINTER(P)]),
    "lq_op_destroy": (None, [P]),
    "lq_op_set_gauge": (I, [P, P, P]),
    "lq_op_set_gauge_host": (I, [P, P, P]),
    "lq_workspace_bytes": (I, [ctypes.POINTER(OpParams), I, ctypes.POINTER(ctypes.c_size_t)]),
    "lq_op_workspace_bytes": (I, [P, I, ctypes.POINTER(ctypes.c_size_t)]),
    "lq_op_bind": (I, [P, P, ctypes.c_size_t]),
    "lq_op_set_params": (I, [P, D, D, P, P]),
    "lq_op_apply": (I, [P, I, I, P, P, I, P]),
    "lq_op_apply_noalloc": (I, [P, I, I, P, P, I, P]),
    "lq_op_apply_host": (I, [P, I, I, P, P, I, P]),
    "lq_field_create": (I, [P, I, I, ctypes.POINTER(P)]),
    "lq_field_destroy": (None, [P]),
    "lq_field_import": (I, [P, P, P]),
    "lq_field_export": (I, [P, P, P]),
    "lq_op_apply_field": (I, [P, I, P, P, P]),
    "lq_op_set_block": (I, [P, I, I]),
    "lq_op_set_option": (I, [P, ctypes.c_char_p, I]),
    "lq_op_get_option": (I, [P, ctypes.c_char_p, ctypes.POINTER(I)]),
    "lq_op_traffic": (I, [P, I, I, I, ctypes.POINTER(D), ctypes.POINTER(D)]),
    "lq_solve": (I, [P, ctypes.POINTER(SolverParams), I, I, P, P, I, ctypes.POINTER(SolveStats), P]),
    "lq_solve_host": (I, [P, ctypes.POINTER(SolverParams), I, I, P, P, I, ctypes.POINTER(SolveStats), P]),
    "lq_batch_create": (I, [ctypes.POINTER(P), I, ctypes.POINTER(I), ctypes.POINTER(P)]),
    "lq_batch_solve": (I, [P, ctypes.POINTER(SolverParams), ctypes.POINTER(P), ctypes.POINTER(P),
                           ctypes.POINTER(SolveStats), P]),
    "lq_batch_destroy": (None, [P]),
    "lq_tune": (I, [P, I, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_size_t, P]),
    "lq_bandwidth_probe": (I, [I, P, P, ctypes.c_size_t, I, ctypes.POINTER(D), P]),
    "lq_pf_force": (I,[P, ctypes.POINTER(SolverParams), I, I, P, P, P, P, ctypes.POINTER(D),
                        ctypes.POINTER(SolveStats), P]),
    "lq_eig_params_default": (None, [ctypes.POINTER(EigParams)]),
    "lq_deflated_guess": (I, [P, I, ctypes.POINTER(D), P, P, P, P]),
    "lq_op_set_deflation": (I, [P, I, ctypes.POINTER(D), P, P]),
    "lq_mg_params_default": (None, [ctypes.POINTER(MGParams)]),
    "lq_mg_create": (I, [P, ctypes.POINTER(MGParams), P, ctypes.POINTER(P), P]),
    "lq_mg_destroy": (I, [P]),
    "lq_mg_solve": (I, [P, ctypes.POINTER(SolverParams), P, P, ctypes.POINTER(SolveStats), P]),
    "lq_mg_vectors": (I, [P, P, P]),
    "lq_mg_coarse_op": (I, [P, ctypes.POINTER(D)]),
    "lq_mg_restrict": (I, [P, P, P, P]),
    "lq_mg_prolong": (I, [P, P, P, P]),
    "lq_mg_coarse_apply": (I, [P, P, P, P]),
    "lq_eigs": (I, [P, ctypes.POINTER(EigParams), P, ctypes.POINTER(D), ctypes.POINTER(D), P,
                    ctypes.POINTER(EigStats), P]),
    "lq_md_params_default": (None, [ctypes.POINTER(MDParams)]),
    "lq_gauge_force": (I, [P, D, P, ctypes.POINTER(D), P]),
    "lq_md_trajectory": (I, [P, ctypes.POINTER(MDParams), ctypes.POINTER(SolverParams), P, P, P,
                             ctypes.POINTER(MDStats), P]),
}

_LIB = None


def load() -> ctypes.CDLL:
    """Load liblq.so and declare every entry point; raises if it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblq.so is not built (run __graft_entry__.build() or "
                               "python paper_2111_04457_amd/build.py); there is no fallback path")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


class LQError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def check(status: int, allow_not_converged: bool = False) -> int:
    if status == LQ_OK or (allow_not_converged and status == LQ_NOT_CONVERGED):
        return status
    msg = load().lq_last_error()
    raise LQError(status, msg.decode() if msg else "")
