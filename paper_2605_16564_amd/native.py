"""ctypes binding of the C ABI in include/pam.h (argument marshalling only).

Every computation runs in libpam.so's HIP kernels; this module only lays out
the C structs and forwards device pointers. Loading fails loudly when the
library has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

LIB_PATH = Path(os.environ.get("PAM_LIB", str(Path(__file__).resolve().parent / "_build" / "libpam.so")))

PAM_OK = 0
PREC = {"f64": 0, "f32": 1, "bf16": 2}
ST_OK, ST_NOCONV, ST_UNDERFLOW, ST_EMPTY, ST_NONFINITE = 0, 1, 2, 3, 4
ERR_NONFINITE = -3

EXPORTS = [
    "pam_create", "pam_destroy", "pam_set_stream", "pam_sync", "pam_last_error", "pam_version",
    "pam_partition_count", "pam_partition_gather", "pam_init_lattice", "pam_fit_subdomains", "pam_refit_nonconverged",
    "pam_refine", "pam_eval", "pam_timing_enable", "pam_timing_read",
    "pam_cnn_param_count", "pam_cnn_forward", "pam_cnn_loss_grad", "pam_cnn_adam",
    "pam_grid_patches", "pam_support_hint", "pam_cnn_labels",
    "pam_eval_blend", "pam_interface_count", "pam_interface_jump", "pam_select_lambda",
    "pam_darcy_solve", "pam_darcy_error", "pam_darcy_coefficient", "pam_darcy_coefficient_cells",
    "pam_eval_noalloc", "pam_graph_enable", "pam_gram_path",
]
TIMING_KINDS = ["gather", "lattice", "assemble", "gram", "solve", "indicator", "mark",
                "eval_bin", "eval", "cnn", "blend", "jump",
                "darcy"]


class PamGrid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_cells", C.c_int32 * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("n_sub", C.c_int32 * 3), ("breaks", C.c_void_p),
                ("overlap", C.c_double)]


class PamDict(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("dim", C.c_int32), ("m_cap", C.c_int32),
                ("m", C.c_void_p), ("c", C.c_void_p), ("sigma", C.c_void_p),
                ("level", C.c_void_p), ("basis", C.c_int32)]

BASIS = {"shepard": 0, "plain": 1}


class PamSamples(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_sub", C.c_int32), ("n_max", C.c_int32),
                ("off", C.c_void_p), ("off_host", C.c_void_p), ("x", C.c_void_p),
                ("y", C.c_void_p), ("h", C.c_void_p)]


class PamEnetOpts(C.Structure):
    _fields_ = [("lambda1", C.c_double), ("lambda2", C.c_double),
                ("lambda1_sub", C.c_void_p), ("lambda2_sub", C.c_void_p),
                ("precision", C.c_int32), ("cd_sweeps", C.c_int32), ("max_iter", C.c_int32),
                ("warm_start", C.c_int32), ("batched", C.c_int32),
                ("support_hint", C.c_void_p), ("team", C.c_int32), ("team_min", C.c_int32),
                ("team_idle_us", C.c_int32)]


class PamFitStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("cd_sweeps", C.c_int32), ("iters", C.c_int32),
                ("support", C.c_int32), ("kkt", C.c_double), ("stream_bytes", C.c_double),
                ("polish", C.c_int32), ("team", C.c_int32), ("solve_us", C.c_double)]


class PamRefineOpts(C.Structure):
    _fields_ = [("k_top", C.c_int32), ("k_top_sub", C.c_void_p), ("max_rounds", C.c_int32),
                ("m_max", C.c_int32), ("eta", C.c_double), ("eps_tol", C.c_double),
                ("space", C.c_int32), ("elem_level", C.c_void_p), ("rounds", C.c_void_p),
                ("round_stats", C.c_void_p), ("cold_rounds", C.c_int32)]


class PamSelectOpts(C.Structure):
    _fields_ = [("n_alpha", C.c_int32), ("k_folds", C.c_int32), ("alpha_min_ratio", C.c_double),
                ("l1_ratio", C.c_double)]


class PamDarcyOpts(C.Structure):
    _fields_ = [("n", C.c_int32 * 2), ("lo", C.c_double * 2), ("hi", C.c_double * 2),
                ("p_left", C.c_double), ("p_right", C.c_double), ("tol", C.c_double),
                ("max_iter", C.c_int32), ("check_every", C.c_int32)]


class PamField(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_sub_axis", C.c_int32 * 3), ("axis_x", C.c_void_p),
                ("sub_base", C.c_int32), ("q_begin", C.c_int64), ("q_end", C.c_int64)]


STATS_BYTES = C.sizeof(PamFitStats)

_lib = None


class PamError(RuntimeError):
    def __init__(self, msg, status=None):
        super().__init__(msg)
        self.status = status


def lib():
    """Load libpam.so (built by paper_2605_16564_amd.build); raise if absent."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise PamError(f"{LIB_PATH} is not built; run python -m paper_2605_16564_amd.build first")
        L = C.CDLL(str(LIB_PATH))
        P = C.c_void_p
        L.pam_create.argtypes = [C.POINTER(P), C.c_int]
        L.pam_destroy.argtypes = [P]
        L.pam_set_stream.argtypes = [P, P]
        L.pam_sync.argtypes = [P]
        L.pam_last_error.restype = C.c_char_p
        L.pam_last_error.argtypes = []
        L.pam_version.restype = C.c_char_p
        L.pam_version.argtypes = []
        L.pam_partition_count.argtypes = [C.POINTER(PamGrid), P, P]
        L.pam_partition_gather.argtypes = [P, C.POINTER(PamGrid), P, P, P, P, P, P]
        L.pam_init_lattice.argtypes = [P, C.POINTER(PamGrid), P, C.c_double, C.POINTER(PamDict)]
        L.pam_fit_subdomains.argtypes = [P, C.POINTER(PamSamples), C.POINTER(PamDict),
                                         C.POINTER(PamEnetOpts), P, P]
        L.pam_refit_nonconverged.argtypes = [P, C.POINTER(PamSamples), C.POINTER(PamDict),
                                             C.POINTER(PamEnetOpts), P, P]
        L.pam_refine.argtypes = [P, C.POINTER(PamSamples), C.POINTER(PamDict), P,
                                 C.POINTER(PamEnetOpts), C.POINTER(PamRefineOpts), P]
        L.pam_eval.argtypes = [P, C.c_int32, C.POINTER(PamField), C.POINTER(PamDict), P, C.c_int32,
                               P, C.c_int64, P, C.c_int32, P]
        L.pam_eval_noalloc.argtypes = [P, C.c_int32, C.POINTER(PamField), C.POINTER(PamDict), P,
                                       C.c_int32, P, C.c_int64, P, C.c_int32, P]
        L.pam_eval_blend.argtypes = [P, C.c_int32, C.POINTER(PamField), C.POINTER(PamDict), P,
                                     C.c_double, C.c_int32, P, C.c_int64, P, C.c_int32, P]
        L.pam_interface_count.argtypes = [C.c_int32, C.POINTER(PamField)]
        L.pam_interface_jump.argtypes = [P, C.c_int32, C.POINTER(PamField), C.POINTER(PamDict), P,
                                         C.c_int32, P]
        L.pam_select_lambda.argtypes = [P, C.POINTER(PamSamples), C.POINTER(PamDict),
                                        C.POINTER(PamEnetOpts), C.POINTER(PamSelectOpts), P, P, P,
                                        P, P, P]
        L.pam_darcy_solve.argtypes = [P, C.POINTER(PamDarcyOpts), P, P, C.c_int32, P, P]
        L.pam_darcy_error.argtypes = [P, C.POINTER(PamDarcyOpts), P, P, P]
        L.pam_darcy_coefficient.argtypes = [P, C.POINTER(PamDarcyOpts), C.POINTER(PamField),
                                            C.POINTER(PamDict), P, C.c_double, P]
        L.pam_darcy_coefficient_cells.argtypes = [P, C.POINTER(PamDarcyOpts), P, P]
        L.pam_timing_enable.argtypes = [P, C.c_int32]
        L.pam_graph_enable.argtypes = [P, C.c_int32]
        L.pam_gram_path.argtypes = [P, C.c_int32]
        L.pam_timing_read.argtypes = [P, P, P, C.c_int32]
        L.pam_cnn_param_count.argtypes = []
        L.pam_cnn_forward.argtypes = [P, P, C.c_int32, P, P, C.c_int32]
        L.pam_cnn_loss_grad.argtypes = [P, P, C.c_int32, P, P, P, P, P, C.c_int32]
        L.pam_cnn_adam.argtypes = [P, P, P, P, P, C.c_int32, C.c_float, C.c_float, C.c_float,
                                   C.c_float]
        L.pam_grid_patches.argtypes = [P, C.POINTER(PamGrid), P, C.c_float, P, P]
        L.pam_support_hint.argtypes = [P, C.POINTER(PamGrid), C.POINTER(PamDict), P, C.c_float, P]
        L.pam_cnn_labels.argtypes = [P, C.POINTER(PamGrid), C.POINTER(PamSamples),
                                     C.POINTER(PamDict), P, P, P, P]
        for name in EXPORTS:
            if name not in ("pam_last_error", "pam_version"):
                getattr(L, name).restype = C.c_int
        L.pam_cnn_param_count.restype = C.c_int64
        L.pam_interface_count.restype = C.c_int64
        _lib = L
    return _lib


def check(status: int, what: str):
    if status != PAM_OK:
        msg = lib().pam_last_error().decode(errors="replace")
        raise PamError(f"{what} failed with status {status}: {msg}", status)
