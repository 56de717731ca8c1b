"""Loading of the in-tree HIP library (liblhmm.so) and its C signatures.

The library is built by ``paper_2512_13267_amd.build`` (hipcc, gfx950).  There
is no fallback: if the library is missing or fails to load, every entry point
raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblhmm.so")

LHMM_OK = 0
LHMM_ERR_ARG = -1
LHMM_ERR_HIP = -2
LHMM_ERR_OOM = -3
LHMM_ERR_STATE = -4

FLAG_BOND = 1
FLAG_CELL = 2
FLAG_NONFINITE = 4
FLAG_ARG = 8
FLAG_THIN = 16
THIN_WIDTH = 3.3

FP32 = 0
FP64 = 1
OPT_NO_GRAPH = 1
OPT_COMPONENTS = 2
CELL_KINDS = {0: "cubic", 1: "kr", 2: "rotated"}

# every symbol include/lhmm.h declares
EXPORTS = (
    "lhmm_micro_create", "lhmm_micro_set_state", "lhmm_micro_get_state", "lhmm_micro_step",
    "lhmm_micro_forces", "lhmm_micro_stress_parts", "lhmm_micro_pair_counts", "lhmm_micro_flags",
    "lhmm_micro_sizes", "lhmm_micro_destroy", "lhmm_last_error", "lhmm_micro_time",
    "lhmm_micro_step_subset", "lhmm_micro_snapshot", "lhmm_micro_restore",
    "lhmm_micro_set_config", "lhmm_micro_get_config", "lhmm_micro_autotune",
    "lhmm_micro_components", "lhmm_micro_pair_total", "lhmm_micro_prepare", "lhmm_box_cell",
    "lhmm_micro_set_afbc",
    "lhmm_sph_create", "lhmm_sph_step", "lhmm_sph_get_state", "lhmm_sph_coupling_state", "lhmm_couple_step",
    "lhmm_sph_destroy",
    "lhmm_sur_create", "lhmm_sur_set_weights", "lhmm_sur_get_weights", "lhmm_sur_get_grads", "lhmm_sur_train_step", "lhmm_sur_forward",
    "lhmm_sur_forward_static",
    "lhmm_sur_push_history", "lhmm_sur_features", "lhmm_sur_gate", "lhmm_sur_destroy", "lhmm_sur_targets",
    "lhmm_sur_blend", "lhmm_sur_history_gradient", "lhmm_sur_augment",
    "lhmm_hybrid_create", "lhmm_hybrid_step", "lhmm_hybrid_state", "lhmm_hybrid_destroy", "lhmm_hybrid_mean_stress",
)
SUR_HIST = 32
SUR_FEATURES = 4 * SUR_HIST + 1
KERNEL_NAMES = ("cell_step", "kick_drift", "bin_box", "forces", "kick2", "box_stress")


class LhmmParams(C.Structure):
    _fields_ = [("a", C.c_double), ("gamma", C.c_double), ("sigma", C.c_double), ("kBT", C.c_double),
                ("mass", C.c_double), ("rc", C.c_double), ("dt", C.c_double), ("H", C.c_double),
                ("R0", C.c_double), ("seed", C.c_uint64), ("chain_len", C.c_int32),
                ("precision", C.c_int32), ("flags", C.c_int32)]


class LhmmBox(C.Structure):
    _fields_ = [("n_particles", C.c_int32), ("n_chains", C.c_int32), ("rng_id", C.c_uint32),
                ("reserved", C.c_int32), ("h0", C.c_double * 9)]


class LhmmSphParams(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("rho0", "eta", "zeta", "c", "theta", "F", "h", "dt", "mass", "Lx", "Ly",
                                            "lambda_star", "alpha")] + [("n_fixed", C.c_int32),
                                                                        ("force_mode", C.c_int32),
                                                                        ("kernel", C.c_int32),
                                                                        ("micro_dim", C.c_int32)]


class LhmmMicroConfig(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("queue_depth", "drain", "busy_lanes", "bin_threads", "graph_chunk", "prune", "fuse_bin",
                                         "groups", "bin_split")]


class LhmmSurParams(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("n_members", "n_in", "n_hidden", "n_out", "max_batch")]


class LhmmHybridParams(C.Structure):
    _fields_ = [("mode", C.c_int32), ("k_micro", C.c_int32), ("hold", C.c_int32), ("replay", C.c_int32),
                ("threshold", C.c_float), ("floor", C.c_float), ("grad_scale", C.c_float),
                ("stress_scale", C.c_float), ("max_grad", C.c_float), ("warm_frac", C.c_float)]


class LhmmHybridStats(C.Structure):
    _fields_ = [("macro_step", C.c_int64), ("micro_box_steps", C.c_int64), ("n_dpd", C.c_int32),
                ("n_entered", C.c_int32), ("n_flagged", C.c_int32), ("n_reset", C.c_int32),
                ("n_out_of_range", C.c_int32), ("n_warm", C.c_int32)]


HYBRID_SURROGATE = 0
HYBRID_DPD = 1


class LhmmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lhmm error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2512_13267_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, dp, u64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)
        L.lhmm_micro_create.argtypes = [C.POINTER(LhmmParams), C.POINTER(LhmmBox), C.c_int32, vp, C.POINTER(vp)]
        L.lhmm_micro_set_state.argtypes = [vp, dp, dp, dp, dp, C.c_uint64]
        L.lhmm_micro_get_state.argtypes = [vp, dp, dp, dp, dp, u64p]
        L.lhmm_micro_step.argtypes = [vp, vp, C.c_int32, vp]
        i32p = C.POINTER(C.c_int32)
        L.lhmm_micro_step_subset.argtypes = [vp, vp, C.c_int32, vp, i32p, C.c_int32]
        L.lhmm_micro_snapshot.argtypes = [vp]
        L.lhmm_micro_set_config.argtypes = [vp, C.POINTER(LhmmMicroConfig)]
        L.lhmm_micro_get_config.argtypes = [vp, C.POINTER(LhmmMicroConfig)]
        L.lhmm_micro_autotune.argtypes = [vp, vp, C.c_int32, C.POINTER(LhmmMicroConfig), dp]
        L.lhmm_micro_restore.argtypes = [vp, i32p, C.c_int32]
        L.lhmm_micro_forces.argtypes = [vp, dp, dp, dp]
        L.lhmm_micro_stress_parts.argtypes = [vp, dp]
        L.lhmm_micro_pair_counts.argtypes = [vp, u64p]
        L.lhmm_micro_pair_total.argtypes = [vp, u64p]
        L.lhmm_micro_components.argtypes = [vp, dp]
        L.lhmm_micro_prepare.argtypes = [vp, C.c_int32]
        L.lhmm_micro_set_afbc.argtypes = [vp, dp, C.c_double]
        L.lhmm_box_cell.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp, C.POINTER(C.c_int32)]
        L.lhmm_micro_flags.argtypes = [vp, C.POINTER(C.c_uint32), C.c_int32]
        L.lhmm_micro_sizes.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        L.lhmm_micro_destroy.argtypes = [vp]
        L.lhmm_micro_time.argtypes = [vp, vp, C.c_int32, dp, vp]
        L.lhmm_sph_create.argtypes = [C.POINTER(LhmmSphParams), C.c_int32, dp, dp, vp, C.POINTER(vp)]
        L.lhmm_sph_step.argtypes = [vp, vp, vp]
        L.lhmm_sph_get_state.argtypes = [vp, dp, dp, dp]
        L.lhmm_sph_coupling_state.argtypes = [vp, dp, dp]
        L.lhmm_couple_step.argtypes = [vp, vp, C.c_int32, C.c_int32]
        L.lhmm_sph_destroy.argtypes = [vp]
        fp = C.POINTER(C.c_float)
        L.lhmm_sur_create.argtypes = [C.POINTER(LhmmSurParams), fp, vp, C.POINTER(vp)]
        L.lhmm_sur_set_weights.argtypes = [vp, fp]
        L.lhmm_sur_get_weights.argtypes = [vp, fp]
        L.lhmm_sur_get_grads.argtypes = [vp, fp]
        L.lhmm_sur_train_step.argtypes = [vp, vp, vp, C.c_int32, C.c_float, vp]
        L.lhmm_sur_forward.argtypes = [vp, vp, C.c_int32, vp]
        L.lhmm_sur_forward_static.argtypes = [vp, vp, C.c_int32, vp]
        L.lhmm_sur_push_history.argtypes = [vp, C.c_int32, vp, C.c_int64, C.c_float, vp]
        L.lhmm_sur_augment.argtypes = [vp, vp, C.c_int32, vp, vp, vp]
        L.lhmm_sur_targets.argtypes = [vp, C.c_int32, C.c_float, vp, vp]
        L.lhmm_sur_blend.argtypes = [vp, vp, vp, C.c_int32, C.c_float, vp, vp]
        L.lhmm_sur_history_gradient.argtypes = [vp, C.c_int32, C.c_int64, C.c_float, vp, vp]
        L.lhmm_sur_features.argtypes = [vp, C.c_int32, C.c_int64, vp, vp, vp]
        L.lhmm_sur_gate.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_float, vp, vp, vp]
        L.lhmm_sur_destroy.argtypes = [vp]
        L.lhmm_hybrid_create.argtypes = [C.POINTER(LhmmHybridParams), vp, vp, vp, fp, C.POINTER(vp)]
        L.lhmm_hybrid_step.argtypes = [vp, C.POINTER(LhmmHybridStats)]
        L.lhmm_hybrid_state.argtypes = [vp, dp, C.POINTER(C.c_uint32)]
        L.lhmm_hybrid_destroy.argtypes = [vp]
        L.lhmm_hybrid_mean_stress.argtypes = [vp, dp, C.c_int32]
        L.lhmm_last_error.restype = C.c_char_p
        for name in EXPORTS:
            if name != "lhmm_last_error":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def check(code: int) -> None:
    if code != LHMM_OK:
        msg = lib().lhmm_last_error().decode(errors="replace")
        raise LhmmError(code, msg)
