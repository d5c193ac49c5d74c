"""ctypes binding of libmpm.so (include/mpm.h).  Marshalling only: every step
of the simulation runs in the library's HIP kernels.  There is no fallback:
if the library is missing this raises."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmpm.so")

MPM_OK = 0
ERR_NAMES = {-1: "MPM_ERR_ARG", -2: "MPM_ERR_OOM", -3: "MPM_ERR_DOMAIN",
             -4: "MPM_ERR_INVERTED", -5: "MPM_ERR_NONFINITE", -6: "MPM_ERR_HIP",
             -7: "MPM_ERR_STATE"}


class MPMError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = lib().mpm_strerror(code).decode() if _lib is not None else ""
        super().__init__(f"{ERR_NAMES.get(code, code)} ({msg}) {what}".strip())
        self.code = code


class Scene(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_grid", ctypes.c_int32),
                ("n_particles", ctypes.c_int32), ("n_act", ctypes.c_int32),
                ("wall", ctypes.c_int32), ("bc", ctypes.c_int32),
                ("dt", ctypes.c_float), ("E", ctypes.c_float),
                ("nu", ctypes.c_float), ("rho", ctypes.c_float),
                ("V0", ctypes.c_float), ("gravity", ctypes.c_float * 3),
                ("act_axis", ctypes.c_float * 3), ("friction", ctypes.c_float)]


class Opts(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("sort", ctypes.c_int32),
                ("scatter", ctypes.c_int32), ("recompute_grids", ctypes.c_int32),
                ("graphs", ctypes.c_int32), ("fusion", ctypes.c_int32),
                ("deterministic", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("rebin", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


class State(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("v", ctypes.c_void_p),
                ("C", ctypes.c_void_p), ("F", ctypes.c_void_p)]


class Controller(ctypes.Structure):
    _fields_ = [("n_comp", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("comp_id", ctypes.c_void_p), ("W", ctypes.c_void_p),
                ("b", ctypes.c_void_p), ("target", ctypes.c_void_p)]


EXPORTS = ["mpm_init", "mpm_destroy", "mpm_set_stream", "mpm_info",
           "mpm_step_forward", "mpm_step_backward", "mpm_rollout",
           "mpm_rollout_backward", "mpm_get_grid", "mpm_act_bank_forward",
           "mpm_act_bank_backward", "mpm_sync_errors", "mpm_strerror",
           "mpm_profile", "mpm_profile_read", "mpm_rollout_ctrl",
           "mpm_rollout_ctrl_backward", "mpm_revolve_steps", "mpm_revolve_split",
           "mpm_set_materials", "mpm_material_grad", "mpm_tape_generation",
           "mpm_step_forward_noalloc", "mpm_set_horizons", "mpm_tape_binnings"]

KERNELS = ["p2g", "grid", "g2p", "adj_scatter", "adj_grid", "adj_gather", "g2p_p2g",
           "adj_fused"]

_lib = None


def lib():
    """Load libmpm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -m paper_1810_01054_amd.build` (no fallback path exists)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64p = ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64)
    sp = ctypes.POINTER(State)
    L.mpm_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Scene), i32,
                           ctypes.POINTER(ctypes.c_int32), vp, ctypes.POINTER(Opts)]
    L.mpm_destroy.argtypes = [vp]
    L.mpm_destroy.restype = None
    L.mpm_set_stream.argtypes = [vp, vp]
    L.mpm_info.argtypes = [vp, i64p, ctypes.POINTER(ctypes.c_int32), i64p]
    L.mpm_step_forward.argtypes = [vp, sp, vp, sp]
    L.mpm_step_backward.argtypes = [vp, sp, vp, sp, sp, vp]
    L.mpm_step_forward_noalloc.argtypes = [ctypes.POINTER(Scene), vp, sp, vp, sp, vp, vp]
    L.mpm_rollout.argtypes = [vp, i32, i32, sp, vp, sp, sp, sp, vp]
    L.mpm_rollout_backward.argtypes = [vp, sp, sp, vp]
    L.mpm_rollout_ctrl.argtypes = [vp, i32, i32, sp, ctypes.POINTER(Controller), sp, vp,
                                   sp, sp, vp, vp, vp]
    L.mpm_rollout_ctrl_backward.argtypes = [vp, sp, sp, vp, vp, vp]
    L.mpm_set_materials.argtypes = [vp, vp, vp]
    L.mpm_set_horizons.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.mpm_material_grad.argtypes = [vp, vp, vp]
    L.mpm_tape_generation.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    L.mpm_tape_binnings.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.mpm_revolve_steps.argtypes = [ctypes.c_int64, ctypes.c_int32]
    L.mpm_revolve_steps.restype = ctypes.c_int64
    L.mpm_revolve_split.argtypes = [ctypes.c_int64, ctypes.c_int32]
    L.mpm_revolve_split.restype = ctypes.c_int64
    L.mpm_get_grid.argtypes = [vp, vp, vp, vp]
    L.mpm_act_bank_forward.argtypes = [vp, i32, i32, i32, ctypes.c_float,
                                       vp, vp, vp, vp]
    L.mpm_act_bank_backward.argtypes = [vp, i32, i32, i32, ctypes.c_float,
                                        vp, vp, vp, vp, vp, vp]
    L.mpm_sync_errors.argtypes = [vp]
    L.mpm_profile.argtypes = [vp, ctypes.c_uint32]
    L.mpm_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_int64),
                                   ctypes.POINTER(ctypes.c_double)]
    L.mpm_strerror.argtypes = [i32]
    L.mpm_strerror.restype = ctypes.c_char_p
    _lib = L
    return L


def check(rc: int, what: str = ""):
    if rc != MPM_OK:
        raise MPMError(rc, what)
