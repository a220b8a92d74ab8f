"""ctypes loader for librmh.so (the HIP library built for gfx950).

There is no fallback: if the library or a GPU is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librmh.so")

RMH_OK = 0
STATUS_NAMES = {
    0: "RMH_OK", 1: "RMH_E_ARG", 2: "RMH_E_SHAPE", 3: "RMH_E_WORKSPACE", 4: "RMH_E_POLES",
    5: "RMH_E_NOCONV", 6: "RMH_E_BREAKDOWN", 7: "RMH_E_HIP", 8: "RMH_E_UNIMPLEMENTED", 9: "RMH_E_HOST",
}

RMH_F64, RMH_F32 = 0, 1
OP_LAPLACIAN, OP_LAPLACIAN_BWD, OP_POWER_SPECTRUM, OP_CHEB_FILTER = 0, 1, 2, 3
OP_RATIONAL_APPLY, OP_RATIONAL_APPLY_BWD, OP_KINETIC_FORCE = 4, 5, 6
OP_CHEB_FILTER_BWD, OP_POWER_SPECTRUM_BWD, OP_GAUGE_FORCE, OP_HEATBATH, OP_LEAPFROG = 7, 8, 9, 10, 11
OP_AUTOTUNE = 12

c_i32, c_i64, c_f64, c_sz, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
P_i32 = ctypes.POINTER(c_i32)
P_f64 = ctypes.POINTER(c_f64)


class RmhCheb(ctypes.Structure):
    _fields_ = [("degree", c_i32), ("n_windows", c_i32), ("edges", P_f64), ("kernel", c_i32)]


class RmhRational(ctypes.Structure):
    _fields_ = [("c", c_f64), ("n_poles", c_i32), ("r", P_f64), ("sigma", P_f64)]


class RmhSolver(ctypes.Structure):
    _fields_ = [("tol", c_f64), ("maxiter", c_i32), ("mode", c_i32), ("delta", c_f64), ("check_every", c_i32),
                ("mixed_switch", c_f64), ("basis", c_i32), ("multishift_target", c_f64)]


class RmhHopConfig(ctypes.Structure):
    _fields_ = [("form", c_i32), ("block", c_i32), ("xcd_remap", c_i32), ("nv", c_i32), ("order", c_i32),
                ("walk", c_i32), ("ns", c_i32), ("tile2", c_i32)]

    def as_tuple(self):
        return tuple(getattr(self, k) for k, _ in self._fields_)


class RmhStats(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("reliable_updates", c_i32), ("refine_iters", c_i32),
                ("refine_rounds", c_i32), ("fp64_iters", c_i32), ("reserved", c_i32),
                ("true_relres_max", c_f64), ("seconds", c_f64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes)
class RmhLeapfrog(ctypes.Structure):
    _fields_ = [("eps", c_f64), ("beta", c_f64), ("fp_tol", c_f64), ("fp_maxiter", c_i32)]


class RmhLeapfrogStats(ctypes.Structure):
    _fields_ = [("p_iters", c_i32), ("u_iters", c_i32), ("p_res", c_f64), ("u_res", c_f64), ("solver", RmhStats)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "solver"}
        d["solver"] = self.solver.as_dict()
        return d


SIGNATURES = {
    "rmh_last_error": (ctypes.c_char_p, []),
    "rmh_version": (c_i32, []),
    "rmh_workspace_bytes": (c_sz, [c_i32, P_i32, c_i32, c_i32, c_i32, c_i32, c_i32]),
    "rmh_pack_links": (c_i32, [P_i32, c_vp, c_vp, c_i32, c_vp]),
    "rmh_unpack_links": (c_i32, [P_i32, c_vp, c_vp, c_vp]),
    "rmh_pack_fields": (c_i32, [P_i32, c_i32, c_vp, c_vp, c_i32, c_vp]),
    "rmh_unpack_fields": (c_i32, [P_i32, c_i32, c_vp, c_i32, c_vp, c_vp]),
    "rmh_convert_f64_f32": (c_i32, [c_vp, c_vp, c_i64, c_vp]),
    "rmh_laplacian_apply": (c_i32, [P_i32, c_vp, c_i32, c_vp, c_vp, c_i32, c_f64, c_vp]),
    "rmh_laplacian_apply_bwd": (c_i32, [P_i32, c_vp, c_i32, c_vp, c_vp, c_i32, c_f64, c_vp, c_vp, c_i32, c_vp]),
    "rmh_cheb_coefficients": (c_i32, [ctypes.POINTER(RmhCheb), P_f64]),
    "rmh_power_spectrum": (c_i32, [P_i32, c_vp, c_i32, c_vp, c_i32, ctypes.POINTER(RmhCheb), P_f64, P_f64,
                                   c_vp, c_sz, c_vp]),
    "rmh_power_spectrum_noalloc": (c_i32, [P_i32, c_vp, c_i32, c_vp, c_i32, ctypes.POINTER(RmhCheb), P_f64, P_f64,
                                           c_vp]),
    "rmh_power_ratio": (c_i32, [ctypes.POINTER(RmhCheb), P_f64, P_f64, c_i32, P_f64]),
    "rmh_trace_moments_free": (c_i32, [P_i32, c_i32, P_f64]),
    "rmh_cheb_filter": (c_i32, [P_i32, c_vp, c_i32, c_vp, c_i32, ctypes.POINTER(RmhCheb), c_vp, c_vp, c_sz, c_vp]),
    "rmh_cheb_filter_bwd": (c_i32, [P_i32, c_vp, c_vp, c_vp, c_i32, ctypes.POINTER(RmhCheb), c_vp, c_vp, c_i32,
                                    c_vp, c_sz, c_vp]),
    "rmh_heatbath_momenta": (c_i32, [P_i32, c_vp, c_vp, c_i32, c_f64, ctypes.POINTER(RmhRational),
                                     ctypes.POINTER(RmhSolver), c_vp, ctypes.POINTER(RmhStats), c_vp, c_sz, c_vp]),
    "rmh_wilson_gauge_force": (c_i32, [P_i32, c_vp, c_f64, c_vp, P_f64, c_vp, c_sz, c_vp]),
    "rmh_power_spectrum_bwd": (c_i32, [P_i32, c_vp, c_vp, c_i32, ctypes.POINTER(RmhCheb), P_f64, c_vp, c_vp,
                                       c_i32, c_vp, c_sz, c_vp]),
    "rmh_rational_from_quadratics": (c_i32, [c_i32, P_f64, P_f64, P_f64, P_f64, P_f64, P_f64]),
    "rmh_rational_kappa": (c_i32, [c_f64, c_i32, P_f64, P_f64, P_f64]),
    "rmh_rational_apply": (c_i32, [P_i32, c_vp, c_vp, c_i32, ctypes.POINTER(RmhRational),
                                   ctypes.POINTER(RmhSolver), c_vp, c_vp, P_f64, ctypes.POINTER(RmhStats),
                                   c_vp, c_sz, c_vp]),
    "rmh_rational_apply_bwd": (c_i32, [P_i32, c_vp, c_vp, c_vp, c_i32, ctypes.POINTER(RmhRational),
                                       ctypes.POINTER(RmhSolver), c_vp, c_vp, c_i32, ctypes.POINTER(RmhStats),
                                       c_vp, c_sz, c_vp]),
    "rmh_link_exp": (c_i32, [P_i32, c_vp, c_vp, c_vp, c_vp]),
    "rmh_link_exp_vjp": (c_i32, [P_i32, c_vp, c_vp, c_vp, c_vp]),
    "rmh_tune_set": (c_i32, [P_i32, c_i32, c_i32, c_i32, ctypes.POINTER(RmhHopConfig)]),
    "rmh_autotune_laplacian": (c_i32, [P_i32, c_vp, c_i32, c_vp, c_vp, c_i32, c_i32, c_i32,
                                       ctypes.POINTER(RmhHopConfig), P_f64, c_vp, c_sz, c_vp]),
    "rmh_tune_save": (c_i32, [ctypes.c_char_p, P_i32]),
    "rmh_tune_load": (c_i32, [ctypes.c_char_p, P_i32]),
    "rmh_tune_clear": (c_i32, []),
    "rmh_profile_enable": (c_i32, [c_i32]),
    "rmh_profile_read": (c_i32, [c_i32, ctypes.POINTER(c_i64), P_f64, P_f64, P_f64]),
    "rmh_kinetic_force": (c_i32, [P_i32, c_vp, c_vp, c_i32, ctypes.POINTER(RmhRational),
                                  ctypes.POINTER(RmhSolver), c_vp, P_f64, c_vp, c_i32,
                                  ctypes.POINTER(RmhStats), c_vp, c_sz, c_vp]),
    "rmh_leapfrog_step": (c_i32, [P_i32, c_vp, c_vp, ctypes.POINTER(RmhRational), ctypes.POINTER(RmhSolver),
                                  ctypes.POINTER(RmhLeapfrog), c_vp, c_vp, ctypes.POINTER(RmhLeapfrogStats),
                                  c_vp, c_sz, c_vp]),
}

_lib = None


class RmhError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        self.status = status
        super().__init__(f"{func} -> {STATUS_NAMES.get(status, status)}: {msg}")


def lib():
    """The loaded library; raises if librmh.so has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2112_04556_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, func: str) -> None:
    if status != RMH_OK:
        raise RmhError(status, func, lib().rmh_last_error().decode())


def lattice_arg(L):
    arr = (c_i32 * 4)(*[int(v) for v in L])
    return arr
