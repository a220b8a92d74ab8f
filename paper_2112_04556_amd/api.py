"""Python binding of the C ABI (argument marshalling only).

Every function takes and returns torch tensors on the GPU (device memory and the
current stream come from PyTorch); all arithmetic runs in the HIP library.  Names
follow the C entry points without the ``rmh_`` prefix.  Layouts are those of
``include/rmh.h``: links SoA (4, 18, V), link fields SoA (n, 4, 8, V).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib as L_
from ._lib import RMH_F32, RMH_F64, check, lattice_arg, lib

__all__ = [
    "Rational", "Solver", "pack_links", "unpack_links", "pack_fields", "unpack_fields", "convert_f64_f32",
    "laplacian_apply", "laplacian_apply_bwd", "cheb_coefficients", "power_spectrum", "power_ratio",
    "trace_moments_free", "cheb_filter", "power_spectrum_noalloc", "rational_from_quadratics", "rational_kappa", "rational_apply",
    "rational_apply_bwd", "kinetic_force", "workspace_bytes", "volume", "tune_set", "tune_clear", "link_exp", "link_exp_vjp",
    "autotune_laplacian", "tune_save", "tune_load", "PURPOSES", "profile_enable", "profile_read", "PROF_CLASSES",
]


def volume(L) -> int:
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return RMH_F64
    if t.dtype == torch.float32:
        return RMH_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev(t: torch.Tensor, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _f64p(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(L_.P_f64)


@dataclass
class Rational:
    """R(Delta) = c + sum_j r_j / (Delta + sigma_j) (Delta units)."""
    c: float
    r: np.ndarray
    sigma: np.ndarray

    def c_struct(self):
        self._r = np.ascontiguousarray(self.r, dtype=np.float64)
        self._s = np.ascontiguousarray(self.sigma, dtype=np.float64)
        return L_.RmhRational(float(self.c), len(self._r), _f64p(self._r), _f64p(self._s))


@dataclass
class Solver:
    tol: float = 1e-10
    maxiter: int = 20000
    mode: int = 0          # 0 = FP64, 1 = FP64 then FP32 with FP64 reliable updates
    delta: float = 0.01         # reliable update once the seed residual fell 100-fold since the last
    check_every: int = 8
    mixed_switch: float = 0.0   # 0: library default (1e-4); < 0: FP32 from the first iteration
    basis: int = 0              # iterations per shift-solution segment (0: library default)
    multishift_target: float = 0.0   # multi-shift stop at this multiple of tol (0: 0.5); > 1 forces refinement

    def c_struct(self):
        return L_.RmhSolver(self.tol, self.maxiter, self.mode, self.delta, self.check_every, self.mixed_switch,
                            self.basis, self.multishift_target)


def workspace_bytes(op: int, L, dtype: int, n_rhs: int, aux: int = 0, degree: int = 0, mode: int = 0) -> int:
    n = lib().rmh_workspace_bytes(op, lattice_arg(L), dtype, n_rhs, aux, degree, mode)
    if n == 0:
        check(L_.RMH_E_ARG, "rmh_workspace_bytes")
    return int(n)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


# ------------------------------------------------------------------------------------------
# layout

def pack_links(L, U: torch.Tensor, dtype=torch.float64) -> torch.Tensor:
    """SoA links (4, 18, V) of the given dtype from complex links (4, V, 3, 3)."""
    V = volume(L)
    aos = torch.view_as_real(U.to(torch.complex128)).contiguous()
    if aos.shape != (4, V, 3, 3, 2):
        raise ValueError(f"links must have shape (4, {V}, 3, 3)")
    out = torch.empty((4, 18, V), dtype=dtype, device=U.device)
    check(lib().rmh_pack_links(lattice_arg(L), _dev(aos, "U"), _dev(out, "out"),
                               _dtype_code(out), _stream(U.device)), "rmh_pack_links")
    return out


def unpack_links(L, U_soa: torch.Tensor) -> torch.Tensor:
    V = volume(L)
    out = torch.empty((4, V, 3, 3, 2), dtype=torch.float64, device=U_soa.device)
    check(lib().rmh_unpack_links(lattice_arg(L), _dev(U_soa, "U_soa"), _dev(out, "out"), _stream(U_soa.device)),
          "rmh_unpack_links")
    return torch.view_as_complex(out)


def pack_fields(L, F_aos: torch.Tensor, dtype=torch.float64) -> torch.Tensor:
    """SoA (n, 4, 8, V) from AoS (n, V, 4, 8) float64."""
    n = F_aos.shape[0]
    out = torch.empty((n, 4, 8, volume(L)), dtype=dtype, device=F_aos.device)
    check(lib().rmh_pack_fields(lattice_arg(L), n, _dev(F_aos, "F_aos"), _dev(out, "out"), _dtype_code(out),
                                _stream(F_aos.device)), "rmh_pack_fields")
    return out


def unpack_fields(L, F_soa: torch.Tensor) -> torch.Tensor:
    n = F_soa.shape[0]
    out = torch.empty((n, volume(L), 4, 8), dtype=torch.float64, device=F_soa.device)
    check(lib().rmh_unpack_fields(lattice_arg(L), n, _dev(F_soa, "F_soa"), _dtype_code(F_soa), _dev(out, "out"),
                                  _stream(F_soa.device)), "rmh_unpack_fields")
    return out


def convert_f64_f32(x: torch.Tensor) -> torch.Tensor:
    out = torch.empty(x.shape, dtype=torch.float32, device=x.device)
    check(lib().rmh_convert_f64_f32(_dev(x, "x"), _dev(out, "out"), x.numel(), _stream(x.device)),
          "rmh_convert_f64_f32")
    return out


# ------------------------------------------------------------------------------------------
# operator

def laplacian_apply(L, U: torch.Tensor, x: torch.Tensor, shift: float = 0.0,
                    out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = (Delta + shift) x for x of shape (n, 4, 8, V)."""
    if U.dtype != x.dtype:
        raise TypeError("U and x must share a dtype")
    y = torch.empty_like(x) if out is None else out
    check(lib().rmh_laplacian_apply(lattice_arg(L), _dev(U, "U"), _dtype_code(x), _dev(x, "x"), _dev(y, "y"),
                                    x.shape[0], float(shift), _stream(x.device)), "rmh_laplacian_apply")
    return y


def laplacian_apply_bwd(L, U, x, g, shift: float = 0.0, grad_x: bool = True, grad_omega: bool = True,
                        per_rhs: bool = False):
    """(grad_x = (Delta + shift) g, grad_omega = d<g, Delta x>/d omega) for y = (Delta + shift) x."""
    n = x.shape[0]
    gx = torch.empty_like(g) if grad_x else None
    go = (torch.empty((n if per_rhs else 1, 4, 8, volume(L)), dtype=torch.float64, device=x.device)
          if grad_omega else None)
    check(lib().rmh_laplacian_apply_bwd(lattice_arg(L), _dev(U, "U"), _dtype_code(x), _dev(x, "x"), _dev(g, "g"),
                                        n, float(shift), gx.data_ptr() if gx is not None else None,
                                        go.data_ptr() if go is not None else None, int(per_rhs),
                                        _stream(x.device)), "rmh_laplacian_apply_bwd")
    return gx, go


# ------------------------------------------------------------------------------------------
# Chebyshev

def _cheb(degree, n_windows, edges, kernel):
    e = None if edges is None else np.ascontiguousarray(edges, dtype=np.float64)
    st = L_.RmhCheb(int(degree), int(n_windows), _f64p(e), int(kernel))
    return st, e


def cheb_coefficients(degree: int, n_windows: int, edges=None, kernel: int = 1) -> np.ndarray:
    st, keep = _cheb(degree, n_windows, edges, kernel)
    coef = np.empty((n_windows, degree + 1))
    check(lib().rmh_cheb_coefficients(ctypes.byref(st), _f64p(coef)), "rmh_cheb_coefficients")
    return coef


def power_spectrum(L, U, F, degree: int, n_windows: int, edges=None, kernel: int = 1):
    """(moments (n, degree+1), power (n, n_windows)) as numpy FP64."""
    n = F.shape[0]
    st, keep = _cheb(degree, n_windows, edges, kernel)
    mom = np.empty((n, degree + 1))
    pw = np.empty((n, n_windows))
    code = _dtype_code(F)
    ws = _workspace(workspace_bytes(L_.OP_POWER_SPECTRUM, L, code, n, n_windows, degree), F.device)
    check(lib().rmh_power_spectrum(lattice_arg(L), _dev(U, "U"), code, _dev(F, "F"), n, ctypes.byref(st),
                                   _f64p(mom), _f64p(pw), ws.data_ptr(), ws.numel(), _stream(F.device)),
          "rmh_power_spectrum")
    return mom, pw


def power_spectrum_noalloc(L, U, F, degree: int, n_windows: int, edges=None, kernel: int = 1):
    """power_spectrum on the library's static device scratch (rmh_power_spectrum_noalloc): no
    workspace tensor, nothing allocated on the device by the call."""
    n = F.shape[0]
    st, keep = _cheb(degree, n_windows, edges, kernel)
    mom = np.empty((n, degree + 1))
    pw = np.empty((n, n_windows))
    check(lib().rmh_power_spectrum_noalloc(lattice_arg(L), _dev(U, "U"), _dtype_code(F), _dev(F, "F"), n,
                                           ctypes.byref(st), _f64p(mom), _f64p(pw), _stream(F.device)),
          "rmh_power_spectrum_noalloc")
    return mom, pw


def power_ratio(degree: int, n_windows: int, trace_moments, power, edges=None, kernel: int = 1) -> np.ndarray:
    st, keep = _cheb(degree, n_windows, edges, kernel)
    tm = np.ascontiguousarray(trace_moments, dtype=np.float64)
    pw = np.ascontiguousarray(power, dtype=np.float64)
    out = np.empty_like(pw)
    check(lib().rmh_power_ratio(ctypes.byref(st), _f64p(tm), _f64p(pw), pw.shape[0], _f64p(out)),
          "rmh_power_ratio")
    return out


def trace_moments_free(L, degree: int) -> np.ndarray:
    out = np.empty(degree + 1)
    check(lib().rmh_trace_moments_free(lattice_arg(L), degree, _f64p(out)), "rmh_trace_moments_free")
    return out


def cheb_filter(L, U, x, degree: int, n_windows: int, edges=None, kernel: int = 1) -> torch.Tensor:
    """y (n_windows, n, 4, 8, V) with y[w] = B_w x."""
    n = x.shape[0]
    st, keep = _cheb(degree, n_windows, edges, kernel)
    code = _dtype_code(x)
    y = torch.empty((n_windows,) + tuple(x.shape), dtype=x.dtype, device=x.device)
    ws = _workspace(workspace_bytes(L_.OP_CHEB_FILTER, L, code, n, n_windows, degree), x.device)
    check(lib().rmh_cheb_filter(lattice_arg(L), _dev(U, "U"), code, _dev(x, "x"), n, ctypes.byref(st),
                                _dev(y, "y"), ws.data_ptr(), ws.numel(), _stream(x.device)), "rmh_cheb_filter")
    return y


def _require_f64(*ts):
    for t in ts:
        if t.dtype != torch.float64:
            raise TypeError("this call takes FP64 links and fields")


def cheb_filter_bwd(L, U, x, gy, degree: int, n_windows: int, edges=None, kernel: int = 1,
                    grad_x: bool = True, grad_omega: bool = True, per_rhs: bool = False):
    """VJP of y_w = B_w x with cotangents gy (n_windows, n, 4, 8, V), all FP64:
    (grad_x = sum_w B_w gy_w, grad_omega = d sum_w <gy_w, y_w> / d omega), None where not requested."""
    n = x.shape[0]
    V = volume(L)
    _require_f64(U, x, gy)
    if tuple(gy.shape) != (n_windows,) + tuple(x.shape):
        raise ValueError(f"gy must have shape {(n_windows,) + tuple(x.shape)}")
    st, keep = _cheb(degree, n_windows, edges, kernel)
    gx = torch.empty_like(x) if grad_x else None
    go = torch.empty((n if per_rhs else 1, 4, 8, V), dtype=torch.float64, device=x.device) if grad_omega else None
    ws = _workspace(workspace_bytes(L_.OP_CHEB_FILTER_BWD, L, RMH_F64, n, n_windows, degree), x.device)
    check(lib().rmh_cheb_filter_bwd(lattice_arg(L), _dev(U, "U"), _dev(x, "x"), _dev(gy, "gy"), n, ctypes.byref(st),
                                    gx.data_ptr() if gx is not None else None,
                                    go.data_ptr() if go is not None else None, int(per_rhs), ws.data_ptr(),
                                    ws.numel(), _stream(x.device)), "rmh_cheb_filter_bwd")
    return gx, go


def power_spectrum_bwd(L, U, F, gamma, degree: int, n_windows: int, edges=None, kernel: int = 1,
                       grad_F: bool = True, grad_omega: bool = True, per_rhs: bool = False):
    """VJP of power[n, w] = <F_n, B_w F_n> with host cotangent gamma (n, n_windows), all FP64:
    (grad_F = 2 sum_w gamma_w B_w F, grad_omega = d sum gamma * power / d omega)."""
    n = F.shape[0]
    V = volume(L)
    _require_f64(U, F)
    st, keep = _cheb(degree, n_windows, edges, kernel)
    gam = np.ascontiguousarray(np.asarray(gamma, np.float64).reshape(n, n_windows))
    gF = torch.empty_like(F) if grad_F else None
    go = torch.empty((n if per_rhs else 1, 4, 8, V), dtype=torch.float64, device=F.device) if grad_omega else None
    ws = _workspace(workspace_bytes(L_.OP_POWER_SPECTRUM_BWD, L, RMH_F64, n, n_windows, degree), F.device)
    check(lib().rmh_power_spectrum_bwd(lattice_arg(L), _dev(U, "U"), _dev(F, "F"), n, ctypes.byref(st), _f64p(gam),
                                       gF.data_ptr() if gF is not None else None,
                                       go.data_ptr() if go is not None else None, int(per_rhs), ws.data_ptr(),
                                       ws.numel(), _stream(F.device)), "rmh_power_spectrum_bwd")
    return gF, go


def heatbath_momenta(L, U, xi, kappa: float, rat: Rational, solver: Solver = Solver()):
    """dict(P, stats): P = R(Delta)^{-1} xi; kappa > 0: as (1 - kappa + kappa Delta) R(Delta) xi for a pole set
    with R^2 ~ (1 - kappa + kappa Delta)^{-1}; kappa = 0: exactly, through the partial fractions of 1/R."""
    _require_f64(U, xi)
    n = xi.shape[0]
    P = torch.empty_like(xi)
    stats = L_.RmhStats()
    ws = _workspace(workspace_bytes(L_.OP_HEATBATH, L, RMH_F64, n, len(rat.r), solver.basis, solver.mode),
                    xi.device)
    rs, ss = rat.c_struct(), solver.c_struct()
    check(lib().rmh_heatbath_momenta(lattice_arg(L), _dev(U, "U"), _dev(xi, "xi"), n, float(kappa),
                                     ctypes.byref(rs), ctypes.byref(ss), P.data_ptr(), ctypes.byref(stats),
                                     ws.data_ptr(), ws.numel(), _stream(xi.device)), "rmh_heatbath_momenta")
    return {"P": P, "stats": stats.as_dict()}


def wilson_gauge_force(L, U, beta: float, want_action: bool = True):
    """(F_G (4, 8, V) FP64 on the device, S_W or None) for FP64 SoA links U."""
    _require_f64(U)
    F = torch.empty((4, 8, volume(L)), dtype=torch.float64, device=U.device)
    S = np.zeros(1)
    ws = _workspace(workspace_bytes(L_.OP_GAUGE_FORCE, L, RMH_F64, 1), U.device)
    check(lib().rmh_wilson_gauge_force(lattice_arg(L), _dev(U, "U"), float(beta), F.data_ptr(),
                                       _f64p(S) if want_action else None, ws.data_ptr(), ws.numel(),
                                       _stream(U.device)), "rmh_wilson_gauge_force")
    return F, (float(S[0]) if want_action else None)


# ------------------------------------------------------------------------------------------
# rational mass term

def rational_from_quadratics(a0, a1, b0, b1):
    a0, a1, b0, b1 = (np.ascontiguousarray(v, dtype=np.float64) for v in (a0, a1, b0, b1))
    n = len(a0)
    r = np.empty(2 * n)
    s = np.empty(2 * n)
    check(lib().rmh_rational_from_quadratics(n, _f64p(a0), _f64p(a1), _f64p(b0), _f64p(b1), _f64p(r), _f64p(s)),
          "rmh_rational_from_quadratics")
    return r, s


def rational_kappa(kappa: float, n: int) -> Rational:
    c = ctypes.c_double()
    r = np.empty(n)
    s = np.empty(n)
    check(lib().rmh_rational_kappa(float(kappa), int(n), ctypes.byref(c), _f64p(r), _f64p(s)), "rmh_rational_kappa")
    return Rational(c.value, r, s)


def rational_apply(L, U, x, rat: Rational, solver: Solver = Solver(), want_poles: bool = False,
                   want_K: bool = True):
    """dict(y, x_poles, K, stats): y = R(Delta) x with every shift at true residual <= tol."""
    n = x.shape[0]
    np_ = len(rat.r)
    y = torch.empty_like(x)
    xp = torch.empty((n, np_) + tuple(x.shape[1:]), dtype=torch.float64, device=x.device) if want_poles else None
    K = np.empty(n) if want_K else None
    stats = L_.RmhStats()
    ws = _workspace(workspace_bytes(L_.OP_RATIONAL_APPLY, L, RMH_F64, n, np_, solver.basis, solver.mode), x.device)
    rs, ss = rat.c_struct(), solver.c_struct()
    check(lib().rmh_rational_apply(lattice_arg(L), _dev(U, "U"), _dev(x, "x"), n, ctypes.byref(rs),
                                   ctypes.byref(ss), _dev(y, "y"), xp.data_ptr() if xp is not None else None,
                                   _f64p(K), ctypes.byref(stats), ws.data_ptr(), ws.numel(), _stream(x.device)),
          "rmh_rational_apply")
    return {"y": y, "x_poles": xp, "K": K, "stats": stats.as_dict()}


def rational_apply_bwd(L, U, x, g, rat: Rational, solver: Solver = Solver(), grad_x: bool = True,
                       per_rhs: bool = False):
    """(grad_x = R(Delta) g, grad_omega = d<g, R(Delta[U]) x>/d omega, stats)."""
    n = x.shape[0]
    np_ = len(rat.r)
    gx = torch.empty_like(g) if grad_x else None
    go = torch.empty((n if per_rhs else 1, 4, 8, volume(L)), dtype=torch.float64, device=x.device)
    stats = L_.RmhStats()
    ws = _workspace(workspace_bytes(L_.OP_RATIONAL_APPLY_BWD, L, RMH_F64, n, np_, solver.basis, solver.mode), x.device)
    rs, ss = rat.c_struct(), solver.c_struct()
    check(lib().rmh_rational_apply_bwd(lattice_arg(L), _dev(U, "U"), _dev(x, "x"), _dev(g, "g"), n,
                                       ctypes.byref(rs), ctypes.byref(ss),
                                       gx.data_ptr() if gx is not None else None, _dev(go, "grad_omega"),
                                       int(per_rhs), ctypes.byref(stats), ws.data_ptr(), ws.numel(),
                                       _stream(x.device)), "rmh_rational_apply_bwd")
    return gx, go, stats.as_dict()


def kinetic_force(L, U, P, rat: Rational, solver: Solver = Solver(), per_rhs: bool = False,
                  want_Y: bool = False, ws: Optional[torch.Tensor] = None):
    """dict(Y, K, dK, stats): K = 1/2 <Y, Y>, Y = R(Delta) P, dK = dK/d omega."""
    n = P.shape[0]
    np_ = len(rat.r)
    Y = torch.empty_like(P) if want_Y else None
    K = np.empty(n)
    dK = torch.empty((n if per_rhs else 1, 4, 8, volume(L)), dtype=torch.float64, device=P.device)
    stats = L_.RmhStats()
    need = workspace_bytes(L_.OP_KINETIC_FORCE, L, RMH_F64, n, np_, solver.basis, solver.mode)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, P.device)
    rs, ss = rat.c_struct(), solver.c_struct()
    check(lib().rmh_kinetic_force(lattice_arg(L), _dev(U, "U"), _dev(P, "P"), n, ctypes.byref(rs),
                                  ctypes.byref(ss), Y.data_ptr() if Y is not None else None, _f64p(K),
                                  _dev(dK, "dK"), int(per_rhs), ctypes.byref(stats), ws.data_ptr(), ws.numel(),
                                  _stream(P.device)), "rmh_kinetic_force")
    return {"Y": Y, "K": K, "dK": dK, "stats": stats.as_dict()}


def leapfrog_step(L, U, P, rat: Rational, eps: float, beta: float, solver: Solver = Solver(),
                  fp_tol: float = 1e-12, fp_maxiter: int = 50, ws: Optional[torch.Tensor] = None):
    """(U', P', stats): one implicit leapfrog step of size eps for H = 1/2 <R(Delta) P, R(Delta) P> + S_W(U)
    (rmh_leapfrog_step).  U: SoA FP64 links (4, 18, V); P: FP64 momentum field (4, 8, V) or (1, 4, 8, V)."""
    _require_f64(U, P)
    U1 = torch.empty_like(U)
    P1 = torch.empty_like(P)
    np_ = len(rat.r)
    need = workspace_bytes(L_.OP_LEAPFROG, L, RMH_F64, 1, np_, solver.basis, solver.mode)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, P.device)
    lf = L_.RmhLeapfrog(float(eps), float(beta), float(fp_tol), int(fp_maxiter))
    stats = L_.RmhLeapfrogStats()
    rs, ss = rat.c_struct(), solver.c_struct()
    check(lib().rmh_leapfrog_step(lattice_arg(L), _dev(U, "U"), _dev(P, "P"), ctypes.byref(rs), ctypes.byref(ss),
                                  ctypes.byref(lf), _dev(U1, "U1"), _dev(P1, "P1"), ctypes.byref(stats),
                                  ws.data_ptr(), ws.numel(), _stream(P.device)), "rmh_leapfrog_step")
    return U1, P1, stats.as_dict()


# ------------------------------------------------------------------------------------------
# link displacements

def link_exp(L, U, omega: torch.Tensor) -> torch.Tensor:
    """exp(i omega.T) U per link (rmh_link_exp): U SoA FP64 (4, 18, V), omega FP64 (4, 8, V)."""
    _require_f64(U, omega)
    out = torch.empty_like(U)
    check(lib().rmh_link_exp(lattice_arg(L), _dev(U, "U"), _dev(omega, "omega"), _dev(out, "U1"),
                             _stream(U.device)), "rmh_link_exp")
    return out


def link_exp_vjp(L, omega: torch.Tensor, g: torch.Tensor) -> torch.Tensor:
    """J(omega)^T g per link (rmh_link_exp_vjp): the derivative with respect to omega of a function
    of exp(i omega.T) U from its left-multiplication derivative g at the displaced links."""
    _require_f64(omega, g)
    out = torch.empty_like(g)
    check(lib().rmh_link_exp_vjp(lattice_arg(L), _dev(omega, "omega"), _dev(g, "g"), _dev(out, "out"),
                                 _stream(g.device)), "rmh_link_exp_vjp")
    return out


# ------------------------------------------------------------------------------------------
# stencil tuning

PURPOSES = {"any": -1, "apply": 0, "cg": 1, "cg64": 2, "moments": 3, "filter": 4, "cheb_bwd": 5, "heatbath": 6}


def _purpose(purpose) -> int:
    return PURPOSES[purpose] if isinstance(purpose, str) else int(purpose)


def tune_set(L, dtype, n_rhs: int, form: int, block: int = 256, xcd_remap: int = 1, nv: int = 4,
             order: int = 0, walk: int = 0, ns: int = 1, purpose="any", tile2: int = 1) -> None:
    """Store a stencil launch configuration for (L, dtype, n_rhs, purpose) (rmh_tune_set)."""
    code = RMH_F64 if dtype == torch.float64 else RMH_F32
    cfg = L_.RmhHopConfig(int(form), int(block), int(xcd_remap), int(nv), int(order), int(walk), int(ns),
                          int(tile2))
    check(lib().rmh_tune_set(lattice_arg(L), code, int(n_rhs), _purpose(purpose), ctypes.byref(cfg)),
          "rmh_tune_set")


def tune_clear() -> None:
    check(lib().rmh_tune_clear(), "rmh_tune_clear")


def tune_save(path: str) -> int:
    """Write the stored configurations to a JSON file (stamped with the device architecture and HIP
    runtime version); returns the entry count."""
    n = ctypes.c_int32(0)
    check(lib().rmh_tune_save(os.fsencode(path), ctypes.byref(n)), "rmh_tune_save")
    return n.value


def tune_load(path: str) -> int:
    """Store the configurations of a file written by tune_save if it was written for this device
    architecture and HIP runtime; returns the count stored (0 for another device or runtime)."""
    n = ctypes.c_int32(0)
    check(lib().rmh_tune_load(os.fsencode(path), ctypes.byref(n)), "rmh_tune_load")
    return n.value


def autotune_laplacian(L, U, x, reps: int = 5, purpose="any"):
    """((form, block, xcd_remap, nv, order, walk, ns, tile2), ms) of the fastest configuration for x's batch
    and the purpose, now stored; ms is the mean time of one timing unit."""
    y = torch.empty_like(x)
    best = L_.RmhHopConfig()
    ms = ctypes.c_double()
    ws = _workspace(workspace_bytes(L_.OP_AUTOTUNE, L, _dtype_code(x), x.shape[0]), x.device)
    check(lib().rmh_autotune_laplacian(lattice_arg(L), _dev(U, "U"), _dtype_code(x), _dev(x, "x"), _dev(y, "y"),
                                       x.shape[0], _purpose(purpose), int(reps), ctypes.byref(best),
                                       ctypes.byref(ms), _dev(ws, "ws"), ws.numel(), _stream(x.device)),
          "rmh_autotune_laplacian")
    return best.as_tuple(), ms.value


# ------------------------------------------------------------------------------------------
# kernel timing

PROF_CLASSES = {"stencil": 0, "cg_residual": 1, "cg_shifts": 2, "force": 3, "cheb_fold": 4}


def profile_enable(on: bool = True) -> None:
    check(lib().rmh_profile_enable(int(bool(on))), "rmh_profile_enable")


def profile_read(cls: str) -> dict:
    """{launches, ms, bytes, items, avg_ms, gbs} accumulated for one kernel class since the last reset."""
    n = L_.c_i64()
    ms = ctypes.c_double()
    by = ctypes.c_double()
    it = ctypes.c_double()
    check(lib().rmh_profile_read(PROF_CLASSES[cls], ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                 ctypes.byref(it)), "rmh_profile_read")
    avg = ms.value / n.value if n.value else 0.0
    gbs = by.value / (ms.value * 1e-3) / 1e9 if ms.value > 0 else 0.0
    return {"launches": n.value, "ms": ms.value, "bytes": by.value, "items": it.value, "avg_ms": avg, "gbs": gbs}
