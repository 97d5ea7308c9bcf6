"""Python binding of librift_ile.so (ctypes; torch for device memory and streams).

Argument marshalling only: every step of the likelihood runs in the HIP
library.  There is no fallback -- if the library or a GPU is missing, calls
raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librift_ile.so")

RIFT_FP64 = 0
RIFT_MIXED = 1
RIFT_FP32 = 2
PRECISIONS = {"fp64": RIFT_FP64, "mixed": RIFT_MIXED, "fp32": RIFT_FP32}

# coordinates of theta rows 3 and 6 in the gradient entry points (the
# gradient is taken in the same coordinates)
RIFT_COORD_COS_INCL = 1
RIFT_COORD_LN_DIST = 2
COORDS = {
    "physical": 0,                                        # incl, dist
    "paper": RIFT_COORD_LN_DIST,                          # incl, ln dist
    "sampler": RIFT_COORD_COS_INCL | RIFT_COORD_LN_DIST,  # cos incl, ln dist
}


def coord_names(coords: int):
    return ("ra", "dec", "psi", "cos_incl" if coords & RIFT_COORD_COS_INCL else "incl", "phiref", "tref",
            "ln_dist" if coords & RIFT_COORD_LN_DIST else "dist")


def _coords(c) -> int:
    return COORDS[c] if isinstance(c, str) else int(c)

EXPORTS = (
    "rift_ile_lnL",
    "rift_ile_lnZ",
    "rift_ile_grad",
    "rift_ile_plan_create",
    "rift_ile_plan_lnZ",
    "rift_ile_plan_grad",
    "rift_ile_plan_tune",
    "rift_ile_plan_get_config",
    "rift_ile_plan_set_config",
    "rift_ile_plan_refined",
    "rift_ile_plan_profile",
    "rift_ile_plan_profile_read",
    "rift_ile_plan_destroy",
    "rift_ile_strerror",
    "rift_ile_version",
    "rift_ile_wide_lnL",
    "rift_ile_wide_lnZ",
    "rift_ile_lnZ_noalloc",
    "rift_ile_leapfrog_drift",
    "rift_ile_plan_lnZ_dmarg",
    "rift_ile_gauss_hermite",
    "rift_ile_pregrid",
    "rift_ile_plan_lnZ_tmarg",
    "rift_ile_plan_lnZ_pmarg",
    "rift_ile_plan_hmc",
    "rift_ile_plan_lnZ_tband",
    "rift_ile_plan_lnZ_erai",
    "rift_ile_moments",
    "rift_ile_plan_grad_dmarg",
    "rift_ile_plan_hmc_dmarg",
    "rift_ile_plan_nuts_dmarg",
    "rift_ile_plan_rwm",
    "rift_ile_mixture_is",
    "rift_ile_plan_hmc_tempered",
    "rift_ile_smc_reweight",
    "rift_ile_smc_resample",
    "rift_ile_plan_nuts",
)

RESPONSES = {"rotation": 1, "arms": 2, "rotation_delay": 3}


class CPoint(ctypes.Structure):
    _fields_ = [
        ("n_det", ctypes.c_int32),
        ("n_modes", ctypes.c_int32),
        ("n_t", ctypes.c_int32),
        ("lm", ctypes.c_void_p),
        ("t0", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("Q", ctypes.c_void_p),
        ("U", ctypes.c_void_p),
        ("V", ctypes.c_void_p),
        ("det_tensor", ctypes.c_void_p),
        ("det_pos", ctypes.c_void_p),
        ("gmst_rad", ctypes.c_double),
        ("d_ref", ctypes.c_double),
    ]


class CPointWide(ctypes.Structure):
    _fields_ = [
        ("n_det", ctypes.c_int32),
        ("n_modes", ctypes.c_int32),
        ("n_t", ctypes.c_int32),
        ("lm", ctypes.c_void_p),
        ("t0", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("response", ctypes.c_int32),
        ("n_terms", ctypes.c_int32),
        ("Q", ctypes.c_void_p),
        ("U", ctypes.c_void_p),
        ("V", ctypes.c_void_p),
        ("det_tensor", ctypes.c_void_p),
        ("det_pos", ctypes.c_void_p),
        ("det_arms", ctypes.c_void_p),
        ("gmst_rad", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("d_ref", ctypes.c_double),
    ]


class CDistPrior(ctypes.Structure):
    _fields_ = [("d_min", ctypes.c_double), ("d_max", ctypes.c_double), ("n_nodes", ctypes.c_int32)]


class CTimeRule(ctypes.Structure):
    _fields_ = [("t_start", ctypes.c_double), ("h", ctypes.c_double), ("n_t", ctypes.c_int32)]


class CPsiRule(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("n_points", ctypes.c_int32)]


PSI_METHODS = {"trapezoid": 0, "laplace": 1, "cells": 2}


class CBandRule(ctypes.Structure):
    _fields_ = [("t_start", ctypes.c_double), ("h", ctypes.c_double), ("n_t", ctypes.c_int32),
                ("n_fine", ctypes.c_int32)]


class CAngleRule(ctypes.Structure):
    _fields_ = [("n_phi", ctypes.c_int32), ("n_psi", ctypes.c_int32)]


class CHmcPrior(ctypes.Structure):
    _fields_ = [("t_min", ctypes.c_double), ("t_max", ctypes.c_double), ("d_min", ctypes.c_double),
                ("d_max", ctypes.c_double)]


class CMixture(ctypes.Structure):
    _fields_ = [("n_comp", ctypes.c_int32), ("alpha", ctypes.c_double), ("scale", ctypes.c_double),
                ("a", ctypes.c_void_p), ("mean", ctypes.c_void_p), ("cov", ctypes.c_void_p),
                ("rows", ctypes.c_int32)]


class CConfig(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("tile_blocks", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("sort", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load librift_ile.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2609_37393_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    P = ctypes.POINTER(CPoint)
    ci = ctypes.c_int
    lib.rift_ile_lnL.argtypes = [P, i64, vp, vp, vp, ci, vp]
    lib.rift_ile_lnZ.argtypes = [P, i32, vp, vp, vp, vp, vp, vp, ci, vp]
    lib.rift_ile_grad.argtypes = [P, i64, vp, ci, vp, vp, ci, vp]
    lib.rift_ile_plan_create.argtypes = [P, i32, vp, ci, vp, ctypes.POINTER(vp)]
    lib.rift_ile_plan_lnZ.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.rift_ile_plan_grad.argtypes = [vp, i32, i64, vp, ci, vp, vp, vp]
    lib.rift_ile_plan_tune.argtypes = [vp, vp, vp, vp]
    lib.rift_ile_plan_get_config.argtypes = [vp, ctypes.POINTER(CConfig)]
    lib.rift_ile_plan_set_config.argtypes = [vp, ctypes.POINTER(CConfig)]
    lib.rift_ile_plan_refined.argtypes = [vp, ctypes.POINTER(i64)]
    lib.rift_ile_plan_profile.argtypes = [vp, ctypes.c_int]
    lib.rift_ile_plan_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    lib.rift_ile_plan_destroy.argtypes = [vp]
    PW = ctypes.POINTER(CPointWide)
    lib.rift_ile_wide_lnL.argtypes = [PW, i64, vp, vp, vp]
    lib.rift_ile_wide_lnZ.argtypes = [PW, i64, vp, vp, vp, vp, vp, vp]
    lib.rift_ile_lnZ_noalloc.argtypes = [P, i32, vp, vp, vp, vp, vp, vp, ci, vp]
    lib.rift_ile_leapfrog_drift.argtypes = [i64, vp, vp, vp, vp]
    lib.rift_ile_plan_lnZ_dmarg.argtypes = [vp, vp, vp, ctypes.POINTER(CDistPrior), vp, vp, vp, vp]
    lib.rift_ile_gauss_hermite.argtypes = [ctypes.c_int, vp, vp]
    lib.rift_ile_pregrid.argtypes = [vp, i64, i32, i32, vp, vp]
    lib.rift_ile_plan_lnZ_tmarg.argtypes = [vp, vp, vp, ctypes.POINTER(CTimeRule), vp, vp, vp, vp]
    lib.rift_ile_plan_lnZ_pmarg.argtypes = [vp, vp, vp, ctypes.POINTER(CPsiRule), vp, vp, vp, vp]
    lib.rift_ile_plan_lnZ_erai.argtypes = [vp, vp, vp, ctypes.POINTER(CAngleRule), vp, vp, vp, vp]
    lib.rift_ile_plan_lnZ_tband.argtypes = [vp, vp, vp, ctypes.POINTER(CBandRule), vp, vp, vp, vp]
    lib.rift_ile_plan_hmc.argtypes = [vp, i32, i64, vp, vp, vp, vp, ctypes.c_double, i32,
                                      ctypes.POINTER(CHmcPrior), vp, vp, vp]
    lib.rift_ile_plan_hmc_tempered.argtypes = [vp, i32, i64, vp, vp, vp, vp, ctypes.c_double, i32,
                                               ctypes.POINTER(CHmcPrior), ctypes.c_double, vp, vp, vp]
    lib.rift_ile_plan_nuts.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, ctypes.c_double, i32,
                                       ctypes.POINTER(CHmcPrior), ctypes.c_double, vp, vp, vp]
    lib.rift_ile_smc_reweight.argtypes = [i64, vp, vp, ctypes.c_double, ctypes.c_double, vp, vp]
    lib.rift_ile_smc_resample.argtypes = [i64, vp, ctypes.c_double, vp, vp, vp, vp]
    lib.rift_ile_moments.argtypes = [i64, vp, vp, vp, vp, vp]
    lib.rift_ile_plan_grad_dmarg.argtypes = [vp, i32, i64, vp, ctypes.POINTER(CDistPrior), vp, vp, vp]
    lib.rift_ile_plan_hmc_dmarg.argtypes = [vp, i32, i64, vp, vp, vp, vp, ctypes.c_double, i32,
                                            ctypes.POINTER(CHmcPrior), ctypes.POINTER(CDistPrior), ctypes.c_double,
                                            vp, vp, vp]
    lib.rift_ile_plan_nuts_dmarg.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, ctypes.c_double, i32,
                                             ctypes.POINTER(CHmcPrior), ctypes.POINTER(CDistPrior), ctypes.c_double,
                                             vp, vp, vp]
    lib.rift_ile_plan_rwm.argtypes = [vp, i32, i64, vp, vp, vp, vp, ctypes.c_double, ctypes.POINTER(CHmcPrior),
                                      ctypes.c_double, vp, vp, vp, vp]
    lib.rift_ile_mixture_is.argtypes = [i64, ctypes.POINTER(CMixture), ctypes.POINTER(CHmcPrior), vp, vp, vp, vp,
                                        vp, vp, vp, vp]
    lib.rift_ile_strerror.argtypes = [ctypes.c_int]
    lib.rift_ile_strerror.restype = ctypes.c_char_p
    lib.rift_ile_version.restype = ctypes.c_int
    for name in EXPORTS:
        getattr(lib, name)
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc < 0:
        msg = load().rift_ile_strerror(rc).decode()
        raise RuntimeError(f"{what} failed: {msg} ({rc})")
    return rc


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_f64(a, device) -> torch.Tensor:
    t = torch.as_tensor(a)
    if t.is_complex():
        t = torch.view_as_real(t.to(torch.complex128).contiguous())
    return t.to(device=device, dtype=torch.float64).contiguous()


@dataclass
class DevicePoint:
    """One intrinsic point with its arrays resident on the GPU (Q, U, V) and the
    small metadata on the host."""
    lm: np.ndarray
    t0: float
    dt: float
    Q: torch.Tensor       # [K, M, n_t, 2] float64 (complex interleaved)
    U: torch.Tensor       # [K, M, M, 2]
    V: torch.Tensor
    det_tensor: np.ndarray
    det_pos: np.ndarray
    gmst: float
    d_ref: float

    @classmethod
    def from_dict(cls, pt, device="cuda"):
        return cls(
            lm=np.ascontiguousarray(pt["lm"], dtype=np.int32),
            t0=float(pt["t0"]),
            dt=float(pt["dt"]),
            Q=_dev_f64(pt["Q"], device),
            U=_dev_f64(pt["U"], device),
            V=_dev_f64(pt["V"], device),
            det_tensor=np.ascontiguousarray(pt["det_tensor"], dtype=np.float64),
            det_pos=np.ascontiguousarray(pt["det_pos"], dtype=np.float64),
            gmst=float(pt["gmst"]),
            d_ref=float(pt["d_ref"]),
        )

    @property
    def device(self):
        return self.Q.device

    def cstruct(self) -> CPoint:
        K, M, n_t = self.Q.shape[:3]
        return CPoint(K, M, n_t, self.lm.ctypes.data, self.t0, self.dt, self.Q.data_ptr(),
                      self.U.data_ptr(), self.V.data_ptr(), self.det_tensor.ctypes.data,
                      self.det_pos.ctypes.data, self.gmst, self.d_ref)


@dataclass
class DeviceWidePoint:
    """A composite-index point (generalised response) with Q, U, V on the GPU."""
    lm: np.ndarray
    t0: float
    dt: float
    response: str
    Q: torch.Tensor       # [K, n_terms, M, n_t, 2] float64
    U: torch.Tensor       # [K, n_terms M, n_terms M, 2]
    V: torch.Tensor
    det_tensor: np.ndarray
    det_pos: np.ndarray
    det_arms: np.ndarray
    gmst: float
    omega: float
    d_ref: float

    @classmethod
    def from_dict(cls, pt, device="cuda"):
        return cls(
            lm=np.ascontiguousarray(pt["lm"], dtype=np.int32), t0=float(pt["t0"]), dt=float(pt["dt"]),
            response=pt["response"], Q=_dev_f64(pt["Q"], device), U=_dev_f64(pt["U"], device),
            V=_dev_f64(pt["V"], device),
            det_tensor=np.ascontiguousarray(pt["det_tensor"], dtype=np.float64),
            det_pos=np.ascontiguousarray(pt["det_pos"], dtype=np.float64),
            det_arms=np.ascontiguousarray(pt["det_arms"], dtype=np.float64),
            gmst=float(pt["gmst"]), omega=float(pt.get("omega", 0.0)), d_ref=float(pt["d_ref"]))

    @property
    def device(self):
        return self.Q.device

    def cstruct(self) -> CPointWide:
        K, n_a, M, n_t = self.Q.shape[:4]
        return CPointWide(K, M, n_t, self.lm.ctypes.data, self.t0, self.dt, RESPONSES[self.response], n_a,
                          self.Q.data_ptr(), self.U.data_ptr(), self.V.data_ptr(), self.det_tensor.ctypes.data,
                          self.det_pos.ctypes.data, self.det_arms.ctypes.data, self.gmst, self.omega, self.d_ref)


def _as_wide(pt, device) -> DeviceWidePoint:
    return pt if isinstance(pt, DeviceWidePoint) else DeviceWidePoint.from_dict(pt, device)


def wide_lnL(point, theta, device="cuda") -> torch.Tensor:
    """lnL [n] of the composite-index likelihood (Eq. (slowrot:lnL:Decomposed))."""
    lib = load()
    p = _as_wide(point, device)
    th = _theta(theta, p.device)
    n = th.shape[1]
    out = torch.empty(n, dtype=torch.float64, device=p.device)
    cp = p.cstruct()
    _check(lib.rift_ile_wide_lnL(ctypes.byref(cp), n, th.data_ptr(), out.data_ptr(), _stream(p.device)),
           "rift_ile_wide_lnL")
    return out


def wide_lnZ(point, theta, lnw=None, want_lnL=False, device="cuda"):
    """(ln Z, n_eff[, lnL]) of the composite-index likelihood over the samples."""
    lib = load()
    p = _as_wide(point, device)
    th = _theta(theta, p.device)
    n = th.shape[1]
    w = None if lnw is None else torch.as_tensor(lnw).to(device=p.device, dtype=torch.float64).contiguous()
    z = torch.empty(1, dtype=torch.float64, device=p.device)
    ne = torch.empty(1, dtype=torch.float64, device=p.device)
    ll = torch.empty(n, dtype=torch.float64, device=p.device) if want_lnL else None
    cp = p.cstruct()
    _check(lib.rift_ile_wide_lnZ(ctypes.byref(cp), n, th.data_ptr(), None if w is None else w.data_ptr(),
                                 z.data_ptr(), ne.data_ptr(), None if ll is None else ll.data_ptr(),
                                 _stream(p.device)), "rift_ile_wide_lnZ")
    return (z, ne, ll) if want_lnL else (z, ne)


def lnL_dmarg(point, theta, d_min, d_max, n_nodes=20, device="cuda") -> torch.Tensor:
    """ln L_d [n]: the likelihood marginalised over distance per sample
    (rift_ile_plan_lnZ_dmarg through a one-point plan)."""
    th = _theta(theta, device)
    n = th.shape[1]
    plan = Plan([point], [n], device=device)
    try:
        out = torch.empty(n, dtype=torch.float64, device=device)
        plan.lnZ_dmarg(th, d_min, d_max, n_nodes, lnL_out=out)
        torch.cuda.synchronize(device)
    finally:
        plan.close()
    return out


def smc_reweight(lnL, lnW, beta, target, out=None):
    """One SMC ladder update in place on lnW (rift_ile_smc_reweight); returns
    out = [beta', dlnZ] (a device tensor)."""
    lib = load()
    o = out if out is not None else torch.empty(2, dtype=torch.float64, device=lnW.device)
    _check(lib.rift_ile_smc_reweight(lnW.numel(), lnL.data_ptr(), lnW.data_ptr(), float(beta), float(target),
                                     o.data_ptr(), _stream(lnW.device)), "rift_ile_smc_reweight")
    return o


def smc_resample(lnW, u, theta_in=None, theta_out=None, ancestors=None):
    """Systematic resampling (rift_ile_smc_resample): theta_out[:, i] =
    theta_in[:, a_i] and/or the ancestors a_i (int64)."""
    lib = load()
    n = lnW.numel()
    _check(lib.rift_ile_smc_resample(n, lnW.data_ptr(), float(u),
                                     None if theta_in is None else theta_in.data_ptr(),
                                     None if theta_out is None else theta_out.data_ptr(),
                                     None if ancestors is None else ancestors.data_ptr(), _stream(lnW.device)),
           "rift_ile_smc_resample")
    return ancestors


def moments(c, lnw=None):
    """Weighted mean [7] and covariance [7, 7] of a cloud c [7, n] on the
    device (rift_ile_moments); lnw [n] log weights or None (equal)."""
    lib = load()
    dev = c.device
    mean = torch.empty(7, dtype=torch.float64, device=dev)
    cov = torch.empty((7, 7), dtype=torch.float64, device=dev)
    n = c.shape[1]
    _check(lib.rift_ile_moments(n, c.data_ptr() if n else None, None if lnw is None else lnw.data_ptr(),
                                mean.data_ptr(), cov.data_ptr(), _stream(dev)), "rift_ile_moments")
    return mean, cov


def mixture_is(alpha, a, mean, cov, scale, box, z, v, u, theta=None, lnw=None, comp=None, status=None, rows=0x7F):
    """Draws from the defensive mixture alpha p + (1 - alpha) sum_m a_m
    N(mean[m], scale cov[m]) and their log weights ln p - ln q
    (rift_ile_mixture_is).  a: host sequence; mean [n_comp, 7], cov
    [n_comp, 7, 7], z, v [7, n], u [n]: device tensors; box = (t_min, t_max,
    d_min, d_max); rows: bit mask of the rows the components sample (the
    weights then cover those rows alone).  Returns (theta [7, n], lnw [n],
    comp [n] int32, status [1] int32)."""
    lib = load()
    dev = u.device
    n = u.numel()
    a_h = np.ascontiguousarray(np.asarray(a, np.float64))
    nc = a_h.size
    theta = theta if theta is not None else torch.empty((7, n), dtype=torch.float64, device=dev)
    lnw = lnw if lnw is not None else torch.empty(n, dtype=torch.float64, device=dev)
    comp = comp if comp is not None else torch.empty(n, dtype=torch.int32, device=dev)
    status = status if status is not None else torch.empty(1, dtype=torch.int32, device=dev)
    mix = CMixture(nc, float(alpha), float(scale), a_h.ctypes.data if nc else None,
                   mean.data_ptr() if nc else None, cov.data_ptr() if nc else None, int(rows))
    pr = CHmcPrior(*[float(x) for x in box])
    ptr = (lambda t: t.data_ptr() if n else None)
    _check(lib.rift_ile_mixture_is(n, ctypes.byref(mix), ctypes.byref(pr), ptr(z), ptr(v), ptr(u), ptr(theta),
                                   ptr(lnw), ptr(comp), status.data_ptr(), _stream(dev)), "rift_ile_mixture_is")
    return theta, lnw, comp, status


def pregrid(q, r: int, out=None, device="cuda") -> torch.Tensor:
    """Fourier refinement by r of complex series q [..., n] (rift_ile_pregrid):
    [..., (n - 1) r + 1] complex128 on the device."""
    lib = load()
    qt = torch.as_tensor(q).to(device=device, dtype=torch.complex128).contiguous()
    n = qt.shape[-1]
    S = int(np.prod(qt.shape[:-1])) if qt.dim() > 1 else 1
    nf = (n - 1) * int(r) + 1
    o = out if out is not None else torch.empty(qt.shape[:-1] + (nf,), dtype=torch.complex128, device=device)
    _check(lib.rift_ile_pregrid(qt.data_ptr(), S, n, int(r), o.data_ptr(), _stream(torch.device(device))),
           "rift_ile_pregrid")
    return o


def gauss_hermite(n: int):
    """The library's n-point rule of the weight exp(-x^2/2) (nodes, weights)."""
    x = np.zeros(n)
    w = np.zeros(n)
    _check(load().rift_ile_gauss_hermite(int(n), x.ctypes.data, w.ctypes.data), "rift_ile_gauss_hermite")
    return x, w


def leapfrog_drift(theta: torch.Tensor, p: torch.Tensor, step):
    """theta += step * p in place (rows as in the sampler's coordinates), with
    cos incl reflected into [-1, 1] and its momentum flipped (rift_ile_leapfrog_drift)."""
    lib = load()
    st = np.ascontiguousarray(step, dtype=np.float64)
    if st.shape != (7,) or theta.shape != p.shape or theta.shape[0] != 7:
        raise ValueError("theta, p: [7, n]; step: [7]")
    _check(lib.rift_ile_leapfrog_drift(theta.shape[1], theta.data_ptr(), p.data_ptr(), st.ctypes.data,
                                       _stream(theta.device)), "rift_ile_leapfrog_drift")


def _as_point(pt, device) -> DevicePoint:
    return pt if isinstance(pt, DevicePoint) else DevicePoint.from_dict(pt, device)


def _theta(theta, device) -> torch.Tensor:
    th = torch.as_tensor(theta)
    if th.ndim != 2 or th.shape[0] != 7:
        raise ValueError("theta must be [7, n]: ra, dec, psi, incl, phiref, tref, dist")
    return th.to(device=device, dtype=torch.float64).contiguous()


def lnL(point, theta, precision: str = "fp64", device="cuda", with_bound=False):
    """lnL [n] of the samples theta [7, n] (Eq. (def:lnL:Decomposed)); with
    `with_bound`, also every value's a-priori bound on |lnL - lnL_FP64| [n]."""
    lib = load()
    p = _as_point(point, device)
    th = _theta(theta, p.device)
    n = th.shape[1]
    out = torch.empty(n, dtype=torch.float64, device=p.device)
    bnd = torch.empty(n, dtype=torch.float64, device=p.device) if with_bound else None
    cp = p.cstruct()
    _check(lib.rift_ile_lnL(ctypes.byref(cp), n, th.data_ptr(), out.data_ptr(),
                            None if bnd is None else bnd.data_ptr(), PRECISIONS[precision],
                            _stream(p.device)), "rift_ile_lnL")
    return (out, bnd) if with_bound else out


def grad(point, theta, coords="sampler", device="cuda"):
    """(lnL [n], gradient [7, n]) with theta rows 3 and 6 in the coordinates
    `coords` ("physical": incl, dist; "paper": incl, ln dist; "sampler":
    cos incl, ln dist; or the RIFT_COORD_* bits) and the gradient taken in
    them."""
    lib = load()
    p = _as_point(point, device)
    th = _theta(theta, p.device)
    n = th.shape[1]
    out = torch.empty(n, dtype=torch.float64, device=p.device)
    g = torch.empty((7, n), dtype=torch.float64, device=p.device)
    cp = p.cstruct()
    _check(lib.rift_ile_grad(ctypes.byref(cp), n, th.data_ptr(), _coords(coords), out.data_ptr(), g.data_ptr(),
                             RIFT_FP64, _stream(p.device)), "rift_ile_grad")
    return out, g


def lnZ(points, theta, n_per_point=None, lnw=None, precision: str = "fp64", want_lnL=False,
        device="cuda"):
    """ln Z and n_eff per point (Eqs. (lnL:MonteCarlo), (neff)); one persistent launch.

    points: list of points; theta [7, N] with the samples of point p in the
    n_per_point[p] consecutive columns after those of the previous points.
    Returns (lnZ [P], neff [P]) or (lnZ, neff, lnL [N]).
    """
    lib = load()
    if not isinstance(points, (list, tuple)):
        points = [points]
    pts = [_as_point(p, device) for p in points]
    dev = pts[0].device
    th = _theta(theta, dev)
    N = th.shape[1]
    counts = np.asarray([N] if n_per_point is None else n_per_point, dtype=np.int64)
    if counts.sum() != N or counts.size != len(pts):
        raise ValueError("n_per_point must sum to theta.shape[1], one count per point")
    cps = (CPoint * len(pts))(*[p.cstruct() for p in pts])
    w = None if lnw is None else torch.as_tensor(lnw).to(device=dev, dtype=torch.float64).contiguous()
    z = torch.empty(len(pts), dtype=torch.float64, device=dev)
    ne = torch.empty(len(pts), dtype=torch.float64, device=dev)
    ll = torch.empty(N, dtype=torch.float64, device=dev) if want_lnL else None
    _check(lib.rift_ile_lnZ(cps, len(pts), counts.ctypes.data, th.data_ptr(),
                            None if w is None else w.data_ptr(), z.data_ptr(), ne.data_ptr(),
                            None if ll is None else ll.data_ptr(), PRECISIONS[precision],
                            _stream(dev)), "rift_ile_lnZ")
    return (z, ne, ll) if want_lnL else (z, ne)


class Plan:
    """Prepared points for repeated (graph-capturable) evaluation."""

    def __init__(self, points, n_per_point, precision: str = "fp64", device="cuda"):
        self.lib = load()
        if not isinstance(points, (list, tuple)):
            points = [points]
        self.points = [_as_point(p, device) for p in points]
        self.device = self.points[0].device
        self.counts = np.asarray(n_per_point, dtype=np.int64)
        self.N = int(self.counts.sum())
        self.precision = precision
        cps = (CPoint * len(self.points))(*[p.cstruct() for p in self.points])
        h = ctypes.c_void_p()
        _check(self.lib.rift_ile_plan_create(cps, len(self.points), self.counts.ctypes.data,
                                             PRECISIONS[precision], _stream(self.device), ctypes.byref(h)),
               "rift_ile_plan_create")
        self.handle = h

    def lnZ(self, theta, lnw=None, lnZ_out=None, neff_out=None, lnL_out=None, err_out=None, bnd_out=None):
        th = theta if (isinstance(theta, torch.Tensor) and theta.is_contiguous() and theta.dtype == torch.float64) \
            else _theta(theta, self.device)
        P = len(self.points)
        z = lnZ_out if lnZ_out is not None else torch.empty(P, dtype=torch.float64, device=self.device)
        ne = neff_out if neff_out is not None else torch.empty(P, dtype=torch.float64, device=self.device)
        _check(self.lib.rift_ile_plan_lnZ(self.handle, th.data_ptr(), None if lnw is None else lnw.data_ptr(),
                                          z.data_ptr(), ne.data_ptr(),
                                          None if lnL_out is None else lnL_out.data_ptr(),
                                          None if bnd_out is None else bnd_out.data_ptr(),
                                          None if err_out is None else err_out.data_ptr(),
                                          _stream(self.device)), "rift_ile_plan_lnZ")
        return z, ne

    def lnZ_dmarg(self, theta, d_min, d_max, n_nodes=20, lnw=None, lnZ_out=None, neff_out=None, lnL_out=None):
        """(ln Z_d, n_eff) per point of the likelihood marginalised over
        distance (prior p(D) ~ D^2 on [d_min, d_max], n_nodes-point adaptive
        Gauss-Hermite rule; rift_ile_plan_lnZ_dmarg); lnL_out receives ln L_d
        per sample.  The distance row of theta is not read."""
        th = theta if (isinstance(theta, torch.Tensor) and theta.is_contiguous() and theta.dtype == torch.float64) \
            else _theta(theta, self.device)
        P = len(self.points)
        z = lnZ_out if lnZ_out is not None else torch.empty(P, dtype=torch.float64, device=self.device)
        ne = neff_out if neff_out is not None else torch.empty(P, dtype=torch.float64, device=self.device)
        pr = CDistPrior(float(d_min), float(d_max), int(n_nodes))
        _check(self.lib.rift_ile_plan_lnZ_dmarg(self.handle, th.data_ptr(), None if lnw is None else lnw.data_ptr(),
                                                ctypes.byref(pr), z.data_ptr(), ne.data_ptr(),
                                                None if lnL_out is None else lnL_out.data_ptr(),
                                                _stream(self.device)), "rift_ile_plan_lnZ_dmarg")
        return z, ne

    def lnZ_tmarg(self, theta, t_start, h, n_t, lnw=None, lnZ_out=None, neff_out=None, lnL_out=None):
        """(ln Z_t, n_eff) per point of the likelihood marginalised over
        geocentric time by the fixed-spacing Simpson rule on n_t times
        t_start + k h (rift_ile_plan_lnZ_tmarg); lnL_out receives ln L_t per
        sample.  The t_ref row of theta is not read."""
        th = theta if (isinstance(theta, torch.Tensor) and theta.is_contiguous() and theta.dtype == torch.float64) \
            else _theta(theta, self.device)
        P = len(self.points)
        z = lnZ_out if lnZ_out is not None else torch.empty(P, dtype=torch.float64, device=self.device)
        ne = neff_out if neff_out is not None else torch.empty(P, dtype=torch.float64, device=self.device)
        rule = CTimeRule(float(t_start), float(h), int(n_t))
        _check(self.lib.rift_ile_plan_lnZ_tmarg(self.handle, th.data_ptr(), None if lnw is None else lnw.data_ptr(),
                                                ctypes.byref(rule), z.data_ptr(), ne.data_ptr(),
                                                None if lnL_out is None else lnL_out.data_ptr(),
                                                _stream(self.device)), "rift_ile_plan_lnZ_tmarg")
        return z, ne

    def lnZ_tband(self, theta, t_start, h, n_t, n_fine, lnw=None, lnZ_out=None, neff_out=None, lnL_out=None):
        """(ln Z_t, n_eff) per point of the likelihood marginalised over
        geocentric time by the band-limited full-window rule
        (rift_ile_plan_lnZ_tband): n_t nodes t_start + j h, n_fine fine
        intervals per node interval; lnL_out receives ln L_t per sample.  The
        t_ref row of theta is not read."""
        th = theta if (isinstance(theta, torch.Tensor) and theta.is_contiguous() and theta.dtype == torch.float64) \
            else _theta(theta, self.device)
        P = len(self.points)
        z = lnZ_out if lnZ_out is not None else torch.empty(P, dtype=torch.float64, device=self.device)
        ne = neff_out if neff_out is not None else torch.empty(P, dtype=torch.float64, device=self.device)
        rule = CBandRule(float(t_start), float(h), int(n_t), int(n_fine))
        _check(self.lib.rift_ile_plan_lnZ_tband(self.handle, th.data_ptr(), None if lnw is None else lnw.data_ptr(),
                                                ctypes.byref(rule), z.data_ptr(), ne.data_ptr(),
                                                None if lnL_out is None else lnL_out.data_ptr(),
                                                _stream(self.device)), "rift_ile_plan_lnZ_tband")
        return z, ne

    def lnZ_erai(self, theta, n_phi, n_psi, lnw=None, lnZ_out=None, neff_out=None, lnL_out=None):
        """(ln Z, n_eff) per point of the likelihood marginalised over phiref
        and psi by exact reconstruction (rift_ile_plan_lnZ_erai) on an
        n_phi x n_psi grid; lnL_out receives the per-sample marginal."""
        th = theta if (isinstance(theta, torch.Tensor) and theta.is_contiguous() and theta.dtype == torch.float64) \
            else _theta(theta, self.device)
        P = len(self.points)
        z = lnZ_out if lnZ_out is not None else torch.empty(P, dtype=torch.float64, device=self.device)
        ne = neff_out if neff_out is not None else torch.empty(P, dtype=torch.float64, device=self.device)
        rule = CAngleRule(int(n_phi), int(n_psi))
        _check(self.lib.rift_ile_plan_lnZ_erai(self.handle, th.data_ptr(), None if lnw is None else lnw.data_ptr(),
                                               ctypes.byref(rule), z.data_ptr(), ne.data_ptr(),
                                               None if lnL_out is None else lnL_out.data_ptr(),
                                               _stream(self.device)), "rift_ile_plan_lnZ_erai")
        return z, ne

    def lnZ_pmarg(self, theta, method="trapezoid", n_points=64, lnw=None, lnZ_out=None, neff_out=None,
                  lnL_out=None):
        """(ln Z_psi, n_eff) per point of the likelihood marginalised over
        polarisation (rift_ile_plan_lnZ_pmarg): method "trapezoid" (n_points on
        the circle) or "laplace"; lnL_out receives ln L_psi per sample."""
        th = theta if (isinstance(theta, torch.Tensor) and theta.is_contiguous() and theta.dtype == torch.float64) \
            else _theta(theta, self.device)
        P = len(self.points)
        z = lnZ_out if lnZ_out is not None else torch.empty(P, dtype=torch.float64, device=self.device)
        ne = neff_out if neff_out is not None else torch.empty(P, dtype=torch.float64, device=self.device)
        rule = CPsiRule(PSI_METHODS[method], int(n_points))
        _check(self.lib.rift_ile_plan_lnZ_pmarg(self.handle, th.data_ptr(), None if lnw is None else lnw.data_ptr(),
                                                ctypes.byref(rule), z.data_ptr(), ne.data_ptr(),
                                                None if lnL_out is None else lnL_out.data_ptr(),
                                                _stream(self.device)), "rift_ile_plan_lnZ_pmarg")
        return z, ne

    def hmc(self, point, theta, z, u, sigma, eps, n_leapfrog, box, lnL_out=None, accepted_out=None, beta=None,
            dmarg=None):
        """One Metropolis-adjusted HMC transition of every chain in place
        (rift_ile_plan_hmc, or rift_ile_plan_hmc_tempered on L^beta p when
        beta is given): theta [7, n] in the sampler coordinates, z [7, n]
        standard normals, u [n] uniforms, sigma [7], box = (t_min, t_max,
        d_min, d_max).  With dmarg = (d_min, d_max, n_nodes), the target is
        the likelihood marginalised over distance (rift_ile_plan_hmc_dmarg).
        Returns (lnL [n], accepted [n] int32)."""
        n = theta.shape[1]
        l = lnL_out if lnL_out is not None else torch.empty(n, dtype=torch.float64, device=self.device)
        acc = accepted_out if accepted_out is not None else torch.empty(n, dtype=torch.int32, device=self.device)
        sg = np.ascontiguousarray(sigma, dtype=np.float64)
        pr = CHmcPrior(*[float(b) for b in box])
        if dmarg is not None:
            dp = CDistPrior(float(dmarg[0]), float(dmarg[1]), int(dmarg[2]))
            _check(self.lib.rift_ile_plan_hmc_dmarg(self.handle, int(point), n, theta.data_ptr(), z.data_ptr(),
                                                    u.data_ptr(), sg.ctypes.data, float(eps), int(n_leapfrog),
                                                    ctypes.byref(pr), ctypes.byref(dp),
                                                    1.0 if beta is None else float(beta), l.data_ptr(),
                                                    acc.data_ptr(), _stream(self.device)), "rift_ile_plan_hmc_dmarg")
        elif beta is None:
            _check(self.lib.rift_ile_plan_hmc(self.handle, int(point), n, theta.data_ptr(), z.data_ptr(),
                                              u.data_ptr(), sg.ctypes.data, float(eps), int(n_leapfrog),
                                              ctypes.byref(pr), l.data_ptr(), acc.data_ptr(), _stream(self.device)),
                   "rift_ile_plan_hmc")
        else:
            _check(self.lib.rift_ile_plan_hmc_tempered(self.handle, int(point), n, theta.data_ptr(), z.data_ptr(),
                                                       u.data_ptr(), sg.ctypes.data, float(eps), int(n_leapfrog),
                                                       ctypes.byref(pr), float(beta), l.data_ptr(), acc.data_ptr(),
                                                       _stream(self.device)), "rift_ile_plan_hmc_tempered")
        return l, acc

    def nuts(self, point, theta, z, dirs, merges, leaves, sigma, eps, max_depth, box, beta=1.0, lnL_out=None,
             info_out=None, dmarg=None):
        """One No-U-Turn transition of every chain in place
        (rift_ile_plan_nuts): theta [7, n] sampler coordinates, z [7, n]
        normals, dirs and merges [max_depth, n] and leaves
        [2^max_depth - 1, n] uniforms.  Returns (lnL [n], info [3, n] int32:
        doublings, leapfrog steps, divergent)."""
        n = theta.shape[1]
        l = lnL_out if lnL_out is not None else torch.empty(n, dtype=torch.float64, device=self.device)
        inf = info_out if info_out is not None else torch.empty((3, n), dtype=torch.int32, device=self.device)
        sg = np.ascontiguousarray(sigma, dtype=np.float64)
        pr = CHmcPrior(*[float(b) for b in box])
        if dmarg is not None:
            dp = CDistPrior(float(dmarg[0]), float(dmarg[1]), int(dmarg[2]))
            _check(self.lib.rift_ile_plan_nuts_dmarg(self.handle, int(point), n, theta.data_ptr(), z.data_ptr(),
                                                     dirs.data_ptr(), merges.data_ptr(), leaves.data_ptr(),
                                                     sg.ctypes.data, float(eps), int(max_depth), ctypes.byref(pr),
                                                     ctypes.byref(dp), float(beta), l.data_ptr(), inf.data_ptr(),
                                                     _stream(self.device)), "rift_ile_plan_nuts_dmarg")
            return l, inf
        _check(self.lib.rift_ile_plan_nuts(self.handle, int(point), n, theta.data_ptr(), z.data_ptr(), dirs.data_ptr(),
                                           merges.data_ptr(), leaves.data_ptr(), sg.ctypes.data, float(eps),
                                           int(max_depth), ctypes.byref(pr), float(beta), l.data_ptr(),
                                           inf.data_ptr(), _stream(self.device)), "rift_ile_plan_nuts")
        return l, inf

    def rwm(self, point, theta, z, u, cov, scale, box, lnL, beta=1.0, accepted_out=None, status_out=None):
        """One random-walk Metropolis move per chain with proposal covariance
        scale cov (rift_ile_plan_rwm); theta [7, n] in the sampler
        coordinates and lnL [n] (lnL at the states) are updated in place.
        Returns (accepted int32 [n], status int32 [1])."""
        n = theta.shape[1]
        acc = accepted_out if accepted_out is not None else torch.empty(n, dtype=torch.int32, device=self.device)
        st = status_out if status_out is not None else torch.empty(1, dtype=torch.int32, device=self.device)
        pr = CHmcPrior(*[float(x) for x in box])
        ptr = (lambda t: t.data_ptr() if n else None)
        _check(self.lib.rift_ile_plan_rwm(self.handle, int(point), n, ptr(theta), ptr(z), ptr(u), cov.data_ptr(),
                                          float(scale), ctypes.byref(pr), float(beta), ptr(lnL), ptr(acc),
                                          st.data_ptr(), _stream(self.device)), "rift_ile_plan_rwm")
        return acc, st

    def grad_dmarg(self, point, theta, d_min, d_max, n_nodes=20, lnLd_out=None, grad_out=None):
        """(ln L_d [n], d ln L_d / d(ra, dec, psi, cos incl, phiref, tref, -)
        [7, n]) of the likelihood marginalised over distance
        (rift_ile_plan_grad_dmarg); theta in the samplers' coordinates, row 6
        not read."""
        th = theta if (isinstance(theta, torch.Tensor) and theta.is_contiguous() and theta.dtype == torch.float64) \
            else _theta(theta, self.device)
        n = th.shape[1]
        ld = lnLd_out if lnLd_out is not None else torch.empty(n, dtype=torch.float64, device=self.device)
        g = grad_out if grad_out is not None else torch.empty((7, n), dtype=torch.float64, device=self.device)
        pr = CDistPrior(float(d_min), float(d_max), int(n_nodes))
        _check(self.lib.rift_ile_plan_grad_dmarg(self.handle, int(point), n, th.data_ptr(), ctypes.byref(pr),
                                                 ld.data_ptr(), g.data_ptr(), _stream(self.device)),
               "rift_ile_plan_grad_dmarg")
        return ld, g

    def grad(self, point, theta, lnL_out=None, grad_out=None, coords="sampler"):
        """Gradient of lnL with theta rows 3 and 6 in the coordinates `coords`
        (as in `grad`), taken in those coordinates."""
        th = theta if (isinstance(theta, torch.Tensor) and theta.is_contiguous() and theta.dtype == torch.float64) \
            else _theta(theta, self.device)
        n = th.shape[1]
        g = grad_out if grad_out is not None else torch.empty((7, n), dtype=torch.float64, device=self.device)
        _check(self.lib.rift_ile_plan_grad(self.handle, int(point), n, th.data_ptr(), _coords(coords),
                                           None if lnL_out is None else lnL_out.data_ptr(), g.data_ptr(),
                                           _stream(self.device)), "rift_ile_plan_grad")
        return g

    def tune(self, theta, lnw=None) -> int:
        return _check(self.lib.rift_ile_plan_tune(self.handle, theta.data_ptr(),
                                                  None if lnw is None else lnw.data_ptr(),
                                                  _stream(self.device)), "rift_ile_plan_tune")

    @property
    def config(self):
        c = CConfig()
        _check(self.lib.rift_ile_plan_get_config(self.handle, ctypes.byref(c)), "get_config")
        return {"block": c.block, "tile_blocks": c.tile_blocks, "blocks_per_cu": c.blocks_per_cu,
                "sort": c.sort}

    @config.setter
    def config(self, cfg):
        cur = self.config
        cur.update(cfg)
        c = CConfig(int(cur["block"]), int(cur["tile_blocks"]), int(cur["blocks_per_cu"]), int(cur["sort"]))
        _check(self.lib.rift_ile_plan_set_config(self.handle, ctypes.byref(c)), "set_config")

    def refined(self) -> int:
        v = ctypes.c_int64()
        _check(self.lib.rift_ile_plan_refined(self.handle, ctypes.byref(v)), "refined")
        return int(v.value)

    def profile(self, enable: bool):
        _check(self.lib.rift_ile_plan_profile(self.handle, 1 if enable else 0), "profile")

    def profile_read(self):
        """(summed kernel ms, launches) of the main evaluation kernel."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(self.lib.rift_ile_plan_profile_read(self.handle, ctypes.byref(ms), ctypes.byref(n)),
               "profile_read")
        return ms.value, int(n.value)

    def close(self):
        if getattr(self, "handle", None):
            self.lib.rift_ile_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LnL(torch.autograd.Function):
    """lnL(theta) with the hand-written adjoint kernel's gradient.

    theta [7, n] holds (ra, dec, psi, incl, phiref, tref, ln dist) by default
    (coords="paper"), or the rows 3 and 6 named by `coords` ("physical":
    incl, dist; "sampler": cos incl, ln dist).  The kernel returns the gradient
    in those same coordinates, and backward only scales it by grad_out."""

    @staticmethod
    def forward(ctx, theta, point, coords="paper"):
        l, g = grad(point, theta.detach(), coords=coords, device=theta.device)
        ctx.save_for_backward(g)
        return l

    @staticmethod
    def backward(ctx, grad_out):
        (g,) = ctx.saved_tensors
        return grad_out[None, :] * g, None, None
