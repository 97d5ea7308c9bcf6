"""FP64 CPU oracle for the factored extrinsic likelihood (test infrastructure).

TEST INFRASTRUCTURE ONLY: only the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this module.  The product path
(the HIP library and its Python binding) never imports, loads or calls it, and
the two share no code.

The arithmetic lives in ``oracle.cpp`` (plain loops, IEEE double, OpenMP over
samples); this module only marshals numpy arrays into it.  ``pregrid`` (the
Fourier refinement of Eq. (q-time-pregrid)), ``lnL_dmarg`` (the adaptive
Gauss-Hermite marginal over distance, Eq. (ap:dgh)), ``lnL_tmarg`` (the
fixed-spacing rule over time, Eq. (ap:tfixed)), ``lnL_tband`` (the
band-limited full-window rule over time, Eq. (ap:tband)), ``lnL_erai`` (the
joint marginal over phiref and psi by exact reconstruction, Eqs.
(ap:angleharm), (ap:nyquist)) and ``lnL_pmarg`` (the
polarisation marginal, Eqs. (ap:psiexp), (ap:psilaplace)), ``hmc_step``
(a Metropolis-adjusted Hamiltonian transition on the gradient, optionally
on the tempered target) and the SMC ladder's ``smc_cess``, ``smc_next_beta``,
``smc_update`` and ``systematic_resample`` (Eq. (sampler-menu:smc-update)),
the cloud's random-walk Metropolis move (``rwm_step``), and the
importance-sampling normalisation with a defensive Gaussian-mixture
proposal (``cloud_moments``, ``mixture_is``, Eq. (sampler-menu:is)) are
written here in numpy on top of the C likelihood.

Every function states the passage of the paper it follows.  Parity status of
each function (what pins it) is listed in the tests' docstrings.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

THETA_NAMES = ("ra", "dec", "psi", "incl", "phiref", "tref", "dist")
GRAD_NAMES = ("ra", "dec", "psi", "cos_incl", "phiref", "tref", "ln_dist")


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (-O2 -fopenmp)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["g++", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c++17", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        d = ctypes.c_double
        p = ctypes.c_void_p
        lib.oracle_ylm.argtypes = [ctypes.c_int, ctypes.c_int, d, d, p]
        lib.oracle_antenna.argtypes = [p, d, d, d, d, p, p]
        lib.oracle_arrival_time.argtypes = [p, d, d, d, d]
        lib.oracle_arrival_time.restype = d
        lib.oracle_interp.argtypes = [p, ctypes.c_int, d, d, ctypes.c_int64, p, p]
        lib.oracle_lnL_factored.argtypes = [ctypes.c_int, ctypes.c_int, p, p, d, p, p, p]
        lib.oracle_lnL_factored.restype = d
        lib.oracle_lnL.argtypes = [p, ctypes.c_int64, p, p, ctypes.c_int]
        lib.oracle_grad.argtypes = [p, ctypes.c_int64, p, p, p, ctypes.c_int]
        lib.oracle_lnZ.argtypes = [ctypes.c_int64, p, p, p, p]
        lib.oracle_rotation_harmonics.argtypes = [p, d, d, p]
        lib.oracle_wide_coef.argtypes = [p, p, p, p]
        lib.oracle_lnL_wide.argtypes = [p, ctypes.c_int64, p, p, ctypes.c_int]
        lib.oracle_lnL_terms.argtypes = [p, ctypes.c_int64, p, p, p, ctypes.c_int]
        _lib = lib
    return _lib


class _CPoint(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32),
        ("M", ctypes.c_int32),
        ("n_t", ctypes.c_int32),
        ("lm", ctypes.c_void_p),
        ("t0", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("Q", ctypes.c_void_p),
        ("U", ctypes.c_void_p),
        ("V", ctypes.c_void_p),
        ("det_tensor", ctypes.c_void_p),
        ("det_pos", ctypes.c_void_p),
        ("gmst", ctypes.c_double),
        ("d_ref", ctypes.c_double),
    ]


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class _Packed:
    cp: _CPoint
    keep: tuple


def _pack(pt) -> _Packed:
    """pt: mapping with lm [M,2], t0, dt, Q [K,M,n_t] complex, U/V [K,M,M] complex,
    det_tensor [K,3,3], det_pos [K,3] (light-seconds), gmst, d_ref."""
    lm = _c(pt["lm"], np.int32)
    Q = _c(pt["Q"], np.complex128)
    U = _c(pt["U"], np.complex128)
    V = _c(pt["V"], np.complex128)
    D = _c(pt["det_tensor"], np.float64)
    R = _c(pt["det_pos"], np.float64)
    K, M, n_t = Q.shape
    assert U.shape == (K, M, M) and V.shape == (K, M, M) and lm.shape == (M, 2)
    assert D.shape == (K, 3, 3) and R.shape == (K, 3)
    cp = _CPoint(K, M, n_t, _ptr(lm).value, float(pt["t0"]), float(pt["dt"]), _ptr(Q).value,
                 _ptr(U).value, _ptr(V).value, _ptr(D).value, _ptr(R).value,
                 float(pt["gmst"]), float(pt["d_ref"]))
    return _Packed(cp, (lm, Q, U, V, D, R))


class _CPointWide(ctypes.Structure):
    _fields_ = [
        ("K", ctypes.c_int32),
        ("M", ctypes.c_int32),
        ("n_t", ctypes.c_int32),
        ("lm", ctypes.c_void_p),
        ("t0", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("response", ctypes.c_int32),
        ("n_a", ctypes.c_int32),
        ("Q", ctypes.c_void_p),
        ("U", ctypes.c_void_p),
        ("V", ctypes.c_void_p),
        ("det_tensor", ctypes.c_void_p),
        ("det_pos", ctypes.c_void_p),
        ("det_arms", ctypes.c_void_p),
        ("gmst", ctypes.c_double),
        ("omega", ctypes.c_double),
        ("d_ref", ctypes.c_double),
    ]


RESPONSES = {"rotation": 1, "arms": 2, "rotation_delay": 3}


def _pack_wide(pt) -> _Packed:
    """pt: mapping as for `_pack` plus response ("rotation" | "arms"), Q [K, n_a, M, n_t],
    U, V [K, n_a M, n_a M] (composite index a M + i), det_arms [K, 2, 3], omega."""
    lm = _c(pt["lm"], np.int32)
    Q = _c(pt["Q"], np.complex128)
    U = _c(pt["U"], np.complex128)
    V = _c(pt["V"], np.complex128)
    D = _c(pt["det_tensor"], np.float64)
    R = _c(pt["det_pos"], np.float64)
    AR = _c(pt["det_arms"], np.float64)
    K, n_a, M, n_t = Q.shape
    A = n_a * M
    assert U.shape == (K, A, A) and V.shape == (K, A, A) and lm.shape == (M, 2) and AR.shape == (K, 2, 3)
    cp = _CPointWide(K, M, n_t, _ptr(lm).value, float(pt["t0"]), float(pt["dt"]), RESPONSES[pt["response"]],
                     n_a, _ptr(Q).value, _ptr(U).value, _ptr(V).value, _ptr(D).value, _ptr(R).value,
                     _ptr(AR).value, float(pt["gmst"]), float(pt.get("omega", 0.0)), float(pt["d_ref"]))
    return _Packed(cp, (lm, Q, U, V, D, R, AR))


# ---------------------------------------------------------------------------
# Building blocks
# ---------------------------------------------------------------------------
def ylm(l: int, m: int, iota: float, phi: float) -> complex:
    """-2Y_lm(iota, phi), Eq. (strain_mode) harmonics (Wigner-d sum)."""
    out = np.zeros(2)
    _load().oracle_ylm(int(l), int(m), float(iota), float(phi), _ptr(out))
    return complex(out[0], out[1])


def antenna(det_tensor, ra, dec, psi, gmst):
    """Static complex antenna factor F = F+ + i Fx of one detector
    (Sec. "Review of the RIFT likelihood", static response).  Returns (F, N)."""
    D = _c(det_tensor, np.float64)
    out = np.zeros(2)
    N = np.zeros(3)
    _load().oracle_antenna(_ptr(D), float(ra), float(dec), float(psi), float(gmst), _ptr(out), _ptr(N))
    return complex(out[0], out[1]), N


def arrival_time(det_pos, ra, dec, gmst, tref):
    """t_k = t_ref - r_k . N (same section; r_k in light-seconds)."""
    r = _c(det_pos, np.float64)
    return _load().oracle_arrival_time(_ptr(r), float(ra), float(dec), float(gmst), float(tref))


def interp(q, t0, dt, t):
    """Four-point cubic read C_3 of a uniformly sampled complex series
    (Eq. (q-time-pregrid)); 4-point Lagrange on nodes j-1..j+2, zero outside."""
    q = _c(q, np.complex128)
    t = _c(np.atleast_1d(t), np.float64)
    out = np.zeros(t.shape[0], np.complex128)
    _load().oracle_interp(_ptr(q), q.shape[0], float(t0), float(dt), t.shape[0], _ptr(t), _ptr(out))
    return out


def lnL_factored(F, Y, x, Qhat, U, V) -> float:
    """Eq. (def:lnL:Decomposed) from F[K], Y[M], x = D_ref/D and Q already read at t_k."""
    F = _c(F, np.complex128)
    Y = _c(Y, np.complex128)
    Qhat = _c(Qhat, np.complex128)
    U = _c(U, np.complex128)
    V = _c(V, np.complex128)
    K, M = Qhat.shape
    return _load().oracle_lnL_factored(K, M, _ptr(F), _ptr(Y), float(x), _ptr(Qhat), _ptr(U), _ptr(V))


# ---------------------------------------------------------------------------
# The path
# ---------------------------------------------------------------------------
def lnL(pt, theta, nthreads: int = 0) -> np.ndarray:
    """lnL for every sample; theta is [7, n] (ra, dec, psi, incl, phiref, tref, dist)."""
    th = _c(theta, np.float64)
    assert th.ndim == 2 and th.shape[0] == 7
    n = th.shape[1]
    out = np.empty(n)
    pk = _pack(pt)
    _load().oracle_lnL(ctypes.byref(pk.cp), n, _ptr(th), _ptr(out), int(nthreads))
    return out


def grad(pt, theta, nthreads: int = 0):
    """(lnL [n], d lnL/d(ra, dec, psi, cos incl, phiref, tref, ln dist) [7, n])."""
    th = _c(theta, np.float64)
    n = th.shape[1]
    out = np.empty(n)
    g = np.empty((7, n))
    pk = _pack(pt)
    _load().oracle_grad(ctypes.byref(pk.cp), n, _ptr(th), _ptr(out), _ptr(g), int(nthreads))
    return out, g


def lnZ(lnL_values, lnw=None):
    """Eq. (lnL:MonteCarlo) in log form with 1/N, and Eq. (neff). Returns (lnZ, neff)."""
    l = _c(lnL_values, np.float64)
    w = None if lnw is None else _c(lnw, np.float64)
    z = np.zeros(1)
    ne = np.zeros(1)
    _load().oracle_lnZ(l.shape[0], _ptr(l), None if w is None else _ptr(w), _ptr(z), _ptr(ne))
    return float(z[0]), float(ne[0])


def lnL_terms(pt, theta, nthreads: int = 0):
    """(K [n], R [n]) with lnL_i(x) = K_i x - R_i x^2 / 2 exactly, x = D_ref / D
    (Eq. (ap:dexp)): K is the data term and R the model norm at the reference
    distance.  The distance row of theta is not read."""
    th = _c(theta, np.float64)
    n = th.shape[1]
    Kv = np.empty(n)
    Rv = np.empty(n)
    pk = _pack(pt)
    _load().oracle_lnL_terms(ctypes.byref(pk.cp), n, _ptr(th), _ptr(Kv), _ptr(Rv), int(nthreads))
    return Kv, Rv


def dist_prior_x(x, d_ref, d_min, d_max, power=2.0):
    """Density in x = d_ref / D of the prior p(D) proportional to D^power on
    [d_min, d_max] (power 2: uniform in Euclidean volume, p_x proportional to
    x^-4), normalised to one, zero outside."""
    x = np.asarray(x, np.float64)
    # int_{d_min}^{d_max} D^power dD
    if power == -1.0:
        norm = np.log(d_max / d_min)
    else:
        norm = (d_max ** (power + 1) - d_min ** (power + 1)) / (power + 1)
    D = d_ref / np.where(x > 0, x, 1.0)
    inside = (x >= d_ref / d_max) & (x <= d_ref / d_min)
    # p_x(x) = p(D(x)) |dD/dx| = p(D) d_ref / x^2
    return np.where(inside, D ** power / norm * d_ref / np.where(x > 0, x, 1.0) ** 2, 0.0)


def lnL_dmarg(pt, theta, d_min, d_max, n_nodes, power=2.0, nthreads: int = 0):
    """ln of the likelihood marginalised over distance, per sample, by the
    adaptive Gauss-Hermite rule of Eq. (ap:dgh): with lnL(x) = K x - R x^2 / 2,
    the peak x* = K / R and width sigma_x = R^-1/2 of Eq. (ap:dpeak) centre and
    scale the n_nodes nodes xi_i (weight exp(-xi^2/2)), and
        int dx p_x(x) e^{lnL(x)} ~ sum_i w~_i p_x(x* + xi_i sigma_x) e^{lnL(x* + xi_i sigma_x)}
    with w~_i = sigma_x W_i e^{xi_i^2 / 2} (the Gaussian factor of the rule
    divided out, since e^{lnL(x* + xi sigma)} = e^{K^2 / 2R} e^{-xi^2 / 2}).
    The prior is p(D) proportional to D^power on [d_min, d_max].  R >= 0
    holds exactly (U positive semi-definite, |Y^T V Y| <= Y^H U Y); R <= 0
    arises only from rounding where the model has no power (F_k Y = 0), and
    there K = 0 as well, lnL = 0 at every distance and the marginal is the
    prior's mass: ln L_d = 0.  A non-finite sample gives NaN."""
    Kv, Rv = lnL_terms(pt, theta, nthreads)
    xi, W = np.polynomial.hermite_e.hermegauss(int(n_nodes))
    d_ref = float(pt["d_ref"])
    nopow = np.isfinite(Kv) & np.isfinite(Rv) & (Rv <= 0.0)
    ok = (Rv > 0.0) & np.isfinite(Kv) & np.isfinite(Rv)
    Ki = np.where(ok, Kv, 0.0)[:, None]
    Ri = np.where(ok, Rv, 1.0)[:, None]
    xs = Ki / Ri
    sig = 1.0 / np.sqrt(Ri)
    x = xs + xi[None, :] * sig                      # [n, nodes]
    lnl = Ki * x - 0.5 * Ri * x * x
    wt = sig * W[None, :] * np.exp(xi * xi / 2.0)[None, :]
    terms = wt * dist_prior_x(x, d_ref, d_min, d_max, power)
    # sum_i terms_i e^{lnl_i}, in log form about the peak value K^2 / 2R
    peak = 0.5 * Ki * Ki / Ri
    s = np.sum(terms * np.exp(lnl - peak), axis=1)
    with np.errstate(divide="ignore"):
        out = peak[:, 0] + np.log(s)
    out[s <= 0] = -np.inf
    out[~ok] = np.nan
    out[nopow] = 0.0
    return out


def grad_dmarg(pt, c, d_min, d_max, n_nodes):
    """(ln L_d [n], d ln L_d / d(ra, dec, psi, cos incl, phiref, tref, -)
    [7, n]) of the likelihood marginalised over distance (Eq. (ap:dgh), prior
    p(D) ~ D^2 on [d_min, d_max]) in the samplers' coordinates c, whose
    distance row is not read (its derivative is 0).  lnL(x) = K x - R x^2 / 2
    exactly (Eq. (ap:dexp)), so the derivative of ln int dx p_x e^{lnL} is
    <x> grad K - <x^2> grad R / 2, the moments taken under the distance
    posterior by the same adaptive rule as lnL_dmarg (node weights
    W_i p_x(x* + xi_i sigma)); grad K and grad R come from the gradient at
    x = 1 and x = 2: g1 = grad K - grad R / 2, g2 = 2 grad K - 2 grad R.
    Where the model has no power (R <= 0) the moments are the prior's
    (numerical quadrature of p_x); with no node inside the prior the value is
    -inf and the derivative 0; a non-finite sample gives NaN."""
    from scipy import integrate as _integrate

    c = np.asarray(c, np.float64)
    d_ref = float(pt["d_ref"])
    th = _to_physical(c)
    t1 = th.copy()
    t1[6] = d_ref
    t2 = th.copy()
    t2[6] = d_ref / 2.0
    _, g1 = grad(pt, t1)
    _, g2 = grad(pt, t2)
    dK = 2.0 * g1 - 0.5 * g2
    dR = 2.0 * g1 - g2
    ld = lnL_dmarg(pt, t1, d_min, d_max, n_nodes)
    Kv, Rv = lnL_terms(pt, t1)
    xi, W = np.polynomial.hermite_e.hermegauss(int(n_nodes))
    n = c.shape[1]
    m1 = np.full(n, np.nan)
    m2 = np.full(n, np.nan)
    ok = np.isfinite(Kv) & np.isfinite(Rv) & (Rv > 0.0)
    xs = np.where(ok, Kv, 0.0) / np.where(ok, Rv, 1.0)
    sig = 1.0 / np.sqrt(np.where(ok, Rv, 1.0))
    x = xs[:, None] + xi[None, :] * sig[:, None]
    om = W[None, :] * dist_prior_x(x, d_ref, d_min, d_max)
    so = om.sum(axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        m1[ok] = (om * x).sum(axis=1)[ok] / so[ok]
        m2[ok] = (om * x * x).sum(axis=1)[ok] / so[ok]
    nopow = np.isfinite(Kv) & np.isfinite(Rv) & (Rv <= 0.0)
    if nopow.any():
        lo, hi = d_ref / d_max, d_ref / d_min
        e1 = _integrate.quad(lambda y: y * dist_prior_x(y, d_ref, d_min, d_max), lo, hi, epsabs=0, epsrel=1e-13)[0]
        e2 = _integrate.quad(lambda y: y * y * dist_prior_x(y, d_ref, d_min, d_max), lo, hi, epsabs=0,
                             epsrel=1e-13)[0]
        m1[nopow], m2[nopow] = e1, e2
    g = m1[None, :] * dK - 0.5 * m2[None, :] * dR
    g[6] = 0.0
    empty = ok & ~(so > 0.0)
    g[:, empty] = 0.0
    bad = ~np.isfinite(Kv) | ~np.isfinite(Rv)
    g[:, bad] = np.nan
    return ld, g


def simpson_weights(n_t: int) -> np.ndarray:
    """Composite Simpson weights on n_t (odd) equally spaced nodes, in units
    of the spacing: (1, 4, 2, 4, ..., 2, 4, 1) / 3."""
    assert n_t >= 3 and n_t % 2 == 1
    w = np.full(n_t, 2.0)
    w[1::2] = 4.0
    w[0] = w[-1] = 1.0
    return w / 3.0


def lnL_tmarg(pt, theta, t_start, h, n_t, nthreads: int = 0):
    """ln of the likelihood marginalised over geocentric time per sample,
    under a prior uniform on [t_start, t_start + (n_t - 1) h], by the
    fixed-spacing rule of Eq. (ap:tfixed) with composite Simpson weights:
        L_t = (1 / T) int dt e^{lnL(t)} ~ (h / T) sum_k w_k e^{lnL(t_start + k h)},
    T = (n_t - 1) h.  Each lnL(t_k) is the oracle's own lnL with t_ref = t_k;
    the time row of theta is not read."""
    th = _c(theta, np.float64)
    n = th.shape[1]
    w = simpson_weights(int(n_t))
    tk = t_start + h * np.arange(n_t)
    big = np.repeat(th, n_t, axis=1)           # sample-major: [7, n * n_t]
    big[5] = np.tile(tk, n)
    l = lnL(pt, big, nthreads).reshape(n, n_t) + np.log(w)[None, :]
    m = np.max(l, axis=1)
    out = np.full(n, np.nan)
    ok = np.isfinite(m)
    out[ok] = m[ok] + np.log(np.sum(np.exp(l[ok] - m[ok, None]), axis=1)) - np.log(n_t - 1.0)
    out[np.isnan(l).any(axis=1)] = np.nan
    return out


def band_values(y, M: int) -> np.ndarray:
    """The band-limited reconstruction of Eq. (ap:tband): from values y [n, ...]
    at the nodes t_j = t_start + j h, the Whittaker-Shannon series
    sum_j y_j sinc((t - t_j) / h) at the fine points t = t_start + (k / M) h,
    k = 0 .. (n - 1) M (M fine intervals in each node interval).  Returns
    [(n - 1) M + 1, ...]."""
    y = np.asarray(y, np.float64)
    n = y.shape[0]
    M = int(M)
    tk = np.arange((n - 1) * M + 1) / M           # fine times in units of h
    S = np.sinc(tk[:, None] - np.arange(n)[None, :])
    return np.tensordot(S, y, axes=(1, 0))


def band_rule(y, base, M: int) -> np.ndarray:
    """ln of the window-averaged exponential of the reconstructed exponent,
    Eq. (ap:tband) under a prior uniform on the node window: with the
    reconstruction v_k = band_values(y, M)_k (the part of the exponent linear
    in the band-limited combination) and the time-independent remainder
    `base`, the trapezoid rule on the fine points,
        ln[(1 / ((n - 1) M)) sum_k w_k e^{v_k + base}],  w = 1, ends 1/2.
    y [n, N], base [N] -> [N]; NaN anywhere in a column gives NaN."""
    v = band_values(y, M) + np.asarray(base, np.float64)[None, :]
    K = v.shape[0]
    lw = np.zeros(K)
    lw[0] = lw[-1] = np.log(0.5)
    l = v + lw[:, None]
    with np.errstate(invalid="ignore"):
        m = np.max(l, axis=0)
    out = np.full(l.shape[1], np.nan)
    ok = np.isfinite(m)
    out[ok] = m[ok] + np.log(np.sum(np.exp(l[:, ok] - m[None, ok]), axis=0)) - np.log(K - 1.0)
    out[np.isnan(l).any(axis=0)] = np.nan
    return out


def lnL_tband(pt, theta, t_start, h, n_t, M, nthreads: int = 0):
    """ln of the likelihood marginalised over geocentric time by the
    band-limited full-window rule, Eq. (ap:tband), per sample: at fixed other
    parameters the data term at the reference distance, kappa(t) = K(t), is
    band limited; it is taken at the n_t nodes t_start + j h (the oracle's own
    K from lnL_terms, Eq. (ap:dexp)), reconstructed at M fine points per node
    interval by the sinc series, and lnL = x kappa - R x^2 / 2
    (x = D_ref / D, R the time-independent model norm) is exponentiated and
    summed there (band_rule).  The time row of theta is not read."""
    th = _c(theta, np.float64)
    n = th.shape[1]
    n_t = int(n_t)
    tk = t_start + h * np.arange(n_t)
    big = np.repeat(th, n_t, axis=1)           # sample-major: [7, n * n_t]
    big[5] = np.tile(tk, n)
    Kt, Rt = lnL_terms(pt, big, nthreads)
    Kt = Kt.reshape(n, n_t)
    R = Rt.reshape(n, n_t)[:, 0]
    x = pt["d_ref"] / th[6]
    y = (x[:, None] * Kt).T                     # [n_t, n]
    return band_rule(y, -0.5 * R * x * x, M)


def lnL_psi_grid(pt, theta, u, nthreads: int = 0):
    """lnL [n, len(u)] at polarisation psi + u / 2 for every sample (the
    oracle's own lnL at each angle)."""
    th = _c(theta, np.float64)
    n = th.shape[1]
    u = np.asarray(u, np.float64)
    big = np.repeat(th, u.size, axis=1)
    big[2] = big[2] + np.tile(u / 2.0, n)
    return lnL(pt, big, nthreads).reshape(n, u.size)


def psi_coefficients(pt, theta, nthreads: int = 0):
    """(a, c1, c2) per sample of lnL as a function of u = 2 (psi' - psi),
    q(u) = a + Re(c1 e^{iu}) + Re(c2 e^{2iu}) (Eq. (ap:psiexp)): the exact
    five-point transform of lnL at u_j = 2 pi j / 5 (the polarisation series
    ends at 4 psi, so five points determine it)."""
    uj = 2.0 * np.pi * np.arange(5) / 5.0
    q = lnL_psi_grid(pt, theta, uj, nthreads)
    ch = q @ np.exp(-1j * np.outer(uj, np.arange(3))) / 5.0  # c^_0, c^_1, c^_2
    return ch[:, 0].real, 2.0 * ch[:, 1], 2.0 * ch[:, 2]


def erai_grid(pt):
    """(N_phi, N_psi) of the exact angular reconstruction (Eqs. (ap:angleharm),
    (ap:nyquist)) for a point's modes: at fixed other parameters lnL is a
    trigonometric polynomial of degree 2 in u = 2 psi and of degree 2 m_max in
    phiref (the data term carries e^{i m phi}, the model norm e^{i (m - m') phi}
    and e^{i (m + m') phi}), so N_psi = 5 and N_phi = 4 m_max + 1 equally
    spaced angles determine it."""
    m_max = int(np.max(np.abs(np.asarray(pt["lm"])[:, 1])))
    return 4 * m_max + 1, 5


def angle_coefficients(pt, theta, nthreads: int = 0):
    """The finite harmonic model of lnL in the angle offsets (alpha, u) from the
    sample's (phiref, 2 psi), Eq. (ap:angleharm):
        lnL(phi + alpha, psi + u / 2) = sum_{q, p} c[q, p] e^{i (q alpha + p u)},
    |q| <= (N_phi - 1) / 2, |p| <= 2, by the exact two-dimensional discrete
    Fourier transform of the oracle's own lnL on the N_phi x 5 product grid
    alpha_j = 2 pi j / N_phi, u_c = 2 pi c / 5.  Returns (c [n, N_phi, 5]
    indexed by (q mod N_phi, p mod 5), the grid's lnL [n, N_phi, 5])."""
    th = _c(theta, np.float64)
    n = th.shape[1]
    Nf, Np = erai_grid(pt)
    al = 2.0 * np.pi * np.arange(Nf) / Nf
    uc = 2.0 * np.pi * np.arange(Np) / Np
    big = np.repeat(th, Nf * Np, axis=1)       # sample-major, then phi, then psi
    big[4] = big[4] + np.tile(np.repeat(al, Np), n)
    big[2] = big[2] + np.tile(np.tile(uc / 2.0, Nf), n)
    L = lnL(pt, big, nthreads).reshape(n, Nf, Np)
    return np.fft.fft2(L, axes=(1, 2)) / (Nf * Np), L


def lnL_erai(pt, theta, n_phi: int, n_psi: int, nthreads: int = 0):
    """ln of the likelihood marginalised over phiref (uniform on [0, 2 pi)) and
    psi (uniform on [0, pi)) by exact-reconstruction adaptive integration
    (ERAI): the finite harmonic model from angle_coefficients, then its
    exponential averaged over the periodic product grid of n_phi x n_psi
    offsets alpha_a = 2 pi a / n_phi, psi offset pi b / n_psi (the periodic
    trapezoid rule on the torus, sized by the caller)."""
    C, _ = angle_coefficients(pt, theta, nthreads)
    n, Nf, Np = C.shape
    qf = np.fft.fftfreq(Nf, 1.0 / Nf)            # 0, 1, .., -1
    pf = np.fft.fftfreq(Np, 1.0 / Np)
    Ea = np.exp(1j * np.outer(2.0 * np.pi * np.arange(int(n_phi)) / int(n_phi), qf))  # [n_phi, Nf]
    Eu = np.exp(1j * np.outer(2.0 * np.pi * np.arange(int(n_psi)) / int(n_psi), pf))  # [n_psi, Np]
    V = np.einsum("aq,nqp,bp->nab", Ea, C, Eu).real.reshape(n, -1)
    out = np.full(n, np.nan)
    with np.errstate(invalid="ignore"):
        m = np.max(V, axis=1)
    ok = np.isfinite(m)
    out[ok] = m[ok] + np.log(np.mean(np.exp(V[ok] - m[ok, None]), axis=1))
    out[np.isnan(V).any(axis=1)] = np.nan
    return out


PSI_CELL_GL = 8          # Gauss-Legendre points per sub-interval of a cell


def psi_stationary(a, c1, c2):
    """The stationary points of q(u) = a + Re(c1 e^{iu}) + Re(c2 e^{2iu}) on
    the circle (Eq. (ap:psicells)): with z = e^{iu}, 2 i z^2 q'(u) = 0 is the
    quartic 2 c2 z^4 + c1 z^3 - conj(c1) z - 2 conj(c2) = 0, whose roots on
    the unit circle are the stationary points.  Roots within 1e-3 of the
    circle are taken as candidates and polished by Newton's method on q'(u);
    a candidate that does not settle on a root of q' is dropped (a pair of
    roots leaving the circle is an inflection, not an extremum).  Returns
    the sorted angles in [0, 2 pi)."""
    roots = np.roots([2.0 * c2, c1, 0.0, -np.conj(c1), -2.0 * np.conj(c2)])
    out = []
    for z in roots:
        if not np.isfinite(z) or abs(abs(z) - 1.0) > 1e-3:
            continue
        u = float(np.angle(z))
        for _ in range(30):
            e1 = np.exp(1j * u)
            d1 = -(c1 * e1).imag - 2.0 * (c2 * e1 * e1).imag
            d2 = -(c1 * e1).real - 4.0 * (c2 * e1 * e1).real
            if d2 == 0.0:
                break
            step = d1 / d2
            u -= step
            if abs(step) < 1e-15:
                break
        e1 = np.exp(1j * u)
        d1 = -(c1 * e1).imag - 2.0 * (c2 * e1 * e1).imag
        scale = abs(c1) + 2.0 * abs(c2)
        if abs(d1) <= 1e-9 * max(scale, 1e-300):
            out.append(u % (2.0 * np.pi))
    out = np.unique(np.round(np.sort(out), 13))
    return out


def psi_cell_breaks(width, sigma):
    """Sub-interval ends, as distances from a cell's higher end, of the
    curvature-sized rule: steps of 2 sigma out to 8 sigma, then doubling
    distances to the cell's far end (a monotone cell's integrand falls away
    from its top over a width sigma = A^{-1/2})."""
    d = [0.0]
    while d[-1] < width:
        nxt = 2.0 * sigma * len(d) if len(d) <= 4 else 2.0 * d[-1]
        d.append(min(width, nxt))
    return np.array(d)


def psi_cells_integral(a, c1, c2):
    """ln[(1 / 2 pi) int_0^{2 pi} e^{q(u)} du] by the cell partition of
    Eq. (ap:psicells): the stationary points cut the circle into cells on
    which q is monotone; each cell is integrated at a density set by its own
    curvature A = -q'' at its higher end: Gauss-Legendre (PSI_CELL_GL points)
    on the sub-intervals of psi_cell_breaks with sigma = min(A^{-1/2},
    width / 8) (a cell whose top is flat, A <= 0, takes width / 8: at least
    four sub-intervals per cell).  With fewer than two
    stationary points (a constant q) the circle is one cell."""
    st = psi_stationary(a, c1, c2)

    def q(u):
        e1 = np.exp(1j * np.asarray(u))
        return a + (c1 * e1).real + (c2 * e1 * e1).real

    def qpp(u):
        e1 = np.exp(1j * u)
        return -(c1 * e1).real - 4.0 * (c2 * e1 * e1).real

    if st.size < 2:
        cells = [(0.0, 2.0 * np.pi)]
    else:
        cells = [(st[k], st[k + 1]) for k in range(st.size - 1)] + [(st[-1], st[0] + 2.0 * np.pi)]
    x, w = np.polynomial.legendre.leggauss(PSI_CELL_GL)
    vals = []
    for lo, hi in cells:
        width = hi - lo
        top_lo = q(lo) >= q(hi)
        A = -qpp(lo if top_lo else hi)
        sigma = min(1.0 / np.sqrt(A), width / 8.0) if A > 0 else width / 8.0
        d = psi_cell_breaks(width, sigma)
        for j in range(d.size - 1):
            h = d[j + 1] - d[j]
            c = d[j] + 0.5 * h + 0.5 * h * x          # distances from the top
            uu = lo + c if top_lo else hi - c
            vals.append(q(uu) + np.log(0.5 * h * w))
    v = np.concatenate(vals)
    m = np.max(v)
    return m + np.log(np.sum(np.exp(v - m))) - np.log(2.0 * np.pi)


def lnL_pmarg(pt, theta, method="trapezoid", n_points=64, nthreads: int = 0):
    """ln of the likelihood marginalised over polarisation per sample, psi
    uniform on [0, pi) (u = 2 psi uniform on the circle):
      trapezoid: ln[(1/n) sum_j e^{lnL(psi + pi j / n)}], the oracle's lnL at
        each of the n angles (the periodic trapezoid rule);
      cells: the stationary-point cells of Eq. (ap:psicells)
        (psi_cells_integral) on the coefficients of psi_coefficients;
      laplace: Eq. (ap:psilaplace) at the dominant maximum of q(u) from
        psi_coefficients: ln L = q(u*) - ln(2 pi A) / 2 with A = -q''(u*),
        u* the best of 32 equally spaced points refined by Newton's method on
        q' = 0, where A >= 100 (the method's relative error O(1/A) is then
        below ~1e-3); otherwise (weak signal, or two maxima merging) the
        periodic trapezoid rule on 256 points of the same q."""
    if method == "cells":
        a, c1, c2 = psi_coefficients(pt, theta, nthreads)
        out = np.full(a.shape[0], np.nan)
        for i in range(a.shape[0]):
            if np.isfinite(a[i]) and np.isfinite(c1[i]) and np.isfinite(c2[i]):
                out[i] = psi_cells_integral(a[i], c1[i], c2[i])
        return out
    if method == "trapezoid":
        n = int(n_points)
        l = lnL_psi_grid(pt, theta, 2.0 * np.pi * np.arange(n) / n, nthreads)
        m = np.max(l, axis=1)
        out = np.full(l.shape[0], np.nan)
        ok = np.isfinite(m)
        out[ok] = m[ok] + np.log(np.sum(np.exp(l[ok] - m[ok, None]), axis=1)) - np.log(n)
        out[np.isnan(l).any(axis=1)] = np.nan
        return out
    a, c1, c2 = psi_coefficients(pt, theta, nthreads)
    out = np.empty(a.shape[0])
    for i in range(a.shape[0]):
        if not (np.isfinite(a[i]) and np.isfinite(c1[i]) and np.isfinite(c2[i])):
            out[i] = np.nan
            continue

        def q(u):
            e1 = np.exp(1j * u)
            return (a[i] + (c1[i] * e1).real + (c2[i] * e1 * e1).real,
                    -(c1[i] * e1).imag - 2.0 * (c2[i] * e1 * e1).imag,
                    -(c1[i] * e1).real - 4.0 * (c2[i] * e1 * e1).real)

        grid = np.pi * np.arange(32) / 16.0
        u = grid[int(np.argmax([q(g)[0] for g in grid]))]
        for _ in range(8):
            v, d1, d2 = q(u)
            if not d2 < 0.0:
                break
            u -= d1 / d2
        v, d1, d2 = q(u)
        A = -d2
        if A >= 100.0:
            out[i] = v - 0.5 * np.log(2.0 * np.pi * A)
        else:
            vals = np.array([q(g)[0] for g in 2.0 * np.pi * np.arange(256) / 256.0])
            mv = vals.max()
            out[i] = mv + np.log(np.mean(np.exp(vals - mv)))
    return out


def _to_physical(c):
    """Sampler coordinates (ra, dec, psi, cos incl, phiref, tref, ln dist) to
    the likelihood's (.., incl, .., .., dist); NaN incl outside [-1, 1]."""
    t = np.array(c, np.float64, copy=True)
    with np.errstate(invalid="ignore"):
        t[3] = np.where(np.abs(c[3]) <= 1.0, np.arccos(np.clip(c[3], -1.0, 1.0)), np.nan)
    t[6] = np.exp(c[6])
    return t


def hmc_log_prior(c, t_min, t_max, d_min, d_max, dmarg=False):
    """ln of the prior density in the sampler coordinates (up to a constant):
    the isotropic, uniform-in-volume prior of the samples (ra, psi, phiref
    periodic; sin dec, cos incl, tref uniform; p(D) ~ D^2 on [d_min, d_max])
    is, in (dec, ln D), ln cos dec + 3 ln D on the box, -inf outside.  With
    `dmarg` (distance marginalised in the likelihood) the distance row is not
    part of the target: no ln D term and no distance box."""
    c = np.asarray(c, np.float64)
    inside = (np.abs(c[1]) < np.pi / 2) & (np.abs(c[3]) <= 1.0) & (c[5] >= t_min) & (c[5] <= t_max)
    if not dmarg:
        inside &= (c[6] >= np.log(d_min)) & (c[6] <= np.log(d_max))
    with np.errstate(invalid="ignore", divide="ignore"):
        v = np.log(np.cos(c[1])) + (0.0 if dmarg else 3.0 * c[6])
    return np.where(inside, v, -np.inf)


def hmc_potential(pt, c, t_min, t_max, d_min, d_max, beta=1.0, dmarg=None):
    """(lnL, U = -beta lnL - ln prior, dU/dc) in the sampler coordinates: the
    tempered target L^beta p of Eq. (sampler-menu:tempered-target) (beta = 1:
    the posterior).  With dmarg = (d_min, d_max, n_nodes) of a distance
    prior, L is the likelihood marginalised over distance (grad_dmarg) and
    the distance row is not part of the target."""
    if dmarg is None:
        l, g = grad(pt, _to_physical(c))
    else:
        l, g = grad_dmarg(pt, c, *dmarg)
    lp = hmc_log_prior(c, t_min, t_max, d_min, d_max, dmarg is not None)
    gp = np.zeros_like(g)
    gp[1] = -np.tan(c[1])
    gp[6] = 0.0 if dmarg is not None else 3.0
    return l, -(beta * l + lp), -(beta * g + gp)


def hmc_trajectory(pt, c0, p0, sigma, eps, n_leapfrog, t_min, t_max, d_min, d_max, beta=1.0, dmarg=None):
    """n_leapfrog leapfrog steps from (c0, p0): half kick, drift c += eps
    sigma^2 p with cos incl folded back into [-1, 1] (period 4) and its
    momentum negated on odd folds, half kick.  Returns (c, p, lnL, U)."""
    sig = np.asarray(sigma, np.float64)[:, None]
    c = np.array(c0, np.float64, copy=True)
    p = np.array(p0, np.float64, copy=True)
    l, U, gU = hmc_potential(pt, c, t_min, t_max, d_min, d_max, beta, dmarg)
    for _ in range(int(n_leapfrog)):
        p = p - 0.5 * eps * gU
        c = c + eps * sig * sig * p
        out = np.isfinite(c[3]) & (np.abs(c[3]) > 1.0)
        r = np.mod(c[3][out] + 1.0, 4.0)
        c[3][out] = 1.0 - np.abs(r - 2.0)
        flip = np.zeros(c.shape[1], bool)
        flip[np.where(out)[0][r > 2.0]] = True
        p[3][flip] = -p[3][flip]
        l, U, gU = hmc_potential(pt, c, t_min, t_max, d_min, d_max, beta, dmarg)
        p = p - 0.5 * eps * gU
    return c, p, l, U


def hmc_step(pt, c0, z, u, sigma, eps, n_leapfrog, t_min, t_max, d_min, d_max, beta=1.0, dmarg=None):
    """One Metropolis-adjusted Hamiltonian Monte Carlo transition per chain
    (the gradient sampler of Sec. "Sampling the differentiable extrinsic
    likelihood"), with the random inputs given: momenta p = z / sigma (mass
    diag(sigma^-2)), n_leapfrog leapfrog steps of size eps on
    U = -lnL - ln prior (the half kicks with the oracle's gradient in the
    sampler coordinates plus the prior's, the drift c += eps sigma^2 p with
    cos incl reflected at +-1 and its momentum flipped), then acceptance when
    ln u < H0 - H1 with H = U + sum sigma^2 p^2 / 2.  Returns (c, lnL at c,
    accepted).  With beta < 1 the target is the tempered L^beta p of Eq.
    (sampler-menu:tempered-target) (the moves of an SMC ladder).  With dmarg =
    (d_min, d_max, n_nodes), the likelihood marginalised over distance: the
    distance row carries no momentum (p_6 = 0), so it is not moved."""
    sig = np.asarray(sigma, np.float64)[:, None]
    l0, U0, _ = hmc_potential(pt, c0, t_min, t_max, d_min, d_max, beta, dmarg)
    p0 = np.asarray(z, np.float64) / sig
    if dmarg is not None:
        p0 = p0.copy()
        p0[6] = 0.0
    H0 = U0 + 0.5 * np.sum(sig * sig * p0 * p0, axis=0)
    c, p, l1, U1 = hmc_trajectory(pt, c0, p0, sigma, eps, n_leapfrog, t_min, t_max, d_min, d_max, beta, dmarg)
    H1 = U1 + 0.5 * np.sum(sig * sig * p * p, axis=0)
    with np.errstate(invalid="ignore"):
        acc = np.log(np.asarray(u, np.float64)) < (H0 - H1)
    acc &= np.isfinite(H1)
    cout = np.where(acc[None, :], c, c0)
    return cout, np.where(acc, l1, l0), acc


NUTS_MAX_DH = 1000.0   # a leaf whose energy exceeds the start's by this much diverges


def _nuts_leapfrog(potential, c, p, gU, d, eps, sig2):
    """One leapfrog step of signed size d eps from (c, p) with gradient gU of
    the potential at c: half kick, drift with cos incl folded back into
    [-1, 1] (its momentum negated on odd folds), half kick.  Returns
    (c, p, gU, lnL, U) at the new point."""
    p = p - 0.5 * d * eps * gU
    c = c + d * eps * sig2 * p
    if np.isfinite(c[3]) and abs(c[3]) > 1.0:
        r = np.mod(c[3] + 1.0, 4.0)
        c = c.copy()
        c[3] = 1.0 - abs(r - 2.0)
        if r > 2.0:
            p = p.copy()
            p[3] = -p[3]
    l, U, g = potential(c[:, None])
    g = g[:, 0]
    p = p - 0.5 * d * eps * g
    return c, p, g, float(l[0]), float(U[0])


def _no_uturn(p_a, p_b, rho, sig2):
    """The generalised no-U-turn condition of a trajectory segment with edge
    momenta p_a, p_b and momentum sum rho (mass diag(1 / sig2))."""
    return float(np.dot(sig2 * p_a, rho)) > 0.0 and float(np.dot(sig2 * p_b, rho)) > 0.0


def nuts_chain(potential, c0, z, dirs, merges, leaves, sigma, eps, max_depth, frozen=()):
    """One No-U-Turn transition (multinomial NUTS with the generalised
    criterion) of one chain, the random numbers given: momenta p = z / sigma
    (mass diag(sigma^-2)); at depth j the trajectory doubles in direction
    -1 if dirs[j] < 1/2 else +1 by a subtree of 2^j leapfrog steps from that
    edge.  Within a subtree the leaves are built outward in order; leaf k
    (weight e^{-H}) replaces the subtree's candidate when the next of
    `leaves` is below its share of the subtree's weight so far, and after
    each leaf every completed aligned block of 2, 4, .. leaves is checked for
    a U-turn.  A U-turn inside the subtree, or a leaf whose energy exceeds
    the start's by NUTS_MAX_DH, discards the subtree and ends the transition;
    otherwise its candidate replaces the transition's with probability
    min(1, W_subtree / W_trajectory) against merges[j], the weights add, and
    a U-turn of the whole trajectory ends it.  At most max_depth doublings.
    potential(c [7, m]) -> (lnL, U, dU/dc).  The rows in `frozen` carry no
    momentum (they are not part of the target).  Returns (c, lnL, depth,
    leapfrog steps, divergent)."""
    sig = np.asarray(sigma, np.float64)
    sig2 = sig * sig
    c0 = np.asarray(c0, np.float64)
    p0 = np.asarray(z, np.float64) / sig
    for a in frozen:
        p0[a] = 0.0
    l0, U0, g0 = potential(c0[:, None])
    l0, U0, g0 = float(l0[0]), float(U0[0]), g0[:, 0]
    H0 = U0 + 0.5 * float(np.sum(sig2 * p0 * p0))
    if not np.isfinite(H0):  # a start outside the prior's support does not move
        return c0, l0, 0, 0, False
    left = right = (c0, p0, g0)
    cand, cand_l = c0, l0
    logW = 0.0
    rho = p0.copy()
    n_leaf = 0
    depth = 0
    div = False
    for j in range(int(max_depth)):
        d = -1.0 if dirs[j] < 0.5 else 1.0
        c, p, g = left if d < 0 else right
        sub_c, sub_l, logWs = None, None, -np.inf
        rho_s = np.zeros(7)
        first = []          # per leaf: its momentum and the running sum before it
        valid = True
        for k in range(2 ** j):
            c, p, g, l, U = _nuts_leapfrog(potential, c, p, g, d, eps, sig2)
            H = U + 0.5 * float(np.sum(sig2 * p * p))
            n_leaf += 1
            if not (H - H0 <= NUTS_MAX_DH):
                valid, div = False, True
                break
            lw = H0 - H
            logWs = np.logaddexp(logWs, lw)
            if leaves[n_leaf - 1] < np.exp(lw - logWs):
                sub_c, sub_l = c, l
            first.append((p.copy(), rho_s.copy()))
            rho_s = rho_s + p
            size = 2
            while size <= k + 1 and (k + 1) % size == 0:
                pa, sa = first[k + 1 - size]
                if not _no_uturn(pa, p, rho_s - sa, sig2):
                    valid = False
                    break
                size *= 2
            if not valid:
                break
        if not valid:
            break
        depth = j + 1
        if merges[j] < np.exp(logWs - logW):
            cand, cand_l = sub_c, sub_l
        logW = np.logaddexp(logW, logWs)
        rho = rho + rho_s
        if d < 0:
            left = (c, p, g)
        else:
            right = (c, p, g)
        if not _no_uturn(left[1], right[1], rho, sig2):
            break
    return cand, cand_l, depth, n_leaf, div


def nuts_step(pt, c0, z, dirs, merges, leaves, sigma, eps, max_depth, t_min, t_max, d_min, d_max, beta=1.0,
              dmarg=None):
    """nuts_chain for every chain on the target L^beta p in the sampler
    coordinates (the potential of hmc_potential).  c0, z [7, n]; dirs,
    merges [max_depth, n]; leaves [2^max_depth - 1, n].  With dmarg =
    (d_min, d_max, n_nodes), the likelihood marginalised over distance and the
    distance row frozen.  Returns (c [7, n], lnL [n], depth [n], steps [n],
    divergent [n])."""
    c0 = np.asarray(c0, np.float64)
    n = c0.shape[1]

    def pot(c):
        return hmc_potential(pt, c, t_min, t_max, d_min, d_max, beta, dmarg)

    out = np.empty_like(c0)
    ll = np.empty(n)
    dep = np.zeros(n, np.int32)
    st = np.zeros(n, np.int32)
    dv = np.zeros(n, bool)
    for i in range(n):
        c, l, dd, ss, vv = nuts_chain(pot, c0[:, i], z[:, i], dirs[:, i], merges[:, i], leaves[:, i], sigma, eps,
                                      max_depth, frozen=(6,) if dmarg is not None else ())
        out[:, i], ll[i], dep[i], st[i], dv[i] = c, l, dd, ss, vv
    return out, ll, dep, st, dv


def rwm_chain(log_target, c0, z, u, cov, scale, l0=None):
    """One random-walk Metropolis move per column (the move of the adaptive
    cloud after resampling, Sec. "Mode coverage, adaptive clouds, and
    evidence": a proposal covariance estimated from the cloud): c' = c + L z
    with L L^T = scale cov (Cholesky), accepted when ln u < ln pi(c') -
    ln pi(c); a NaN or -inf target at c' rejects.  log_target(c) -> [n];
    l0: ln pi at c0 if known.  Returns (c, ln pi, accepted)."""
    c0 = np.asarray(c0, np.float64)
    L = np.linalg.cholesky(scale * np.asarray(cov, np.float64))
    c1 = c0 + L @ np.asarray(z, np.float64)
    t0 = log_target(c0) if l0 is None else np.asarray(l0, np.float64)
    t1 = log_target(c1)
    with np.errstate(invalid="ignore"):
        acc = np.log(np.asarray(u, np.float64)) < t1 - t0
    acc &= np.isfinite(t1)
    return np.where(acc, c1, c0), np.where(acc, t1, t0), acc


def rwm_step(pt, c0, z, u, cov, scale, t_min, t_max, d_min, d_max, lnL0, beta=1.0):
    """The move on the tempered target L^beta p of Eq.
    (sampler-menu:tempered-target) in the sampler coordinates (the prior of
    hmc_log_prior; a proposal outside its box is rejected): accepted when
    ln u < beta (lnL' - lnL) + ln p(c') - ln p(c), with L^0 = 1.  lnL0: lnL at
    c0.  Returns (c, lnL, accepted)."""
    c0 = np.asarray(c0, np.float64)
    lnL0 = np.asarray(lnL0, np.float64)
    L = np.linalg.cholesky(scale * np.asarray(cov, np.float64))
    c1 = c0 + L @ np.asarray(z, np.float64)
    lp0 = hmc_log_prior(c0, t_min, t_max, d_min, d_max)
    lp1 = hmc_log_prior(c1, t_min, t_max, d_min, d_max)
    inside = np.isfinite(lp1)
    l1 = np.full(c0.shape[1], np.nan)
    if inside.any():
        l1[inside] = lnL(pt, _to_physical(c1[:, inside]))
    with np.errstate(invalid="ignore"):
        d = (0.0 if beta == 0.0 else beta * (l1 - lnL0)) + lp1 - lp0
        acc = inside & (np.log(np.asarray(u, np.float64)) < d)
    return np.where(acc, c1, c0), np.where(acc, l1, lnL0), acc


def _lse(v):
    v = np.asarray(v, np.float64)
    m = np.max(v)
    if not np.isfinite(m):
        return m if not np.isnan(v).any() else np.nan
    return m + np.log(np.sum(np.exp(v - m)))


def _tempered(lnL, dbeta):
    """dbeta ln L with L^0 = 1 also where L = 0 (ln L = -inf)."""
    lnL = np.asarray(lnL, np.float64)
    return np.zeros_like(lnL) if dbeta == 0.0 else dbeta * lnL


def smc_cess(lnW, lnL, dbeta):
    """Conditional effective sample size fraction of the incremental weights
    r_i = L_i^dbeta of Eq. (sampler-menu:smc-update) under the current
    normalised weights W: (sum W r)^2 / sum W r^2, in (0, 1] (1 at dbeta = 0).
    Computed in log space."""
    lnW = np.asarray(lnW, np.float64)
    lnL = np.asarray(lnL, np.float64)
    lw = lnW - _lse(lnW)
    return float(np.exp(2.0 * _lse(lw + _tempered(lnL, dbeta)) - _lse(lw + _tempered(lnL, 2.0 * dbeta))))


def smc_next_beta(lnW, lnL, beta, target):
    """The next rung of the tempering ladder chosen from the effective sample
    size of the incremental weights: the largest beta' in (beta, 1] with
    smc_cess(beta' - beta) >= target (the fraction is non-increasing in the
    step: it is 2 K(d) - K(2 d) for the convex cumulant function K), 1 if the
    whole remaining step qualifies; by bisection to the rounding of the
    step."""
    rest = 1.0 - beta
    if smc_cess(lnW, lnL, rest) >= target:
        return 1.0
    lo, hi = 0.0, rest
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if smc_cess(lnW, lnL, mid) >= target:
            lo = mid
        else:
            hi = mid
    return beta + lo


def smc_update(lnW, lnL, beta, beta_new):
    """The normalisation update of Eq. (sampler-menu:smc-update): with W the
    normalised weights at beta and r_i = L_i^(beta_new - beta),
    ln(Z_new / Z_old) = ln sum_i W_i r_i, and the new normalised log weights
    ln W_i + ln r_i - that.  Returns (dlnZ, lnW_new)."""
    lnW = np.asarray(lnW, np.float64)
    lw = lnW - _lse(lnW)
    v = lw + _tempered(lnL, beta_new - beta)
    d = _lse(v)
    return d, v - d


def systematic_resample(lnW, u):
    """Systematic resampling of n draws from the normalised weights with one
    uniform u in [0, 1): a_i = the first k whose cumulative weight exceeds
    (i + u) / n."""
    lnW = np.asarray(lnW, np.float64)
    n = lnW.size
    w = np.exp(lnW - _lse(lnW))
    C = np.cumsum(w)
    U = (np.arange(n) + u) / n
    a = np.searchsorted(C, U, side="right")
    return np.minimum(a, n - 1)


# ---------------------------------------------------------------------------
# The importance-sampling normalisation of Eq. (sampler-menu:is) with the
# defensive proposal of Sec. "Mode coverage, adaptive clouds, and evidence":
# q = alpha p + (1 - alpha) sum_m a_m N(mu_m, s C_m), one Gaussian component
# per recovered mode, fitted by the moments of that mode's chains or cloud,
# with s > 1 widening its tails.  Coordinates are the samplers' (ra, dec, psi,
# cos incl, phiref, tref, ln D); ra, psi and phiref are periodic, so a
# component is the density of its Gaussian draw taken modulo those periods.

IS_PERIODS = ((0, 2.0 * np.pi), (2, np.pi), (4, 2.0 * np.pi))


def _rows(rows):
    """The sampled rows of a bit mask (bit j: row j), all seven for None."""
    return list(range(7)) if rows is None else [j for j in range(7) if (int(rows) >> j) & 1]


def is_log_prior(c, t_min, t_max, d_min, d_max, rows=None):
    """ln p of the samples' prior, normalised, in the sampler coordinates on
    the box ra, phiref in [0, 2 pi), psi in [0, pi), |dec| < pi/2,
    |cos incl| <= 1, tref in [t_min, t_max], D in [d_min, d_max]: the product
    of the one-dimensional densities 1/(2 pi), cos(dec)/2, 1/pi, 1/2,
    1/(2 pi), 1/(t_max - t_min) and 3 D^3 / (d_max^3 - d_min^3) (p(D) ~ D^2
    and dD = D d ln D); -inf outside the box.  With `rows` (a bit mask), the
    marginal density of those rows alone."""
    c = np.asarray(c, np.float64)
    S = _rows(rows)
    inside = [(c[0] >= 0.0) & (c[0] < 2 * np.pi), np.abs(c[1]) < np.pi / 2, (c[2] >= 0.0) & (c[2] < np.pi),
              np.abs(c[3]) <= 1.0, (c[4] >= 0.0) & (c[4] < 2 * np.pi), (c[5] >= t_min) & (c[5] <= t_max),
              (c[6] >= np.log(d_min)) & (c[6] <= np.log(d_max))]
    with np.errstate(invalid="ignore", divide="ignore"):
        dens = [np.full(c.shape[1], -np.log(2 * np.pi)), np.log(np.cos(c[1])) - np.log(2.0),
                np.full(c.shape[1], -np.log(np.pi)), np.full(c.shape[1], -np.log(2.0)),
                np.full(c.shape[1], -np.log(2 * np.pi)), np.full(c.shape[1], -np.log(t_max - t_min)),
                np.log(3.0) + 3.0 * c[6] - np.log(d_max ** 3 - d_min ** 3)]
    ok = np.ones(c.shape[1], bool)
    v = np.zeros(c.shape[1])
    for j in S:
        ok &= inside[j]
        v = v + dens[j]
    return np.where(ok, v, -np.inf)


def cloud_moments(c, lnw=None):
    """Weighted mean and covariance of a cloud (the moments that fit one
    component): with normalised weights W_i (equal without lnw),
    mu = sum_i W_i c_i and C = sum_i W_i (c_i - mu)(c_i - mu)^T, over the
    samples of non-zero weight.  NaN when no sample has weight or a weight is
    NaN."""
    c = np.asarray(c, np.float64)
    n = c.shape[1]
    if n == 0:
        return np.full(7, np.nan), np.full((7, 7), np.nan)
    if lnw is None:
        W = np.full(n, 1.0 / n)
    else:
        lw = np.asarray(lnw, np.float64)
        t = _lse(lw)
        if not np.isfinite(t):
            return np.full(7, np.nan), np.full((7, 7), np.nan)
        W = np.exp(lw - t)
    keep = W > 0
    mu = np.sum(W[keep] * c[:, keep], axis=1)
    d = c[:, keep] - mu[:, None]
    return mu, (W[keep] * d) @ d.T


def wrapped_normal_logpdf(c, mu, cov, images=6, rows=None):
    """ln of the density, at the columns of c, of x ~ N(mu, cov) with ra, psi
    and phiref taken modulo their periods: the sum of the Gaussian density
    over the lattice of periodic images of each point, here the images within
    `images` periods of the one nearest the mean in each periodic row.  With
    `rows`, the Gaussian of those rows alone (mean and covariance restricted
    to them)."""
    S = _rows(rows)
    c = np.asarray(c, np.float64)[S]
    cov = np.asarray(cov, np.float64)[np.ix_(S, S)]
    Cinv = np.linalg.inv(cov)
    _, logdet = np.linalg.slogdet(cov)
    d = c - np.asarray(mu, np.float64)[S][:, None]
    per = [(S.index(j), P) for j, P in IS_PERIODS if j in S]
    for j, P in per:
        d[j] -= P * np.round(d[j] / P)
    ks = np.arange(-images, images + 1, dtype=np.float64)
    grids = np.meshgrid(*([ks] * len(per)), indexing="ij") if per else []
    off = np.zeros((grids[0].size if per else 1, len(S)))
    for g, (j, P) in zip(grids, per):
        off[:, j] = g.ravel() * P
    out = np.empty(d.shape[1])
    for s0 in range(0, d.shape[1], 128):
        e = d[None, :, s0:s0 + 128] + off[:, :, None]       # [image, rows, chunk]
        q = -0.5 * np.sum(e * np.matmul(Cinv, e), axis=1)   # [image, chunk]
        m = np.max(q, axis=0)
        out[s0:s0 + 128] = m + np.log(np.sum(np.exp(q - m), axis=0))
    return out - 0.5 * logdet - 0.5 * len(S) * np.log(2 * np.pi)


def mixture_log_density(c, alpha, a, mean, cov, scale, t_min, t_max, d_min, d_max, rows=None):
    """ln q of the defensive mixture q = alpha p + (1 - alpha) sum_m a_m
    N_m, N_m the wrapped Gaussian of mean mean[m] and covariance
    scale cov[m]; with `rows`, the density of those rows alone."""
    c = np.asarray(c, np.float64)
    parts = []
    if alpha > 0:
        parts.append(np.log(alpha) + is_log_prior(c, t_min, t_max, d_min, d_max, rows))
    for m in range(len(a)):
        if a[m] > 0 and alpha < 1:
            parts.append(np.log((1.0 - alpha) * a[m]) +
                         wrapped_normal_logpdf(c, mean[m], scale * np.asarray(cov[m]), rows=rows))
    P = np.array(parts)
    mx = np.max(P, axis=0)
    with np.errstate(invalid="ignore"):
        out = mx + np.log(np.sum(np.exp(P - mx), axis=0))
    return np.where(np.isneginf(mx), -np.inf, out)


def _prior_draw(w, t_min, t_max, d_min, d_max):
    return np.array([2 * np.pi * w[0], np.arcsin(2 * w[1] - 1), np.pi * w[2], 2 * w[3] - 1, 2 * np.pi * w[4],
                     t_min + (t_max - t_min) * w[5], np.log(d_min ** 3 + w[6] * (d_max ** 3 - d_min ** 3)) / 3.0])


def mixture_draw(alpha, a, mean, cov, scale, t_min, t_max, d_min, d_max, z, v, u, rows=None):
    """Independent draws from q with the caller's random numbers: u [n] in
    [0, 1) picks the prior when u < alpha, else component m, the first with
    u < alpha + (1 - alpha) (a_0 + .. + a_m) (the last one if none); a prior
    draw takes the inverse distribution functions of v [7, n] (ra = 2 pi v0,
    dec = asin(2 v1 - 1), psi = pi v2, cos incl = 2 v3 - 1, phiref = 2 pi v4,
    tref = t_min + (t_max - t_min) v5, ln D = ln(d_min^3 + v6 (d_max^3 -
    d_min^3)) / 3); a component draw is mean[m] + L z with L L^T = scale
    cov[m] (Cholesky), z [7, n] standard normals, then ra, psi, phiref
    reduced into [0, P).  With `rows`, a component draws those rows (the
    Cholesky factor of their covariance applied to z at those rows) and the
    others from the prior as a prior draw does.  Returns
    (c [7, n], comp [n]: -1 for the prior)."""
    z = np.asarray(z, np.float64)
    v = np.asarray(v, np.float64)
    u = np.asarray(u, np.float64)
    S = _rows(rows)
    n = u.size
    c = np.empty((7, n))
    comp = np.full(n, -1, np.int64)
    ncomp = len(a)
    cum = np.cumsum(np.asarray(a, np.float64))
    T = alpha + (1.0 - alpha) * cum
    for i in range(n):
        c[:, i] = _prior_draw(v[:, i], t_min, t_max, d_min, d_max)
        if u[i] < alpha or ncomp == 0:
            continue
        m = int(np.argmax(u[i] < T)) if np.any(u[i] < T) else ncomp - 1
        L = np.linalg.cholesky(scale * np.asarray(cov[m], np.float64)[np.ix_(S, S)])
        x = np.asarray(mean[m], np.float64)[S] + L @ z[S, i]
        for k, j in enumerate(S):
            P = dict(IS_PERIODS).get(j)
            c[j, i] = x[k] - P * np.floor(x[k] / P) if P else x[k]
        comp[i] = m
    return c, comp


def mixture_is(alpha, a, mean, cov, scale, t_min, t_max, d_min, d_max, z, v, u, rows=None):
    """Draws from the defensive mixture and their log weights ln p - ln q of
    Eq. (sampler-menu:is), so that ln Z = lnZ(lnL(theta), lnw).  Returns
    (theta [7, n] in the likelihood's coordinates, lnw [n], comp [n]).  A draw
    outside the prior's box has lnw = -inf and is returned moved onto the box
    (dec, cos incl, tref and ln D clamped), so its likelihood is finite.
    With `rows`, p and q are the densities of those rows alone: the weights of
    a likelihood marginalised over the other rows (their draws are the
    prior's and do not enter the weight)."""
    box = (t_min, t_max, d_min, d_max)
    c, comp = mixture_draw(alpha, a, mean, cov, scale, *box, z, v, u, rows)
    lp = is_log_prior(c, *box, rows)
    lq = mixture_log_density(c, alpha, a, mean, cov, scale, *box, rows)
    lnw = np.where(np.isfinite(lp), lp - lq, -np.inf)
    cc = c.copy()
    cc[1] = np.clip(cc[1], -np.pi / 2, np.pi / 2)
    cc[3] = np.clip(cc[3], -1.0, 1.0)
    cc[5] = np.clip(cc[5], t_min, t_max)
    cc[6] = np.clip(cc[6], np.log(d_min), np.log(d_max))
    th = cc.copy()
    th[3] = np.arccos(cc[3])
    th[6] = np.exp(cc[6])
    return th, lnw, comp


def rotation_harmonics(det_tensor, dec, psi):
    """A_n, n = -2..2, of F(g) = sum_n A_n e^{i n g} over the Greenwich hour
    angle g at fixed dec, psi (Eq. (slowrot:Fharm))."""
    out = np.zeros(10)
    _load().oracle_rotation_harmonics(_ptr(_c(det_tensor, np.float64)), float(dec), float(psi), _ptr(out))
    return out[0::2] + 1j * out[1::2]


def wide_coef(pt, theta1):
    """Composite coefficients C~ [K, n_a] and arrival times t_k [K] of one sample
    (Eqs. (slowrot:postphase), (fsize:bp))."""
    pk = _pack_wide(pt)
    K, n_a = pk.cp.K, pk.cp.n_a
    C = np.zeros(2 * K * n_a)
    tk = np.zeros(K)
    _load().oracle_wide_coef(ctypes.byref(pk.cp), _ptr(_c(theta1, np.float64)), _ptr(C), _ptr(tk))
    return (C[0::2] + 1j * C[1::2]).reshape(K, n_a), tk


def lnL_wide(pt, theta, nthreads: int = 0) -> np.ndarray:
    """Composite-index lnL, Eq. (slowrot:lnL:Decomposed), for theta [7, n]."""
    th = _c(theta, np.float64)
    n = th.shape[1]
    out = np.empty(n)
    pk = _pack_wide(pt)
    _load().oracle_lnL_wide(ctypes.byref(pk.cp), n, _ptr(th), _ptr(out), int(nthreads))
    return out


def pregrid(q, r: int):
    """Fourier refinement of a sampled complex series, Eq. (q-time-pregrid).

    Append the reversed copy (so the periodic extension is continuous), FFT,
    zero-pad the spectrum by r (the Nyquist bin split in halves between +/-),
    inverse FFT times r, and keep the samples spanning the original window:
    (N-1) r + 1 fine samples at spacing h/r, fine[j r] == q[j].
    """
    q = np.asarray(q, np.complex128)
    n = q.shape[-1]
    refl = np.concatenate([q, q[..., ::-1]], axis=-1)
    L = 2 * n
    spec = np.fft.fft(refl, axis=-1)
    big = np.zeros(q.shape[:-1] + (L * r,), np.complex128)
    half = L // 2
    big[..., :half] = spec[..., :half]
    big[..., -half + 1:] = spec[..., half + 1:]
    big[..., half] = 0.5 * spec[..., half]
    big[..., L * r - half] = 0.5 * spec[..., half]
    fine = np.fft.ifft(big, axis=-1) * r
    return fine[..., : (n - 1) * r + 1]
