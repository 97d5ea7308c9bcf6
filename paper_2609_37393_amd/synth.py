"""Seeded synthetic inputs shaped like the paper's workloads.

This module is shared by the tests, the oracle checks and the benchmark, and
it deliberately contains none of the likelihood's arithmetic: no antenna
pattern, arrival-time, harmonic, interpolation or likelihood code.  It only

* draws detector geometry (response tensors, positions),
* draws smooth two-sided mode spectra h_lm(f) and per-detector noise weights,
* synthesises detector data from *given* response-folded coefficients and
  arrival times (the injection is an input: the caller decides what it is),
* forms the precomputed arrays Q, U, V by their inner-product definitions
  (Eq. (QUV): Q_{k,lm}(t) = <T_t h_lm | d>_k, U = <h_lm|h_l'm'>, V = <h*_lm|h_l'm'>),
* draws extrinsic samples from the priors of the workloads.

Inner product: <a|b> = 2 sum_f df conj(a(f)) b(f) / S_k(f) over the two-sided
grid |f| >= f_lo (the discretised form of the paper's definition), so the
per-bin weight is w_k(f) = 2 df / S_k(f).

The Q table is evaluated exactly at the requested sample rate (an inverse FFT
of the band-limited spectrum), i.e. the table an ideal Fourier refinement of
the native-rate series converges to.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299792458.0
R_EARTH_M = 6371.0e3

# Mode list in importance order; every workload's mode set is a prefix of it.
MODE_ORDER = [
    (2, 2), (2, -2), (2, 1), (2, -1), (3, 3), (3, -3), (2, 0), (3, 2), (3, -2),
    (4, 4), (4, -4), (3, 1), (3, -1), (4, 3), (4, -3), (3, 0), (4, 2), (4, -2),
    (4, 1), (4, -1), (4, 0),
]


def _rng(seed, *tags):
    return np.random.default_rng(np.random.SeedSequence([int(seed)] + [int(t) for t in tags]))


def modes(M: int) -> np.ndarray:
    if not 1 <= M <= len(MODE_ORDER):
        raise ValueError(f"M must be in 1..{len(MODE_ORDER)}")
    return np.array(MODE_ORDER[:M], dtype=np.int32)


def network(K: int, seed: int, radius_m: float = R_EARTH_M):
    """L-shaped detectors at random points of a sphere of the given radius.

    det_tensor_k = (x x^T - y y^T)/2 with orthonormal arm directions x, y;
    det_pos_k in light-seconds; gmst uniform in [0, 2 pi).
    """
    rng = _rng(seed, 11)
    D = np.zeros((K, 3, 3))
    R = np.zeros((K, 3))
    arms = np.zeros((K, 2, 3))
    for k in range(K):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        R[k] = n * radius_m / C_LIGHT
        x = rng.normal(size=3)
        x /= np.linalg.norm(x)
        y = rng.normal(size=3)
        y -= x * np.dot(x, y)
        y /= np.linalg.norm(y)
        D[k] = 0.5 * (np.outer(x, x) - np.outer(y, y))
        arms[k, 0] = x
        arms[k, 1] = y
    gmst = float(rng.uniform(0.0, 2.0 * np.pi))
    return {"det_tensor": D, "det_pos": R, "gmst": gmst, "det_arms": arms}


def freq_grid(f_hi: int = 1700):
    """Integer two-sided frequency grid -f_hi..f_hi (df = 1 Hz, 1-s period)."""
    return np.arange(-f_hi, f_hi + 1, dtype=np.float64)


def mode_spectra(M, seed: int, f_lo: float = 20.0, f_hi: int = 1700,
                 f_c: float = 150.0, width_s: float = 1e-3):
    """Two-sided spectra G_lm(f) of Gaussian-enveloped chirp peaks.

    env(f) = exp(-(|f| - f_c)^2 / (2 sigma_f^2)), sigma_f = 1/(2 pi width),
    times a seeded phase exp(i(phi0 + 2 pi f tau + beta f^2)) per mode and
    sign of f.  Quadrupole modes get amplitude 1, the others 0.1-0.5.
    """
    lm = modes(M) if np.isscalar(M) else np.asarray(M, np.int32)
    M = lm.shape[0]
    rng = _rng(seed, 22)
    f = freq_grid(f_hi)
    sigma_f = 1.0 / (2.0 * np.pi * width_s)
    env = np.exp(-((np.abs(f) - f_c) ** 2) / (2.0 * sigma_f**2))
    env[np.abs(f) < f_lo] = 0.0
    G = np.zeros((M, f.size), np.complex128)
    for i, (l, m) in enumerate(lm):
        amp = 1.0 if l == 2 and abs(m) == 2 else rng.uniform(0.1, 0.5)
        phi0 = rng.uniform(0, 2 * np.pi, size=2)
        tau = rng.normal(0.0, 2e-4, size=2)
        beta = rng.normal(0.0, 2e-6, size=2)
        pos = f > 0
        ph = np.where(pos, phi0[0] + 2 * np.pi * f * tau[0] + beta[0] * f**2,
                      phi0[1] + 2 * np.pi * f * tau[1] + beta[1] * f**2)
        # negative frequencies carry less power (a mode is mostly one-sided)
        side = np.where(pos, 1.0, rng.uniform(0.2, 0.6))
        G[i] = amp * side * env * np.exp(1j * ph)
    return f, G


def noise_weights(K: int, f: np.ndarray, seed: int, df: float = 1.0):
    """w_k(f) = 2 df / S_k(f) for smooth seeded PSDs S_k (scale-free)."""
    rng = _rng(seed, 33)
    w = np.zeros((K, f.size))
    af = np.maximum(np.abs(f), 1.0)
    for k in range(K):
        f0 = rng.uniform(40.0, 80.0)
        f1 = rng.uniform(300.0, 900.0)
        S = (f0 / af) ** 4 + 1.0 + (af / f1) ** 2
        S *= rng.uniform(0.5, 2.0)
        w[k] = 2.0 * df / S
    return w


def random_injection(K: int, M: int, seed: int):
    """Generic rank-one response-folded coefficients z_k = a_k y and arrival times.

    Not tied to any extrinsic parameters (no response arithmetic here): a
    complex vector y over modes, a complex detector factor a_k with |a_k| <= 1,
    and arrival times within the geocentric light-travel span.
    """
    rng = _rng(seed, 44)
    y = rng.normal(size=M) + 1j * rng.normal(size=M)
    y[:2] *= 4.0  # quadrupole-dominated
    y /= np.linalg.norm(y)
    a = rng.uniform(0.3, 1.0, size=K) * np.exp(1j * rng.uniform(0, 2 * np.pi, size=K))
    z = a[:, None] * y[None, :]
    tk = rng.uniform(-0.02, 0.02, size=K)
    return {"z": z, "tk": tk}


def _strain(z, tk, f, G):
    """h_k(f) = 1/2 e^{-2 pi i f t_k} [sum z_lm G_lm(f) + sum conj(z_lm) conj(G_lm(-f))]."""
    Gm = G[:, ::-1]  # G(-f) on the symmetric grid
    hY = z @ G                      # [K, nf]
    hYc = np.conj(z) @ np.conj(Gm)  # [K, nf]
    return 0.5 * np.exp(-2j * np.pi * f[None, :] * tk[:, None]) * (hY + hYc)


def make_point(K: int, M: int, n_t: int, fs: float, snr: float, seed: int,
               injection=None, net=None, noise: bool = True, d_ref: float = 100.0,
               keep_spectra: bool = False, lm=None):
    """One intrinsic point: Q [K, M, n_t] on t_j = t0 + j/fs with t0 = -(n_t//2)/fs,
    U, V [K, M, M], the network, and the injection scaled to network SNR `snr`.

    injection: {"z": [K, M] complex, "tk": [K]} (response-folded coefficients and
    arrival times); default is `random_injection`.  lm: explicit [M, 2] mode
    list (default: the first M of MODE_ORDER).
    """
    lm = modes(M) if lm is None else np.asarray(lm, np.int32)
    M = lm.shape[0]
    f, G = mode_spectra(lm, seed)
    w = noise_weights(K, f, seed)
    net = net if net is not None else network(K, seed)
    inj = injection if injection is not None else random_injection(K, M, seed)
    z = np.asarray(inj["z"], np.complex128)
    tk = np.asarray(inj["tk"], np.float64)
    h = _strain(z, tk, f, G)
    rho2 = float(np.sum(w * np.abs(h) ** 2))
    scale = snr / np.sqrt(rho2) if rho2 > 0 else 0.0
    h *= scale
    d = h.copy()
    if noise:
        rng = _rng(seed, 55)
        pos = f > 0
        nz = np.zeros((K, f.size), np.complex128)
        sig = np.sqrt(1.0 / np.where(w > 0, w, np.inf))
        nz[:, pos] = sig[:, pos] * (rng.normal(size=(K, pos.sum())) +
                                   1j * rng.normal(size=(K, pos.sum()))) / np.sqrt(2.0)
        # Hermitian symmetry n(-f) = conj(n(f)) for real noise (symmetric grid)
        nz[:, f < 0] = np.conj(nz[:, pos][:, ::-1])
        d = d + nz
    # U, V by definition
    U = np.einsum("kf,if,jf->kij", w, np.conj(G), G)
    V = np.einsum("kf,if,jf->kij", w, G[:, ::-1], G)
    # Q_{k,lm}(t) = sum_f w_k e^{2 pi i f t} conj(G_lm(f)) d_k(f), evaluated by an
    # inverse FFT at rate fs (period 1 s, df = 1 Hz).
    nfft = int(round(fs))
    if abs(nfft - fs) > 1e-9 or f[-1] >= fs / 2:
        raise ValueError("fs must be an integer rate above twice the band edge")
    X = np.zeros((K, M, nfft), np.complex128)
    bins = np.mod(f.astype(np.int64), nfft)
    X[:, :, bins] = w[:, None, :] * np.conj(G)[None, :, :] * d[:, None, :]
    full = np.fft.ifft(X, axis=-1) * nfft
    j0 = n_t // 2
    idx = np.mod(np.arange(n_t) - j0, nfft)
    Q = full[:, :, idx]
    pt = {
        "lm": lm,
        "t0": -j0 / fs,
        "dt": 1.0 / fs,
        "Q": Q,
        "U": U,
        "V": V,
        "det_tensor": net["det_tensor"],
        "det_pos": net["det_pos"],
        "det_arms": net.get("det_arms"),
        "gmst": net["gmst"],
        "d_ref": float(d_ref),
        "snr": float(snr),
        "inj_scale": float(scale),
        "half_dd": 0.5 * float(np.sum(w * np.abs(d) ** 2)),
    }
    if keep_spectra:
        pt["spectra"] = {"f": f, "G": G, "w": w, "d": d, "h": h, "z": z * scale, "tk": tk}
    return pt


def prior_samples(n: int, seed: int, tref_s: float = 0.01, dmin: float = 10.0,
                  dmax: float = 1000.0) -> np.ndarray:
    """theta [7, n]: ra U[0,2pi), sin dec U[-1,1], psi U[0,pi), cos incl U[-1,1],
    phiref U[0,2pi), tref U[-tref_s, tref_s], p(D) ~ D^2 on [dmin, dmax]."""
    rng = _rng(seed, 66)
    th = np.empty((7, n))
    th[0] = rng.uniform(0.0, 2 * np.pi, n)
    th[1] = np.arcsin(rng.uniform(-1.0, 1.0, n))
    th[2] = rng.uniform(0.0, np.pi, n)
    th[3] = np.arccos(rng.uniform(-1.0, 1.0, n))
    th[4] = rng.uniform(0.0, 2 * np.pi, n)
    th[5] = rng.uniform(-tref_s, tref_s, n)
    u = rng.uniform(0.0, 1.0, n)
    th[6] = (dmin**3 + u * (dmax**3 - dmin**3)) ** (1.0 / 3.0)
    return th


def weighted_samples(n: int, seed: int, sigma_t: float = 0.003, dmin: float = 10.0,
                     dmax: float = 1000.0, tref_s: float = 0.01):
    """Importance draws: t_ref ~ N(0, sigma_t) truncated to +-tref_s, D log-uniform;
    returns (theta, lnw) with lnw = ln p - ln q for the prior of `prior_samples`."""
    rng = _rng(seed, 77)
    th = prior_samples(n, seed)
    t = rng.normal(0.0, sigma_t, size=4 * n)
    t = t[np.abs(t) <= tref_s][:n]
    while t.size < n:
        extra = rng.normal(0.0, sigma_t, size=n)
        t = np.concatenate([t, extra[np.abs(extra) <= tref_s]])[:n]
    th[5] = t
    lo, hi = np.log(dmin), np.log(dmax)
    th[6] = np.exp(rng.uniform(lo, hi, n))
    # ln p: uniform t on [-tref_s, tref_s], D^2 on [dmin, dmax]
    from math import erf, sqrt
    norm_t = erf(tref_s / (sigma_t * sqrt(2.0)))
    lnp_t = -np.log(2 * tref_s)
    lnq_t = -0.5 * (th[5] / sigma_t) ** 2 - np.log(sigma_t * np.sqrt(2 * np.pi) * norm_t)
    lnp_d = np.log(3.0 * th[6] ** 2 / (dmax**3 - dmin**3))
    lnq_d = -np.log(th[6] * (hi - lo))
    return th, (lnp_t - lnq_t) + (lnp_d - lnq_d)


def perturbed_samples(theta0, sigma, n: int, seed: int) -> np.ndarray:
    """theta0 + sigma * z (z standard normal) in (ra, dec, psi, cos incl, phiref,
    tref, ln dist) coordinates; returns theta [7, n] in the sampler's variables."""
    rng = _rng(seed, 88)
    z = rng.normal(size=(7, n))
    th0 = np.asarray(theta0, np.float64)
    sig = np.asarray(sigma, np.float64)
    th = np.empty((7, n))
    th[0] = th0[0] + sig[0] * z[0]
    th[1] = np.clip(th0[1] + sig[1] * z[1], -np.pi / 2, np.pi / 2)
    th[2] = th0[2] + sig[2] * z[2]
    ci = np.clip(np.cos(th0[3]) + sig[3] * z[3], -1.0 + 1e-9, 1.0 - 1e-9)
    th[3] = np.arccos(ci)
    th[4] = th0[4] + sig[4] * z[4]
    th[5] = th0[5] + sig[5] * z[5]
    th[6] = np.exp(np.log(th0[6]) + sig[6] * z[6])
    return th


# ---------------------------------------------------------------------------
# Workloads (shapes of the paper's benchmarks)
# ---------------------------------------------------------------------------
WORKLOADS = {
    # name: K, M, n_t, fs, snr, n_samples
    "c1_k2_m2_4096hz": dict(K=2, M=2, n_t=410, fs=4096.0, snr=20.0, n=10_000),
    "c2_k3_m21_32khz": dict(K=3, M=21, n_t=6554, fs=32768.0, snr=600.0, n=1_000_000),
    "c4_k3_m9_32khz": dict(K=3, M=9, n_t=6554, fs=32768.0, snr=600.0, n=4096),
    "c5_k5_m21_32khz": dict(K=5, M=21, n_t=13108, fs=32768.0, snr=1000.0, n=10_000_000),
}


def batched_points(n_points: int, seed: int, K: int = 3, fs: float = 32768.0,
                   m_choices=(2, 4, 9, 16, 21), nt_range=(400, 6554), snr_range=(20.0, 1000.0),
                   injection_fn=None, net=None):
    """Uneven batch of intrinsic points sharing one network: M_p ~ U{m_choices},
    n_t,p ~ U{nt_range}, snr_p log-uniform on snr_range."""
    rng = _rng(seed, 99)
    net = net if net is not None else network(K, seed)
    pts = []
    for p in range(n_points):
        M = int(rng.choice(m_choices))
        n_t = int(rng.integers(nt_range[0], nt_range[1] + 1))
        snr = float(snr_range[0] * (snr_range[1] / snr_range[0]) ** rng.uniform())
        sub = int(seed) * 100003 + p
        inj = injection_fn(K, M, sub) if injection_fn is not None else random_injection(K, M, sub)
        pts.append(make_point(K, M, n_t, fs, snr, sub, injection=inj, net=net))
    return pts


# ---------------------------------------------------------------------------
# Composite-index banks (generalised response)
# ---------------------------------------------------------------------------
SIDEREAL_RATE = 7.292115e-5  # rad/s


def make_point_wide(K: int, M: int, n_a: int, n_t: int, fs: float, snr: float, seed: int,
                    response: str = "rotation", omega: float = SIDEREAL_RATE, net=None,
                    noise: bool = True, d_ref: float = 100.0, lm=None, keep_spectra: bool = False):
    """One intrinsic point of the composite-index likelihood: a bank of n_a x M
    templates chi_(a,lm) (index a M + i), its Q [K, n_a, M, n_t], U, V
    [K, n_a M, n_a M] by their inner-product definitions (Eq. (slowrot:QUV)),
    and an injection made of the bank's templates, scaled to network SNR `snr`.

    The bank's templates are generic stand-ins with the shapes of the paper's
    (the elementary modulated templates, or the frequency-weighted modes of the
    finite-arm expansion, are built upstream of the likelihood): chi_(a,lm)(f) =
    h_lm(f) w_a(f), with w_a(f) = 1 for the leading term (a = 2, n = 0, for the
    rotation responses, the term (p = 0, n = 0) with the delay drift; a = 0 for
    the arms) and otherwise a smooth seeded
    complex weight of amplitude 0.2-0.6.  The injection's coefficients are a
    generic rank-one z_(k,(a,lm)) = alpha_(k,a) y_lm with arrival times t_k.
    """
    lm = modes(M) if lm is None else np.asarray(lm, np.int32)
    M = lm.shape[0]
    f, G = mode_spectra(lm, seed)
    rng = _rng(seed, 123)
    lead = 2 if response in ("rotation", "rotation_delay") else 0
    Wt = np.ones((n_a, f.size), np.complex128)
    for a in range(n_a):
        if a == lead:
            continue
        amp = rng.uniform(0.2, 0.6)
        tau = rng.normal(0.0, 3e-4)
        ph0 = rng.uniform(0.0, 2 * np.pi)
        slope = rng.normal(0.0, 1e-3)
        Wt[a] = amp * (1.0 + slope * (np.abs(f) - 150.0) / 150.0) * np.exp(1j * (ph0 + 2 * np.pi * f * tau))
    Gw = (Wt[:, None, :] * G[None, :, :]).reshape(n_a * M, f.size)
    w = noise_weights(K, f, seed)
    net = net if net is not None else network(K, seed)
    yv = rng.normal(size=M) + 1j * rng.normal(size=M)
    yv[:2] *= 4.0
    yv /= np.linalg.norm(yv)
    alpha = rng.uniform(0.2, 1.0, size=(K, n_a)) * np.exp(1j * rng.uniform(0, 2 * np.pi, size=(K, n_a)))
    alpha[:, lead] *= 3.0
    z = (alpha[:, :, None] * yv[None, None, :]).reshape(K, n_a * M)
    tk = rng.uniform(-0.02, 0.02, size=K)
    h = _strain(z, tk, f, Gw)
    rho2 = float(np.sum(w * np.abs(h) ** 2))
    scale = snr / np.sqrt(rho2) if rho2 > 0 else 0.0
    h *= scale
    d = h.copy()
    if noise:
        nrng = _rng(seed, 55)
        pos = f > 0
        nz = np.zeros((K, f.size), np.complex128)
        sig = np.sqrt(1.0 / np.where(w > 0, w, np.inf))
        nz[:, pos] = sig[:, pos] * (nrng.normal(size=(K, pos.sum())) +
                                    1j * nrng.normal(size=(K, pos.sum()))) / np.sqrt(2.0)
        nz[:, f < 0] = np.conj(nz[:, pos][:, ::-1])
        d = d + nz
    U = np.einsum("kf,if,jf->kij", w, np.conj(Gw), Gw)
    V = np.einsum("kf,if,jf->kij", w, Gw[:, ::-1], Gw)
    nfft = int(round(fs))
    if abs(nfft - fs) > 1e-9 or f[-1] >= fs / 2:
        raise ValueError("fs must be an integer rate above twice the band edge")
    A = n_a * M
    X = np.zeros((K, A, nfft), np.complex128)
    bins = np.mod(f.astype(np.int64), nfft)
    X[:, :, bins] = w[:, None, :] * np.conj(Gw)[None, :, :] * d[:, None, :]
    full = np.fft.ifft(X, axis=-1) * nfft
    j0 = n_t // 2
    idx = np.mod(np.arange(n_t) - j0, nfft)
    Q = full[:, :, idx].reshape(K, n_a, M, n_t)
    out = {
        "lm": lm, "t0": -j0 / fs, "dt": 1.0 / fs, "Q": Q, "U": U, "V": V,
        "det_tensor": net["det_tensor"], "det_pos": net["det_pos"], "det_arms": net["det_arms"],
        "gmst": net["gmst"], "d_ref": float(d_ref), "response": response, "n_a": int(n_a),
        "omega": float(omega if response in ("rotation", "rotation_delay") else 0.0), "snr": float(snr),
        "half_dd": 0.5 * float(np.sum(w * np.abs(d) ** 2)),
    }
    if keep_spectra:
        out["spectra"] = {"f": f, "G": Gw, "w": w, "d": d}
    return out


def widen_static(pt, n_a: int, response: str = "rotation"):
    """The static point `pt` as a composite-index point whose every template
    equals its mode (chi_(a,lm) = h_lm for all a): the bank the generalised
    likelihood reduces to when the expansion is trivial (zero rotation rate,
    or the arms' zeroth order alone)."""
    K, M, n_t = pt["Q"].shape
    Q = np.repeat(pt["Q"][:, None, :, :], n_a, axis=1)
    U = np.tile(pt["U"], (1, n_a, n_a))
    V = np.tile(pt["V"], (1, n_a, n_a))
    out = dict(pt)
    out.update({"Q": Q, "U": U, "V": V, "response": response, "n_a": int(n_a), "omega": 0.0})
    if "det_arms" not in out:
        raise ValueError("the point needs det_arms (synth.network provides them)")
    return out
