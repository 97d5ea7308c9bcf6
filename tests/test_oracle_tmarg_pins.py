"""Pins of the oracle's marginal over geocentric time (Eq. (ap:tfixed), the
fixed-spacing rule with composite Simpson weights) against what the
mathematics fixes, not against the oracle itself:

* Simpson's rule integrates cubics exactly: the weights reproduce the
  integrals of 1, t, t^2, t^3 over the window;
* a likelihood constant in time (a point whose correlation tables vanish:
  lnL = -x^2 quad / 4 at every t) gives that constant exactly (the rule's
  weights sum to the window);
* against Gauss-Legendre quadrature of e^{lnL(t)} on every piece between the
  times where an arrival time crosses a table node (lnL(t) is smooth there;
  the four-point read is C0 across), with lnL(t) the oracle's own likelihood
  at each t: the rule converges as the spacing shrinks, to within 1e-6 at
  the finest;
* the time row of theta is not read.
"""
import numpy as np
import pytest

from paper_2609_37393_amd import synth


def test_simpson_weights_integrate_cubics(oracle_mod):
    for n_t in (3, 5, 11, 101):
        w = oracle_mod.simpson_weights(n_t)
        h = 0.37
        t = -1.2 + h * np.arange(n_t)
        a, b = t[0], t[-1]
        for p in range(4):
            got = h * np.sum(w * t ** p)
            want = (b ** (p + 1) - a ** (p + 1)) / (p + 1)
            assert abs(got - want) <= 1e-13 * max(1.0, abs(want)), (n_t, p)


def test_constant_likelihood(oracle_mod):
    pt = synth.make_point(3, 4, 500, 4096.0, 50.0, 3)
    pt = dict(pt)
    pt["Q"] = np.zeros_like(pt["Q"])
    th = synth.prior_samples(20, 4)
    want = oracle_mod.lnL(pt, th)  # no data term: the same at every time
    got = oracle_mod.lnL_tmarg(pt, th, -0.01, 1e-4, 201)
    assert np.all(np.abs(got - want) <= 1e-12 * (np.abs(want) + 1.0))


def _kink_quadrature(oracle_mod, pt, th1, t_start, T):
    """ln[(1/T) int e^{lnL(t)} dt] over the window by 10-point Gauss-Legendre
    on every piece between the times where a detector's arrival time crosses
    a table node (the four-point read is smooth between them, C0 across)."""
    ra, dec = th1[0], th1[1]
    g = pt["gmst"] - ra
    N = np.array([np.cos(dec) * np.cos(g), -np.cos(dec) * np.sin(g), np.sin(dec)])
    brk = [t_start, t_start + T]
    for r in pt["det_pos"]:
        d = r @ N  # t_k = t - d
        j = np.arange(np.floor((t_start - d - pt["t0"]) / pt["dt"]), np.ceil((t_start + T - d - pt["t0"]) / pt["dt"]) + 1)
        tb = pt["t0"] + j * pt["dt"] + d
        brk.extend(tb[(tb > t_start) & (tb < t_start + T)])
    brk = np.unique(np.array(brk))
    x, w = np.polynomial.legendre.leggauss(10)
    a, b = brk[:-1, None], brk[1:, None]
    tt = (0.5 * (b - a) * x[None, :] + 0.5 * (b + a)).ravel()
    ww = (0.5 * (b - a) * w[None, :]).ravel()
    big = np.repeat(th1[:, None], tt.size, axis=1)
    big[5] = tt
    l = oracle_mod.lnL(pt, big)
    m = l.max()
    return m + np.log(np.sum(ww * np.exp(l - m)) / T)


def test_against_piecewise_quadrature(oracle_mod):
    """At SNR 30 the peak in time is ~0.3 ms wide; a 4 ms window around the
    injection holds it whole.  The rule converges to the piecewise
    Gauss-Legendre integral of the oracle's own lnL(t)."""
    pt = synth.make_point(3, 9, 3000, 32768.0, 30.0, 5)
    th, _ = synth.weighted_samples(200, 6)
    pick = np.argsort(oracle_mod.lnL(pt, th))[-3:]  # three draws near the peak
    th = th[:, pick]
    t_start, T = -0.002, 0.004
    want = np.array([_kink_quadrature(oracle_mod, pt, th[:, i], t_start, T) for i in range(th.shape[1])])
    errs = []
    for n_t in (41, 161, 641):
        got = oracle_mod.lnL_tmarg(pt, th, t_start, T / (n_t - 1), n_t)
        errs.append(np.abs(got - want).max())
    assert errs[-1] <= 1e-6, errs
    assert errs[0] > errs[1] > errs[2], errs


def test_time_row_not_read(oracle_mod):
    pt = synth.make_point(2, 4, 800, 4096.0, 40.0, 7)
    th = synth.prior_samples(30, 8)
    a = oracle_mod.lnL_tmarg(pt, th, -0.02, 1e-3, 41)
    th2 = th.copy()
    th2[5] = np.random.default_rng(1).uniform(-1, 1, th.shape[1])
    assert np.array_equal(oracle_mod.lnL_tmarg(pt, th2, -0.02, 1e-3, 41), a)
