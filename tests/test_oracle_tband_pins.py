"""Pins of the oracle's band-limited full-window rule over geocentric time
(Eq. (ap:tband)) against what the mathematics fixes, not against the oracle
itself:

* the Whittaker-Shannon series reproduces a band-limited signal from its
  samples: a Gaussian-windowed cosine well inside the window, with its band
  below the nodes' Nyquist rate, comes back at every fine point to within
  its aliasing and truncation error (about 1e-9 here);
* with one fine interval per node interval (M = 1) the sinc weights are the
  identity and the rule is the trapezoid rule on the nodes;
* the rule converges, as M grows, to adaptive quadrature of the exponential
  of the same closed-form exponent over the window (the weights and the
  1/T normalisation);
* on the likelihood, M = 1 gives the trapezoid rule over the oracle's own
  lnL at the node times (so the exponent is x K - R x^2 / 2 with K the data
  term and R the model norm), and the time row of theta is not read.
"""
import numpy as np
from scipy import integrate

from paper_2609_37393_amd import synth


def _signal(t, t0=20.3, w=3.0, nu=0.15):
    """A Gaussian-windowed cosine in units of the node spacing: its spectrum
    is a Gaussian of width 1/(2 pi w) around nu, far below 1/2 at the nodes'
    Nyquist rate."""
    return np.exp(-0.5 * ((t - t0) / w) ** 2) * np.cos(2 * np.pi * nu * t + 0.4)


def test_reconstruction_of_a_band_limited_signal(oracle_mod):
    n = 41
    y = _signal(np.arange(n, dtype=float))
    for M in (1, 3, 8, 16):
        got = oracle_mod.band_values(y, M)
        want = _signal(np.arange((n - 1) * M + 1) / M)
        assert got.shape == want.shape
        assert np.max(np.abs(got - want)) <= 1e-8, (M, np.max(np.abs(got - want)))
    # several columns at once, each its own signal
    Y = np.stack([_signal(np.arange(n, dtype=float), t0=c) for c in (18.5, 20.0, 21.5)], axis=1)
    got = oracle_mod.band_values(Y, 4)
    tf = np.arange((n - 1) * 4 + 1) / 4
    for c, t0 in enumerate((18.5, 20.0, 21.5)):
        assert np.max(np.abs(got[:, c] - _signal(tf, t0=t0))) <= 1e-8


def test_one_fine_interval_is_the_trapezoid_rule(oracle_mod):
    rng = np.random.default_rng(1)
    n, N = 17, 6
    y = rng.normal(size=(n, N)) * 5
    base = rng.normal(size=N)
    got = oracle_mod.band_rule(y, base, 1)
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    want = np.log(np.sum(w[:, None] * np.exp(y + base[None, :]), axis=0) / (n - 1))
    assert np.all(np.abs(got - want) <= 1e-12 * (1 + np.abs(want)))
    # NaN in a column poisons that column only
    y[3, 2] = np.nan
    got = oracle_mod.band_rule(y, base, 1)
    assert np.isnan(got[2]) and np.all(np.isfinite(np.delete(got, 2)))


def test_rule_converges_to_quadrature(oracle_mod):
    n, A, base = 41, 12.0, -3.0
    y = A * _signal(np.arange(n, dtype=float))[:, None]
    T = n - 1.0
    val, _ = integrate.quad(lambda t: np.exp(A * _signal(t) + base), 0.0, T, limit=400, epsabs=0, epsrel=1e-13)
    want = np.log(val / T)
    errs = []
    for M in (1, 2, 4, 8, 16):
        got = oracle_mod.band_rule(y, np.array([base]), M)[0]
        errs.append(abs(got - want))
    assert errs[-1] <= 1e-8, errs
    assert errs[0] > 1e-3 and errs[2] < errs[0] * 1e-2, errs


def test_likelihood_at_one_fine_interval_and_time_row(oracle_mod):
    pt = synth.make_point(3, 9, 2000, 16384.0, 40.0, 12)
    th = synth.prior_samples(30, 13)
    th[5] = 0.0
    t_start, h, n_t = -2e-3, 1.0 / 4096.0, 17
    got = oracle_mod.lnL_tband(pt, th, t_start, h, n_t, 1)
    tk = t_start + h * np.arange(n_t)
    big = np.repeat(th, n_t, axis=1)
    big[5] = np.tile(tk, th.shape[1])
    l = oracle_mod.lnL(pt, big).reshape(th.shape[1], n_t)
    lw = np.zeros(n_t)
    lw[0] = lw[-1] = np.log(0.5)
    m = np.max(l, axis=1)
    want = m + np.log(np.sum(np.exp(l + lw[None, :] - m[:, None]), axis=1)) - np.log(n_t - 1.0)
    S = np.max(np.abs(l), axis=1) + 1.0
    assert np.all(np.abs(got - want) <= 1e-11 * S), np.max(np.abs(got - want) / S)
    th2 = th.copy()
    th2[5] = 123.0
    assert np.array_equal(oracle_mod.lnL_tband(pt, th2, t_start, h, n_t, 4),
                          oracle_mod.lnL_tband(pt, th, t_start, h, n_t, 4))
