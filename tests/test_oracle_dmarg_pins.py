"""Pins of the oracle's distance marginal (Sec. "Distance: locating a moving
peak", Eqs. (ap:dexp), (ap:dpeak), (ap:dgh)) against what the mathematics
fixes, not against the oracle itself:

* the terms: lnL(x) = K x - R x^2 / 2 reproduces the oracle's own lnL at every
  distance (the quadratic of Eq. (ap:dexp));
* closed form: with a prior flat in x = D_ref / D (p(D) proportional to D^-2)
  the Gaussian integral is exact, int dx e^{K x - R x^2/2} / (x_max - x_min)
  = sqrt(2 pi / R) e^{K^2 / 2R} / (x_max - x_min), and a Gauss-Hermite rule of
  any order reproduces it;
* the uniform-in-volume prior (p(D) proportional to D^2, p_x proportional to
  x^-4): the rule against adaptive quadrature in D of p(D) e^{lnL(D)} with
  lnL(D) from the oracle's lnL at each D, where the peak lies well inside
  the prior (the rule's error there is far below the bar);
* convergence in the node count, independence of the distance row, and the
  rule's behaviour for a peak far outside the prior (every node outside: -inf).
"""
import numpy as np
import pytest
from scipy import integrate

from paper_2609_37393_amd import synth


def _peaked_samples(pt, n, seed, oracle_mod, widths=9.0):
    """Draws whose peak in x lies more than `widths` sigma_x above x = 0 (so
    that every node of the rules below lies at x > 0)."""
    th, _ = synth.weighted_samples(20 * n, seed)
    K, R = oracle_mod.lnL_terms(pt, th)
    good = np.where((R > 0) & (K > widths * np.sqrt(np.maximum(R, 1e-300))))[0][:n]
    assert good.size >= n // 2
    return th[:, good]


def test_terms_reproduce_lnL(oracle_mod):
    pt = synth.make_point(3, 9, 3000, 32768.0, 200.0, 11)
    th = synth.prior_samples(300, 12)
    K, R = oracle_mod.lnL_terms(pt, th)
    for D in (15.0, 100.0, 440.0, 1000.0):
        t = th.copy()
        t[6] = D
        x = pt["d_ref"] / D
        want = oracle_mod.lnL(pt, t)
        got = K * x - 0.5 * R * x * x
        assert np.all(np.abs(got - want) <= 1e-12 * (np.abs(K * x) + np.abs(R * x * x) + 1.0))
    assert np.all(R >= 0.0)


@pytest.mark.parametrize("n_nodes", [1, 3, 20])
def test_flat_in_x_prior_is_the_gaussian_integral(oracle_mod, n_nodes):
    pt = synth.make_point(3, 4, 3000, 32768.0, 300.0, 13)
    th = _peaked_samples(pt, 40, 14, oracle_mod)
    d_min, d_max = 1e-3, 1e9  # every node inside for these peaks
    got = oracle_mod.lnL_dmarg(pt, th, d_min, d_max, n_nodes, power=-2.0)
    K, R = oracle_mod.lnL_terms(pt, th)
    xr = pt["d_ref"] / d_min - pt["d_ref"] / d_max
    want = 0.5 * K * K / R + 0.5 * np.log(2.0 * np.pi / R) - np.log(xr)
    assert np.all(np.abs(got - want) <= 1e-12 * (np.abs(want) + 1.0)), np.abs(got - want).max()


@pytest.mark.parametrize("snr", [60.0, 600.0])
def test_volume_prior_against_quadrature_in_distance(oracle_mod, snr):
    pt = synth.make_point(3, 9, 6554, 32768.0, snr, 15)
    th = _peaked_samples(pt, 8, 16, oracle_mod)
    d_min, d_max = 1.0, 1000.0
    got = oracle_mod.lnL_dmarg(pt, th, d_min, d_max, 24)
    K, R = oracle_mod.lnL_terms(pt, th)
    norm = (d_max ** 3 - d_min ** 3) / 3.0
    checked = 0
    for i in range(th.shape[1]):
        Dpk = pt["d_ref"] * R[i] / K[i]
        if not (2 * d_min < Dpk < 0.5 * d_max):
            continue
        checked += 1
        peak = 0.5 * K[i] ** 2 / R[i]

        def f(D):
            t = np.repeat(th[:, i:i + 1], 1, axis=1).copy()
            t[6, 0] = D
            return D * D / norm * np.exp(oracle_mod.lnL(pt, t)[0] - peak)

        sD = Dpk / (K[i] / np.sqrt(R[i]))  # the width in D at the peak
        lo, hi = max(d_min, Dpk - 40 * sD), min(d_max, Dpk + 40 * sD)
        val, err = integrate.quad(f, lo, hi, points=[Dpk], epsabs=0.0, epsrel=1e-13, limit=400)
        want = peak + np.log(val)
        assert abs(got[i] - want) <= 1e-9 * (abs(peak) + 1.0), (snr, i, got[i], want)
    assert checked >= 3


def test_node_count_convergence_and_distance_row(oracle_mod):
    pt = synth.make_point(3, 9, 3000, 32768.0, 150.0, 17)
    th = _peaked_samples(pt, 30, 18, oracle_mod)
    a = oracle_mod.lnL_dmarg(pt, th, 10.0, 1000.0, 20)
    b = oracle_mod.lnL_dmarg(pt, th, 10.0, 1000.0, 40)
    fin = np.isfinite(a)
    assert fin.sum() >= 10
    assert np.all(np.abs(a[fin] - b[fin]) <= 1e-9 * (np.abs(b[fin]) + 1.0))
    t2 = th.copy()
    t2[6] = np.random.default_rng(3).uniform(10, 1000, th.shape[1])
    assert np.array_equal(oracle_mod.lnL_dmarg(pt, t2, 10.0, 1000.0, 20), a)


def test_peak_far_outside_the_prior(oracle_mod):
    pt = synth.make_point(3, 4, 3000, 32768.0, 600.0, 19)
    th = _peaked_samples(pt, 10, 20, oracle_mod)
    K, R = oracle_mod.lnL_terms(pt, th)
    Dpk = pt["d_ref"] * R / K
    # a prior box far beyond every peak (widths are ~1/SNR of the distance)
    d_min = 50.0 * Dpk.max()
    got = oracle_mod.lnL_dmarg(pt, th, d_min, 2 * d_min, 20)
    assert np.all(got == -np.inf)
