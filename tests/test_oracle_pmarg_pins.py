"""Pins of the oracle's marginal over polarisation (Sec. "Angles: finite
harmonic content", Eqs. (ap:psiexp), (ap:psilaplace)) against what the paper
and the mathematics fix, not against the oracle itself:

* the finite harmonic content: the five-point coefficients (a, c1, c2)
  reproduce the oracle's lnL at any polarisation (the series ends at 4 psi);
* the trapezoid rule converges to adaptive quadrature of e^{lnL(psi)} over
  [0, pi) (the oracle's own lnL at each psi);
* a model norm independent of psi (V = 0) leaves a single harmonic,
  q = a + kappa cos(u - u0), whose integral is the Bessel function
  e^{a} I_0(kappa); Laplace's method then errs by ~1/(8 kappa), so the
  product of its error and A = kappa tends to 1/8 (the O(1/A) law the paper
  states and observes);
* the integral covers the whole period: the psi row only moves the points.
"""
import numpy as np
import pytest
from scipy import integrate, special

from paper_2609_37393_amd import synth


def _near(pt, oracle_mod, n, seed):
    th, _ = synth.weighted_samples(20 * n, seed)
    l = oracle_mod.lnL(pt, th)
    return th[:, np.argsort(l)[-n:]]


def test_five_point_coefficients_reproduce_lnL(oracle_mod):
    pt = synth.make_point(3, 9, 3000, 32768.0, 100.0, 21)
    th = np.concatenate([synth.prior_samples(20, 22), _near(pt, oracle_mod, 10, 23)], axis=1)
    a, c1, c2 = oracle_mod.psi_coefficients(pt, th)
    u = np.random.default_rng(1).uniform(0, 2 * np.pi, 17)
    l = oracle_mod.lnL_psi_grid(pt, th, u)
    q = a[:, None] + (c1[:, None] * np.exp(1j * u)).real + (c2[:, None] * np.exp(2j * u)).real
    scale = np.abs(a) + np.abs(c1) + np.abs(c2) + 1.0
    assert np.all(np.abs(q - l) <= 1e-12 * scale[:, None]), (np.abs(q - l) / scale[:, None]).max()


def test_trapezoid_converges_to_quadrature(oracle_mod):
    pt = synth.make_point(3, 9, 3000, 32768.0, 40.0, 24)
    th = _near(pt, oracle_mod, 4, 25)
    want = []
    for i in range(th.shape[1]):
        peak = oracle_mod.lnL_psi_grid(pt, th[:, i:i + 1], np.linspace(0, 2 * np.pi, 721)).max()

        def f(psi):
            t = th[:, i:i + 1].copy()
            t[2, 0] = psi
            return np.exp(oracle_mod.lnL(pt, t)[0] - peak)

        v, _ = integrate.quad(f, 0.0, np.pi, epsabs=0.0, epsrel=1e-12, limit=400)
        want.append(peak + np.log(v / np.pi))
    want = np.array(want)
    errs = [np.abs(oracle_mod.lnL_pmarg(pt, th, "trapezoid", n) - want).max() for n in (8, 32, 128)]
    assert errs[-1] <= 1e-9, errs
    assert errs[0] >= errs[1] >= errs[2], errs


def test_single_harmonic_bessel_and_laplace_law(oracle_mod):
    pt = dict(synth.make_point(2, 4, 3000, 32768.0, 150.0, 26))
    pt["V"] = np.zeros_like(pt["V"])  # the model norm no longer depends on psi
    th = _near(pt, oracle_mod, 6, 27)
    a, c1, c2 = oracle_mod.psi_coefficients(pt, th)
    assert np.all(np.abs(c2) <= 1e-12 * (np.abs(a) + np.abs(c1)))
    kappa = np.abs(c1)
    exact = a + kappa + np.log(special.i0e(kappa))
    # the trapezoid rule on the circle errs by ~I_n(kappa) / I_0(kappa) ~ e^{-n^2 / 2 kappa}
    trap = oracle_mod.lnL_pmarg(pt, th, "trapezoid", 4096)
    assert np.all(np.abs(trap - exact) <= 1e-10 * (np.abs(exact) + 1.0))
    lap = oracle_mod.lnL_pmarg(pt, th, "laplace")
    prod = (exact - lap) * kappa
    big = kappa > 200.0
    assert big.sum() >= 2
    assert np.all(np.abs(prod[big] - 0.125) <= 0.01), prod


def test_psi_row_moves_only_the_points(oracle_mod):
    pt = synth.make_point(3, 4, 3000, 32768.0, 60.0, 28)
    th = _near(pt, oracle_mod, 8, 29)
    t2 = th.copy()
    t2[2] += np.random.default_rng(2).uniform(0, np.pi, th.shape[1])
    for method, n in (("trapezoid", 256), ("laplace", 0)):
        a = oracle_mod.lnL_pmarg(pt, th, method, n)
        b = oracle_mod.lnL_pmarg(pt, t2, method, n)
        assert np.all(np.abs(a - b) <= 1e-9 * (np.abs(a) + 1.0)), method
