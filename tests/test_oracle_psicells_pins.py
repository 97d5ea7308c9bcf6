"""Pins of the oracle's polarisation marginal by stationary-point cells
(Eq. (ap:psicells)) against what the mathematics fixes:

* the stationary points are zeros of q'(u), and they are all of them: their
  count equals the sign changes of q' on a fine grid (for coefficient sets
  whose extrema are well separated), two for a single harmonic;
* the integral over the cells matches adaptive quadrature of e^{q} over the
  circle, from weak to strong amplitudes and for one, two or three peaks;
* on the likelihood, the method agrees with the periodic trapezoid rule on
  many points (both converge to the same integral).
"""
import numpy as np
from scipy import integrate

from paper_2609_37393_amd import synth


def _q(a, c1, c2, u):
    e = np.exp(1j * u)
    return a + (c1 * e).real + (c2 * e * e).real


def _dq(c1, c2, u):
    e = np.exp(1j * u)
    return -(c1 * e).imag - 2.0 * (c2 * e * e).imag


def _cases():
    rng = np.random.default_rng(1)
    out = [(0.3, 2.0 + 1.0j, 0.0 + 0.0j),            # one harmonic: a max and a min
           (-1.0, 0.1 + 0.0j, 3.0 - 2.0j),           # two peaks
           (0.0, 1e-12 + 0j, 1e-12 + 0j)]            # nearly constant
    for amp in (0.5, 5.0, 50.0, 500.0, 5e4):
        for _ in range(4):
            c1 = amp * (rng.normal() + 1j * rng.normal())
            c2 = amp * rng.uniform(0, 0.8) * (rng.normal() + 1j * rng.normal())
            out.append((rng.normal() * amp, c1, c2))
    return out


def test_stationary_points_are_all_the_zeros(oracle_mod):
    u = np.linspace(0, 2 * np.pi, 200001)
    for a, c1, c2 in _cases():
        st = oracle_mod.psi_stationary(a, c1, c2)
        scale = abs(c1) + 2 * abs(c2)
        if scale < 1e-9:
            continue
        assert np.all(np.abs(_dq(c1, c2, st)) <= 1e-9 * scale)
        d = _dq(c1, c2, u)
        changes = np.count_nonzero(np.sign(d[1:]) != np.sign(d[:-1]))
        # well separated extrema: no two closer than the grid
        if st.size >= 2 and np.min(np.diff(np.r_[st, st[0] + 2 * np.pi])) > 1e-3:
            assert st.size == changes, (a, c1, c2, st, changes)
    st = oracle_mod.psi_stationary(0.0, 1.0 + 0.0j, 0.0j)
    assert np.allclose(np.sort(st), [0.0, np.pi], atol=1e-12)  # q = a + cos u


def test_cells_match_adaptive_quadrature(oracle_mod):
    for a, c1, c2 in _cases():
        got = oracle_mod.psi_cells_integral(a, c1, c2)
        # quadrature about the maximum, split at the grid's best point
        u = np.linspace(0, 2 * np.pi, 4097)
        qs = _q(a, c1, c2, u)
        m = qs.max()
        ub = u[np.argmax(qs)]
        pts = sorted(set([0.0, 2 * np.pi, ub] + list(oracle_mod.psi_stationary(a, c1, c2))))
        val = 0.0
        for lo, hi in zip(pts[:-1], pts[1:]):
            if hi > lo:
                val += integrate.quad(lambda t: np.exp(_q(a, c1, c2, t) - m), lo, hi, epsabs=0, epsrel=1e-13,
                                      limit=400)[0]
        want = m + np.log(val / (2 * np.pi))
        assert abs(got - want) <= 1e-9 * max(1.0, abs(want)), (a, c1, c2, got, want)


def test_likelihood_cells_equal_a_fine_trapezoid(oracle_mod):
    pt = synth.make_point(3, 9, 2000, 16384.0, 80.0, 21)
    th = synth.prior_samples(30, 22)
    got = oracle_mod.lnL_pmarg(pt, th, "cells")
    want = oracle_mod.lnL_pmarg(pt, th, "trapezoid", 2048)
    assert np.all(np.abs(got - want) <= 1e-9 * np.maximum(1.0, np.abs(want)))
