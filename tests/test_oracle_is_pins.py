"""Pins of the oracle's importance-sampling normalisation (Eq.
(sampler-menu:is)) with the defensive Gaussian-mixture proposal of Sec. "Mode
coverage, adaptive clouds, and evidence", against what the mathematics fixes:

* the prior density is normalised on its box, with the shapes cos(dec) and
  D^3 in ln D (a product of one-dimensional integrals by quadrature), and the
  prior draws follow its distribution functions (Kolmogorov-Smirnov);
* a wrapped component integrates to one over the periodic torus (periodic
  trapezoid rule over (ra, psi) of a correlated component, times the
  independent factors) and
  equals the plain multivariate normal density where no image matters;
* component draws have the component's mean and covariance (a transposed
  Cholesky factor fails on a correlated covariance) and wrap into the box
  with the mass the Gaussian puts across the boundary;
* the moments are the closed form for two weighted points and do not change
  when every log weight moves by a constant;
* the estimator is unbiased: with L = 1 the mean weight is 1, and for a
  likelihood bump of known integral the estimate lies within four standard
  errors.  Weighting each draw by its own component density instead of the
  full mixture is biased, and that planted mistake fails the pin;
* for a likelihood marginalised over some rows (the `rows` mask): the
  restricted component is the full one integrated over a left-out row (by
  quadrature), the restricted prior is normalised, all seven rows are the
  default bit for bit, and the estimate of a bump over the sampled rows is
  unbiased while the left-out rows take prior draws.
"""
import numpy as np
import pytest
from scipy import integrate, stats

BOX = (-0.01, 0.01, 10.0, 1000.0)


def _interior():
    return np.array([1.0, 0.3, 1.2, 0.2, 2.5, 0.001, np.log(300.0)])


def test_prior_is_normalised(oracle_mod):
    c0 = _interior()
    lp0 = oracle_mod.is_log_prior(c0[:, None], *BOX)[0]
    ranges = [(0, 2 * np.pi), (-np.pi / 2, np.pi / 2), (0, np.pi), (-1, 1), (0, 2 * np.pi), (BOX[0], BOX[1]),
              (np.log(BOX[2]), np.log(BOX[3]))]
    total = 0.0
    for j, (lo, hi) in enumerate(ranges):
        def f(s, j=j):
            c = c0.copy()
            c[j] = s
            return np.exp(oracle_mod.is_log_prior(c[:, None], *BOX)[0] - lp0)
        val, _ = integrate.quad(f, lo, hi, limit=200, epsabs=0, epsrel=1e-12)
        total += np.log(val)
        if j == 1:
            assert abs(f(0.7) - np.cos(0.7) / np.cos(c0[1])) < 1e-14
        if j == 6:
            assert abs(f(np.log(500.0)) - (500.0 / 300.0) ** 3) < 1e-12
    # p separable: int p = prod_j int p(.., s_j, ..) ds_j / p(c0)^6
    assert abs(total + lp0) < 1e-10, total + lp0
    out = c0.copy()
    out[3] = 1.0 + 1e-12
    assert np.isneginf(oracle_mod.is_log_prior(out[:, None], *BOX)[0])


def test_prior_draws_follow_the_prior(oracle_mod):
    rng = np.random.default_rng(1)
    n = 4000
    c, comp = oracle_mod.mixture_draw(1.0, [], [], [], 1.0, *BOX, rng.normal(size=(7, n)), rng.uniform(size=(7, n)),
                                      rng.uniform(size=n))
    assert np.all(comp == -1)
    t_min, t_max, d_min, d_max = BOX
    cdfs = [lambda x: x / (2 * np.pi), lambda x: (1 + np.sin(x)) / 2, lambda x: x / np.pi, lambda x: (x + 1) / 2,
            lambda x: x / (2 * np.pi), lambda x: (x - t_min) / (t_max - t_min),
            lambda x: (np.exp(3 * x) - d_min ** 3) / (d_max ** 3 - d_min ** 3)]
    for j in range(7):
        assert stats.kstest(c[j], cdfs[j]).pvalue > 1e-3, j
    assert np.all(np.isfinite(oracle_mod.is_log_prior(c, *BOX)))


def _corr_cov(broad=False):
    s = np.array([2.5, 0.05, 1.2, 0.1, 2.5, 0.002, 0.1]) if broad else np.array([0.3, 0.05, 0.2, 0.1, 0.4, 0.002, 0.1])
    R = np.eye(7)
    R[0, 2] = R[2, 0] = 0.6
    return np.outer(s, s) * R


@pytest.mark.parametrize("broad", [False, True], ids=["narrow", "broad"])
def test_wrapped_component_is_normalised(oracle_mod, broad):
    """Broad: the periodic widths are 0.4 of their periods, so images beyond
    the nearest one carry a few per cent of the mass."""
    cov = _corr_cov(broad)
    mu = np.array([0.1, 0.2, 3.0, 0.0, 6.1, 0.0, 5.0])  # ra, psi and phiref near their period's edge
    rest = np.array([0.25, -0.05, 0.0005, 5.1])  # dec, cos incl, tref, ln D
    phi = 0.3

    # the periodic trapezoid rule on the torus: its error for a smooth periodic
    # integrand is the aliasing of the Fourier coefficients beyond the grid,
    # here below 1e-15 (wrapped widths 0.3 in 2 pi and 0.2 in pi, 96 x 48 nodes)
    ra, psi = np.meshgrid(np.arange(96) * (2 * np.pi / 96), np.arange(48) * (np.pi / 48), indexing="ij")
    c = np.empty((7, ra.size))
    c[0], c[2] = ra.ravel(), psi.ravel()
    c[1], c[3], c[4], c[5], c[6] = rest[0], rest[1], phi, rest[2], rest[3]
    val = np.sum(np.exp(oracle_mod.wrapped_normal_logpdf(c, mu, cov))) * (2 * np.pi / 96) * (np.pi / 48)
    # the (ra, psi) block is independent of the others: the torus integral
    # leaves the product of the other rows' densities
    want = 1.0
    for j, x in zip((1, 3, 5, 6), rest):
        want *= stats.norm.pdf(x, mu[j], np.sqrt(cov[j, j]))
    s4 = np.sqrt(cov[4, 4])
    want *= sum(stats.norm.pdf(phi + 2 * np.pi * k, mu[4], s4) for k in range(-20, 21))
    assert abs(val / want - 1) < 1e-12, val / want


def test_narrow_component_is_the_normal_density(oracle_mod):
    cov = _corr_cov() * 0.01
    mu = np.array([3.0, 0.2, 1.5, 0.0, 3.0, 0.0, 5.0])
    x = np.random.default_rng(2).multivariate_normal(mu, cov, size=50).T
    got = oracle_mod.wrapped_normal_logpdf(x, mu, cov)
    want = stats.multivariate_normal(mu, cov).logpdf(x.T)
    assert np.allclose(got, want, rtol=0, atol=1e-11)


def test_component_draws_have_its_moments(oracle_mod):
    rng = np.random.default_rng(3)
    cov = _corr_cov()
    mu = np.array([3.0, 0.2, 1.5, 0.1, 3.0, 0.0, 5.0])
    n = 20000
    c, comp = oracle_mod.mixture_draw(0.0, [1.0], [mu], [cov], 2.0, *BOX, rng.normal(size=(7, n)),
                                      rng.uniform(size=(7, n)), rng.uniform(size=n))
    assert np.all(comp == 0)
    C = 2.0 * cov
    m = c.mean(axis=1)
    se = np.sqrt(np.diag(C) / n)
    assert np.all(np.abs(m - mu) < 5 * se)
    S = np.cov(c)
    # the (ra, psi) covariance pins the orientation of the factor
    for j, k in ((0, 2), (0, 0), (2, 2), (6, 6)):
        se_jk = np.sqrt((C[j, j] * C[k, k] + C[j, k] ** 2) / n)
        assert abs(S[j, k] - C[j, k]) < 5 * se_jk, (j, k, S[j, k], C[j, k])


def test_draws_wrap_across_the_boundary(oracle_mod):
    rng = np.random.default_rng(4)
    cov = np.diag([0.2, 0.01, 0.1, 0.01, 0.1, 1e-6, 0.01]) ** 2
    mu = np.array([0.1, 0.0, 1.0, 0.0, 3.0, 0.0, 5.0])
    n = 20000
    c, _ = oracle_mod.mixture_draw(0.0, [1.0], [mu], [cov], 1.0, *BOX, rng.normal(size=(7, n)),
                                   rng.uniform(size=(7, n)), rng.uniform(size=n))
    assert np.all((c[0] >= 0) & (c[0] < 2 * np.pi))
    frac = np.mean(c[0] > np.pi)
    want = stats.norm.cdf(-0.1 / 0.2)
    assert abs(frac - want) < 5 * np.sqrt(want * (1 - want) / n)


def test_moments_closed_form(oracle_mod):
    x1 = np.arange(7.0)
    x2 = x1[::-1] * 0.5
    lw = np.log([0.3, 0.9])
    mu, C = oracle_mod.cloud_moments(np.stack([x1, x2], axis=1), lw)
    w1, w2 = 0.25, 0.75
    assert np.allclose(mu, w1 * x1 + w2 * x2, rtol=1e-15, atol=1e-15)
    assert np.allclose(C, w1 * w2 * np.outer(x1 - x2, x1 - x2), rtol=1e-14, atol=1e-14)
    rng = np.random.default_rng(5)
    c = rng.normal(size=(7, 100))
    lw = rng.normal(size=100)
    m1, C1 = oracle_mod.cloud_moments(c, lw)
    m2, C2 = oracle_mod.cloud_moments(c, lw + 123.0)
    assert np.allclose(m1, m2, rtol=1e-13, atol=1e-14) and np.allclose(C1, C2, rtol=1e-12, atol=1e-14)
    # a sample of zero weight is not read
    c2 = np.concatenate([c, np.full((7, 1), np.nan)], axis=1)
    m3, C3 = oracle_mod.cloud_moments(c2, np.r_[lw, -np.inf])
    assert np.array_equal(m3, m1) and np.array_equal(C3, C1)


def _bump(c, ra0, ci0, s_r, s_c):
    return -0.5 * ((c[0] - ra0) / s_r) ** 2 - 0.5 * ((c[3] - ci0) / s_c) ** 2


def _mixture():
    cov = np.diag([0.15, 0.3, 0.6, 0.15, 1.0, 0.006, 0.8]) ** 2
    means = [np.array([1.0, 0.0, 1.5, 0.2, 3.0, 0.0, 5.5]), np.array([1.2, 0.1, 1.5, 0.3, 3.0, 0.0, 5.5]),
             np.array([4.0, -0.5, 1.0, -0.5, 1.0, 0.0, 6.0])]
    return [0.5, 0.3, 0.2], means, [cov, cov, cov]


@pytest.mark.parametrize("alpha", [0.0, 0.2])
def test_is_estimate_is_unbiased(oracle_mod, alpha):
    rng = np.random.default_rng(6)
    a, means, covs = _mixture()
    n = 24000
    th, lnw, comp = oracle_mod.mixture_is(alpha, a, means, covs, 1.5, *BOX, rng.normal(size=(7, n)),
                                          rng.uniform(size=(7, n)), rng.uniform(size=n))
    w = np.exp(lnw)
    if alpha > 0:
        # L = 1: E_q[p / q] = 1 (q > 0 on the whole box)
        assert abs(w.mean() - 1.0) < 4 * w.std() / np.sqrt(n)
    # a bump of known prior mean: Z = E_p[L] = (sqrt(2 pi) s_r / (2 pi)) (sqrt(2 pi) s_c / 2)
    s_r, s_c = 0.1, 0.08
    c = th.copy()
    c[3] = np.cos(th[3])
    lnL = _bump(c, 1.1, 0.25, s_r, s_c)
    Z = np.sqrt(2 * np.pi) * s_r / (2 * np.pi) * np.sqrt(2 * np.pi) * s_c / 2
    terms = np.exp(lnL + lnw)
    assert abs(terms.mean() - Z) < 4 * terms.std() / np.sqrt(n), (terms.mean(), Z)
    z, _ = oracle_mod.lnZ(lnL, lnw)
    assert abs(z - np.log(terms.mean())) < 1e-12
    # the planted mistake: each draw weighted by its own component alone
    bad = lnw.copy()
    for m in range(3):
        sel = comp == m
        lq = np.log((1 - alpha) * a[m]) + oracle_mod.wrapped_normal_logpdf(c[:, sel], means[m], 1.5 * covs[m])
        bad[sel] = oracle_mod.is_log_prior(c[:, sel], *BOX) - lq
    tb = np.exp(lnL + bad)
    assert abs(tb.mean() - Z) > 4 * tb.std() / np.sqrt(n)


def test_restricted_component_is_the_marginal(oracle_mod):
    """Leaving out ln D (row 6) gives the full wrapped density integrated over
    ln D: the Gaussian's marginal is its sub-covariance, images included."""
    cov = _corr_cov(broad=True)
    cov[6, 0] = cov[0, 6] = 0.5 * np.sqrt(cov[0, 0] * cov[6, 6])  # coupled to a periodic row
    mu = np.array([0.1, 0.2, 3.0, 0.0, 6.1, 0.0, 5.0])
    c = np.array([2.5, 0.25, 0.4, -0.05, 0.3, 0.0005, 0.0])
    got = oracle_mod.wrapped_normal_logpdf(c[:, None], mu, cov, rows=0b0111111)[0]

    def f(x):
        cc = c.copy()
        cc[6] = x
        return np.exp(oracle_mod.wrapped_normal_logpdf(cc[:, None], mu, cov)[0] - got)
    val, _ = integrate.quad(f, mu[6] - 12 * np.sqrt(cov[6, 6]), mu[6] + 12 * np.sqrt(cov[6, 6]), epsabs=0,
                            epsrel=1e-12, limit=200)
    assert abs(val - 1.0) < 1e-10, val


def test_restricted_prior_and_default_rows(oracle_mod):
    c0 = _interior()
    lp0 = oracle_mod.is_log_prior(c0[:, None], *BOX, rows=0b1000010)[0]

    def f(lnd, dec):
        c = c0.copy()
        c[1], c[6] = dec, lnd
        return np.exp(oracle_mod.is_log_prior(c[:, None], *BOX, rows=0b1000010)[0])
    val, _ = integrate.dblquad(f, -np.pi / 2, np.pi / 2, np.log(BOX[2]), np.log(BOX[3]), epsabs=0, epsrel=1e-10)
    assert abs(val - 1.0) < 1e-8, val
    assert np.isfinite(lp0)
    rng = np.random.default_rng(9)
    a, means, covs = _mixture()
    n = 300
    args = (0.2, a, means, covs, 1.5, *BOX, rng.normal(size=(7, n)), rng.uniform(size=(7, n)), rng.uniform(size=n))
    t1, w1, c1 = oracle_mod.mixture_is(*args)
    t2, w2, c2 = oracle_mod.mixture_is(*args, rows=0b1111111)
    assert np.array_equal(t1, t2) and np.array_equal(w1, w2) and np.array_equal(c1, c2)


def test_is_estimate_unbiased_over_sampled_rows(oracle_mod):
    """A likelihood marginalised over phiref and ln D (rows 4 and 6 left out):
    the components sample the other five rows, the left-out rows are prior
    draws, and the weights carry the five rows' densities only."""
    rng = np.random.default_rng(10)
    a, means, covs = _mixture()
    rows = 0b0101111
    n = 24000
    th, lnw, comp = oracle_mod.mixture_is(0.2, a, means, covs, 1.5, *BOX, rng.normal(size=(7, n)),
                                          rng.uniform(size=(7, n)), rng.uniform(size=n), rows=rows)
    c = th.copy()
    c[3] = np.cos(th[3])
    c[6] = np.log(th[6])
    # left-out rows follow the prior whatever the component
    assert stats.kstest(c[4], lambda x: x / (2 * np.pi)).pvalue > 1e-3
    assert stats.kstest(c[6], lambda x: (np.exp(3 * x) - BOX[2] ** 3) / (BOX[3] ** 3 - BOX[2] ** 3)).pvalue > 1e-3
    s_r, s_c = 0.1, 0.08
    lnL = _bump(c, 1.1, 0.25, s_r, s_c)
    Z = np.sqrt(2 * np.pi) * s_r / (2 * np.pi) * np.sqrt(2 * np.pi) * s_c / 2
    terms = np.exp(lnL + lnw)
    assert abs(terms.mean() - Z) < 4 * terms.std() / np.sqrt(n), (terms.mean(), Z)
    # the full seven-row weights on these draws are wrong: the left-out rows
    # were not drawn from the components
    full = oracle_mod.is_log_prior(c, *BOX) - oracle_mod.mixture_log_density(c, 0.2, a, means, covs, 1.5, *BOX)
    tf = np.exp(lnL + full)
    assert abs(tf.mean() - Z) > 4 * tf.std() / np.sqrt(n)
