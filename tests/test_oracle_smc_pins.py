"""Pins of the oracle's SMC ladder (Eq. (sampler-menu:smc-update) on the
tempered targets of Eq. (sampler-menu:tempered-target)) and of its tempered
moves, against what the mathematics fixes:

* the normalisation ratios telescope: without resampling, the sum of the
  updates from beta = 0 to 1 is the prior-Monte-Carlo estimate
  ln[(1/N) sum_i L_i] (Eq. (sampler-menu:is) with q = p), and the final
  weights are proportional to L;
* the effective-size fraction lies in [1/N, 1] (Cauchy-Schwarz), is 1 at a
  zero step and for a constant likelihood, tends to 1/N when one sample
  dominates, and does not increase with the step;
* the chosen rung meets the target fraction (or is the last rung);
* systematic resampling draws every index floor(N W) or ceil(N W) times, in
  order, and is the identity for equal weights;
* the tempered potential's gradient is the derivative of the tempered
  potential, and at beta = 0 only the prior remains;
* the cloud's random-walk Metropolis move keeps a correlated Gaussian
  target under a mismatched proposal; its increments have covariance
  scale C; a ratio of 1 is always taken and a NaN target never; at beta = 0
  it is the prior's Metropolis move and at beta = 1 the move on L p;
* in the local Gaussian limit the fraction, the chosen rung and the update
  follow from Z_a ~ a^(-d/2) in closed form, with the retained fraction
  [beta (2 - beta)]^(d/2) of Eq. (temper:cost) at the whole remaining step.
"""
import numpy as np

from paper_2609_37393_amd import synth


def _lnL(n, seed, spread=40.0):
    rng = np.random.default_rng(seed)
    return -0.5 * spread * rng.chisquare(3, n)


def test_updates_telescope_to_prior_monte_carlo(oracle_mod):
    lnL = _lnL(5000, 1)
    lnW = np.zeros(5000)
    total = 0.0
    betas = [0.0, 0.02, 0.1, 0.35, 0.7, 1.0]
    for b0, b1 in zip(betas[:-1], betas[1:]):
        d, lnW = oracle_mod.smc_update(lnW, lnL, b0, b1)
        total += d
    m = lnL.max()
    want = m + np.log(np.mean(np.exp(lnL - m)))
    assert abs(total - want) <= 1e-12 * max(1.0, abs(want))
    ref = lnL - (m + np.log(np.sum(np.exp(lnL - m))))
    assert np.max(np.abs(lnW - ref)) <= 1e-10


def test_cess_bounds_and_monotone(oracle_mod):
    n = 400
    lnL = _lnL(n, 2)
    lnW = np.random.default_rng(3).normal(size=n)
    assert abs(oracle_mod.smc_cess(lnW, lnL, 0.0) - 1.0) <= 1e-14
    assert abs(oracle_mod.smc_cess(lnW, np.full(n, -3.7), 0.8) - 1.0) <= 1e-14
    prev = 1.0
    for d in np.linspace(0.0, 1.0, 41)[1:]:
        c = oracle_mod.smc_cess(lnW, lnL, d)
        assert 1.0 / n - 1e-15 <= c <= prev + 1e-15
        prev = c
    spike = np.zeros(n)
    spike[7] = 1e4
    assert abs(oracle_mod.smc_cess(np.zeros(n), spike, 1.0) - 1.0 / n) <= 1e-12
    # -inf likelihoods drop out of every step but the zero step
    lnL2 = lnL.copy()
    lnL2[::5] = -np.inf
    assert abs(oracle_mod.smc_cess(lnW, lnL2, 0.0) - 1.0) <= 1e-14
    assert 0 < oracle_mod.smc_cess(lnW, lnL2, 0.3) < 1


def test_next_rung_meets_the_target(oracle_mod):
    n = 2000
    lnL = _lnL(n, 4)
    lnW = np.zeros(n)
    beta = 0.0
    for target in (0.5, 0.8, 0.3):
        b = oracle_mod.smc_next_beta(lnW, lnL, beta, target)
        assert beta < b <= 1.0
        if b < 1.0:
            assert abs(oracle_mod.smc_cess(lnW, lnL, b - beta) - target) <= 1e-9
        _, lnW = oracle_mod.smc_update(lnW, lnL, beta, b)
        beta = b
    assert oracle_mod.smc_next_beta(lnW, lnL, beta, 1e-6) == 1.0
    # a larger target takes a smaller step
    assert oracle_mod.smc_next_beta(np.zeros(n), lnL, 0.0, 0.9) < oracle_mod.smc_next_beta(np.zeros(n), lnL, 0.0, 0.5)


def test_systematic_resampling_counts(oracle_mod):
    rng = np.random.default_rng(5)
    for n in (1, 7, 1000):
        lnW = rng.normal(size=n) * 3
        W = np.exp(lnW - lnW.max())
        W /= W.sum()
        for u in (0.0, 0.37, 0.999):
            a = oracle_mod.systematic_resample(lnW, u)
            assert a.shape == (n,) and np.all(np.diff(a) >= 0) and a.min() >= 0 and a.max() < n
            cnt = np.bincount(a, minlength=n)
            assert np.all(cnt >= np.floor(n * W - 1e-9)) and np.all(cnt <= np.ceil(n * W + 1e-9))
    assert np.array_equal(oracle_mod.systematic_resample(np.zeros(50), 0.5), np.arange(50))


def test_tempered_potential(oracle_mod):
    sig = np.array([1e-3, 1e-3, 5e-3, 5e-3, 5e-3, 3e-6, 5e-3])
    box = (-0.01, 0.01, 10.0, 1000.0)
    pt = synth.make_point(3, 9, 6554, 32768.0, 100.0, 41)
    th, _ = synth.weighted_samples(2000, 42)
    best = th[:, np.argmax(oracle_mod.lnL(pt, th))]
    c = synth.perturbed_samples(best, sig, 5, 43)
    c[3] = np.cos(c[3])
    c[6] = np.log(c[6])
    beta = 0.3
    l, U, gU = oracle_mod.hmc_potential(pt, c, *box, beta=beta)
    lp = oracle_mod.hmc_log_prior(c, *box)
    assert np.allclose(U, -(beta * l + lp), rtol=0, atol=1e-9 * np.abs(l).max())
    h = np.array([1e-6, 1e-6, 1e-6, 1e-6, 1e-6, 1e-10, 1e-6])
    for a in range(7):
        cp, cm = c.copy(), c.copy()
        cp[a] += h[a]
        cm[a] -= h[a]
        fd = (oracle_mod.hmc_potential(pt, cp, *box, beta=beta)[1] -
              oracle_mod.hmc_potential(pt, cm, *box, beta=beta)[1]) / (2 * h[a])
        assert np.all(np.abs(fd - gU[a]) <= 1e-4 * (np.abs(gU[a]) + np.abs(fd)) + 1e-3 * np.abs(U) * 1e-9 / h[a]), a
    _, U0, g0 = oracle_mod.hmc_potential(pt, c, *box, beta=0.0)
    assert np.array_equal(U0, -lp)
    assert np.all(g0[[0, 2, 3, 4, 5]] == 0) and np.allclose(g0[1], np.tan(c[1])) and np.all(g0[6] == -3.0)


def _gauss_target(scale):
    scale = np.asarray(scale, np.float64)
    return lambda c: -0.5 * np.sum((np.asarray(c) / scale[:, None]) ** 2, axis=0)


def test_rwm_leaves_a_gaussian_invariant(oracle_mod):
    """The cloud's random-walk Metropolis move keeps its target: exact draws
    of a correlated Gaussian, three moves each with a proposal covariance that
    does not match, keep their mean and variance within sampling error."""
    rng = np.random.default_rng(21)
    n = 6000
    A = rng.normal(size=(7, 7)) * 0.3 + np.eye(7)
    Sig = A @ A.T
    Li = np.linalg.inv(np.linalg.cholesky(Sig))
    logpi = (lambda c: -0.5 * np.sum((Li @ np.asarray(c)) ** 2, axis=0))
    c = np.linalg.cholesky(Sig) @ rng.normal(size=(7, n))
    prop = np.diag(np.diag(Sig))  # the diagonal only: a mismatched proposal
    acc_all = []
    for _ in range(3):
        c, _, acc = oracle_mod.rwm_chain(logpi, c, rng.normal(size=(7, n)), rng.uniform(size=n), prop, 2.38 ** 2 / 7)
        acc_all.append(acc.mean())
    assert 0.1 < np.mean(acc_all) < 0.9
    w = Li @ c  # whitened: unit normal if the target is kept
    assert np.all(np.abs(w.mean(axis=1)) < 4.0 / np.sqrt(n)), w.mean(axis=1)
    assert np.all(np.abs(w.var(axis=1) - 1.0) < 4.0 * np.sqrt(2.0 / n)), w.var(axis=1)


def test_rwm_proposal_and_decisions(oracle_mod):
    """The proposal's increments have covariance scale C (a transposed
    Cholesky factor fails on a correlated C); a move whose target ratio is 1
    is always taken, one to a NaN or -inf target never; at beta = 0 the
    tempered move on the likelihood is the prior's Metropolis move."""
    rng = np.random.default_rng(22)
    n = 40000
    C = np.eye(7) * 0.04
    C[0, 2] = C[2, 0] = 0.03
    flat = (lambda c: np.zeros(np.asarray(c).shape[1]))
    c0 = np.zeros((7, n))
    c1, _, acc = oracle_mod.rwm_chain(flat, c0, rng.normal(size=(7, n)), rng.uniform(size=n), C, 0.5)
    assert acc.all()
    S = np.cov(c1)
    assert abs(S[0, 2] - 0.5 * 0.03) < 5 * np.sqrt((0.02 * 0.02 + 0.015 ** 2) / n)
    assert abs(S[0, 0] - 0.02) < 5 * 0.02 * np.sqrt(2.0 / n)
    nan_t = (lambda c: np.where(np.asarray(c)[0] == 0.0, 0.0, np.nan))
    _, _, acc = oracle_mod.rwm_chain(nan_t, c0[:, :100], rng.normal(size=(7, 100)), rng.uniform(size=100), C, 1.0)
    assert not acc.any()
    # beta = 0 on the likelihood: the decision is the prior ratio alone
    pt = synth.make_point(2, 4, 2000, 16384.0, 50.0, 23)
    th, _ = synth.weighted_samples(400, 24)
    c = th.copy()
    c[3] = np.cos(c[3])
    c[6] = np.log(c[6])
    box = (-0.01, 0.01, 10.0, 1000.0)
    l0 = oracle_mod.lnL(pt, th)
    z, u = rng.normal(size=(7, 400)), rng.uniform(size=400)
    got_c, got_l, got_a = oracle_mod.rwm_step(pt, c, z, u, C * 0.01, 1.0, *box, l0, beta=0.0)
    lp = (lambda x: oracle_mod.hmc_log_prior(x, *box))
    want_c, _, want_a = oracle_mod.rwm_chain(lp, c, z, u, C * 0.01, 1.0)
    assert np.array_equal(got_a, want_a) and np.array_equal(got_c, want_c)
    # and beta = 1 is the Metropolis move on L p
    got_c, got_l, got_a = oracle_mod.rwm_step(pt, c, z, u, C * 0.01, 1.0, *box, l0, beta=1.0)
    post = (lambda x: np.where(np.isfinite(lp(x)),
                               oracle_mod.lnL(pt, oracle_mod._to_physical(np.where(np.isfinite(lp(x)), x, c)))
                               + lp(x), -np.inf))
    want_c, _, want_a = oracle_mod.rwm_chain(post, c, z, u, C * 0.01, 1.0)
    assert np.array_equal(got_a, want_a)
    assert 0.05 < got_a.mean() < 0.95


def _tempered_gauss(n, d, beta, seed):
    """Exact draws x ~ N(0, I / beta) of the tempered target L^beta for
    L = exp(-|x|^2 / 2) under a flat prior, and their ln L."""
    x = np.random.default_rng(seed).normal(size=(n, d)) / np.sqrt(beta)
    return -0.5 * np.sum(x * x, axis=1)


def _log_frac_se(lnL, dbeta):
    """Delta-method standard error of the log of the sampled fraction
    mean(r)^2 / mean(r^2), r = L^dbeta."""
    r = np.exp(dbeta * lnL)
    m1, m2 = r.mean(), (r * r).mean()
    g = np.stack([2.0 * r / m1, -(r * r) / m2])
    return float(np.sqrt(np.cov(g).sum() / r.size))


def test_cess_local_gaussian_limit(oracle_mod):
    """In the local Gaussian limit with a flat prior, Z_a scales as a^(-d/2),
    so the fraction of the incremental weights L^dbeta over draws from the
    rung at beta is Z_(beta+dbeta)^2 / (Z_beta Z_(beta+2 dbeta)) =
    [beta (beta + 2 dbeta) / (beta + dbeta)^2]^(d/2) and the normalisation
    ratio is (beta / (beta + dbeta))^(d/2); the whole remaining step
    dbeta = 1 - beta gives the retained fraction [beta (2 - beta)]^(d/2) of
    Eq. (temper:cost).  Exact draws of that limit check the oracle's
    fraction, its chosen rung and its update within six standard errors."""
    n, d = 400_000, 6
    for beta, seed in ((0.05, 31), (0.3, 32), (0.8, 33)):
        lnL = _tempered_gauss(n, d, beta, seed)
        lnW = np.zeros(n)
        rest = 1.0 - beta
        want = 0.5 * d * np.log(beta * (2.0 - beta))
        got = np.log(oracle_mod.smc_cess(lnW, lnL, rest))
        assert abs(got - want) <= 6.0 * _log_frac_se(lnL, rest), (beta, got, want)
        for target in (0.5, 0.9):
            b = oracle_mod.smc_next_beta(lnW, lnL, beta, target)
            db = b - beta
            if want - np.log(target) > 6.0 * _log_frac_se(lnL, rest):
                assert b == 1.0  # the whole remaining step qualifies
            else:
                assert 0.0 < db < rest
                frac = 0.5 * d * np.log(beta * (beta + 2.0 * db) / (beta + db) ** 2)
                assert abs(frac - np.log(target)) <= 6.0 * _log_frac_se(lnL, db), (beta, target, b)
            dz, _ = oracle_mod.smc_update(lnW, lnL, beta, b)
            r = np.exp(db * lnL)
            assert abs(dz + 0.5 * d * np.log(b / beta)) <= 6.0 * r.std() / (r.mean() * np.sqrt(n)), (beta, target, dz)
