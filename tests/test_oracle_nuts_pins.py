"""Pins of the oracle's No-U-Turn transition (the gradient sampler of
Sec. "Sampler menu": multinomial NUTS with the generalised criterion),
against what the mathematics fixes:

* one doubling is one leapfrog step with Metropolis acceptance: at depth 1
  the transition equals the (separately pinned) HMC transition with one
  step, forward or, with the momentum negated, backward;
* it leaves its target invariant: started from exact draws of a Gaussian
  target, one transition per chain returns draws whose mean and variance
  match the target's within their sampling error (a wrong leaf weight,
  merge rule or U-turn check breaks this at the step size used);
* the U-turn criterion stops a trajectory after a fixed fraction of the
  target's oscillation period: a step four times smaller takes about two
  more doublings.
"""
import numpy as np

from paper_2609_37393_amd import synth

SIG = np.array([1e-3, 1e-3, 5e-3, 5e-3, 5e-3, 3e-6, 5e-3])
BOX = (-0.01, 0.01, 10.0, 1000.0)


def _gauss(scale):
    scale = np.asarray(scale, np.float64)

    def pot(c):
        c = np.asarray(c, np.float64)
        U = 0.5 * np.sum((c / scale[:, None]) ** 2, axis=0)
        return -U, U, c / scale[:, None] ** 2

    return pot


def test_depth_one_is_one_step_hmc(oracle_mod):
    pt = synth.make_point(3, 9, 6554, 32768.0, 100.0, 41)
    th, _ = synth.weighted_samples(4000, 42)
    best = th[:, np.argmax(oracle_mod.lnL(pt, th))]
    c0 = synth.perturbed_samples(best, SIG, 12, 43)
    c0[3] = np.cos(c0[3])
    c0[6] = np.log(c0[6])
    rng = np.random.default_rng(1)
    z = rng.normal(size=c0.shape)
    u = rng.uniform(size=12)
    for sgn, dirs in ((1.0, np.full((1, 12), 0.75)), (-1.0, np.full((1, 12), 0.25))):
        leaves = rng.uniform(size=(1, 12))
        got_c, got_l, dep, st, dv = oracle_mod.nuts_step(pt, c0, z, dirs, u[None, :], leaves, SIG, 0.4, 1, *BOX)
        want_c, want_l, acc = oracle_mod.hmc_step(pt, c0, sgn * z, u, SIG, 0.4, 1, *BOX)
        assert np.all(st == 1) and not dv.any()
        assert np.allclose(got_c, want_c, rtol=0, atol=1e-12 * np.abs(c0).max())
        assert np.allclose(got_l, want_l, rtol=1e-13, atol=0)


def test_transition_leaves_a_gaussian_invariant(oracle_mod):
    rng = np.random.default_rng(2)
    scale = np.array([1.0, 2.0, 0.5, 0.1, 3.0, 1.5, 0.7])
    pot = _gauss(scale)
    n = 3000
    c0 = rng.normal(size=(7, n)) * scale[:, None]
    sig = scale * np.array([1.3, 0.8, 1.0, 1.0, 0.6, 1.2, 0.9])  # a mass that does not match exactly
    D = 6
    out = np.empty_like(c0)
    steps = 0
    for i in range(n):
        c, _, _, s, _ = oracle_mod.nuts_chain(pot, c0[:, i], rng.normal(size=7), rng.uniform(size=D), rng.uniform(size=D),
                                              rng.uniform(size=2 ** D - 1), sig, 0.7, D)
        out[:, i] = c
        steps += s
    assert steps / n > 3  # the trajectories do move
    z = out / scale[:, None]
    # mean 0, variance 1 per coordinate within about four standard errors
    assert np.all(np.abs(z.mean(axis=1)) < 4.0 / np.sqrt(n)), z.mean(axis=1)
    assert np.all(np.abs(z.var(axis=1) - 1.0) < 4.0 * np.sqrt(2.0 / n)), z.var(axis=1)
    # and the chains did not stay put
    assert np.mean(np.all(out == c0, axis=0)) < 0.2


def test_uturn_length_scales_with_the_period(oracle_mod):
    """On a unit Gaussian with the matching mass a trajectory from near the
    mode turns after about a quarter period (the edge momentum reverses
    against the summed momentum), so its doubling depth is about
    log2(pi / (2 eps)): a step four times smaller adds about two doublings."""
    pot = _gauss(np.ones(7))
    mean = []
    for eps in (0.05, 0.0125):
        rng = np.random.default_rng(3)
        deps = []
        for _ in range(20):
            c0 = rng.normal(size=7) * 0.1
            c, _, dep, st, dv = oracle_mod.nuts_chain(pot, c0, rng.normal(size=7), np.full(10, 0.75), np.zeros(10),
                                                      np.zeros(1023), np.ones(7), eps, 10)
            assert not dv and dep < 10
            deps.append(dep)
        mean.append(np.mean(deps))
    assert 4 <= mean[0] <= 6, mean
    # two more doublings in the continuum; the discrete phase of the turn
    # within a doubling makes the sample mean move by 1 to 2.5
    assert 1.0 <= mean[1] - mean[0] <= 2.5, mean
