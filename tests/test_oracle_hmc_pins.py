"""Pins of the oracle's Hamiltonian transition (a gradient sampler on the
likelihood, Sec. "Sampling the differentiable extrinsic likelihood") against
what the mathematics fixes, not against the oracle itself:

* the potential's gradient is the derivative of the potential (central
  differences of U = -lnL - ln prior, each from the oracle's own lnL);
* the leapfrog integrator is second order: at a fixed trajectory length,
  halving the step cuts the energy error about four times;
* it is reversible: from the end state with the momentum negated, the same
  steps return to the start (the cos incl reflection included);
* at a vanishing step the energy is conserved, so chains inside the prior
  box are accepted, and a proposal that leaves the box is rejected.
"""
import numpy as np

from paper_2609_37393_amd import synth

SIG = np.array([1e-3, 1e-3, 5e-3, 5e-3, 5e-3, 3e-6, 5e-3])
BOX = (-0.01, 0.01, 10.0, 1000.0)


def _start(oracle_mod, pt, n, seed):
    th, _ = synth.weighted_samples(40 * n, seed)
    best = th[:, np.argmax(oracle_mod.lnL(pt, th))]
    c = synth.perturbed_samples(best, SIG, n, seed + 1)
    c[3] = np.cos(c[3])
    c[6] = np.log(c[6])
    return c


def test_potential_gradient(oracle_mod):
    pt = synth.make_point(3, 9, 6554, 32768.0, 100.0, 41)
    c = _start(oracle_mod, pt, 6, 42)
    _, U, gU = oracle_mod.hmc_potential(pt, c, *BOX)
    h = np.array([1e-6, 1e-6, 1e-6, 1e-6, 1e-6, 1e-10, 1e-6])
    for a in range(7):
        cp, cm = c.copy(), c.copy()
        cp[a] += h[a]
        cm[a] -= h[a]
        fd = (oracle_mod.hmc_potential(pt, cp, *BOX)[1] - oracle_mod.hmc_potential(pt, cm, *BOX)[1]) / (2 * h[a])
        assert np.all(np.abs(fd - gU[a]) <= 1e-4 * (np.abs(gU[a]) + np.abs(fd)) + 1e-3 * np.abs(U) * 1e-9 / h[a]), a


def test_leapfrog_second_order_and_reversible(oracle_mod):
    pt = synth.make_point(3, 9, 6554, 32768.0, 100.0, 43)
    c0 = _start(oracle_mod, pt, 8, 44)
    z = np.random.default_rng(1).normal(size=c0.shape)
    p0 = z / SIG[:, None]
    _, U0, _ = oracle_mod.hmc_potential(pt, c0, *BOX)
    H0 = U0 + 0.5 * np.sum(SIG[:, None] ** 2 * p0 * p0, axis=0)
    dH = []
    for eps, L in ((0.04, 5), (0.02, 10), (0.01, 20)):
        c, p, _, U = oracle_mod.hmc_trajectory(pt, c0, p0, SIG, eps, L, *BOX)
        dH.append(np.median(np.abs(U + 0.5 * np.sum(SIG[:, None] ** 2 * p * p, axis=0) - H0)))
    assert 2.5 < dH[0] / dH[1] < 6.0 and 2.5 < dH[1] / dH[2] < 6.0, dH
    c1, p1, _, _ = oracle_mod.hmc_trajectory(pt, c0, p0, SIG, 0.02, 10, *BOX)
    c2, p2, _, _ = oracle_mod.hmc_trajectory(pt, c1, -p1, SIG, 0.02, 10, *BOX)
    assert np.all(np.abs(c2 - c0) <= 1e-9 * SIG[:, None] * 1e3), np.abs((c2 - c0) / SIG[:, None]).max()
    assert np.all(np.abs(p2 + p0) <= 1e-6 * (np.abs(p0) + 1.0 / SIG[:, None]))


def test_acceptance_limits(oracle_mod):
    pt = synth.make_point(3, 9, 6554, 32768.0, 100.0, 45)
    c0 = _start(oracle_mod, pt, 16, 46)
    z = np.random.default_rng(2).normal(size=c0.shape)
    u = np.random.default_rng(3).uniform(0.05, 1.0, c0.shape[1])
    c, l, acc = oracle_mod.hmc_step(pt, c0, z, u, SIG, 1e-4, 2, *BOX)
    assert acc.all()
    # a box that excludes every proposal in time: all rejected, the states kept
    box = (c0[5].max() + 1.0, c0[5].max() + 2.0, 10.0, 1000.0)
    c, l, acc = oracle_mod.hmc_step(pt, c0, z, u, SIG, 1e-4, 2, *box)
    assert not acc.any() and np.array_equal(c, c0)
