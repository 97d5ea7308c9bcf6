"""Pins of the oracle's gradient of the likelihood marginalised over
distance (``grad_dmarg``; Eqs. (ap:dexp), (ap:dgh)) against what the
mathematics fixes:

* it is the derivative of ln L_d: central finite differences of the
  marginal (64-node rule) in each of the six sampled rows, cos incl
  included, at SNR 100, where the distance posterior is narrow against the
  prior's variation (sigma_x / x* of a few per cent).  At SNR 30 it is not:
  the x^-4 prior then bends the integrand over the peak, and the rule's own
  derivative departs from the integral's by ~5e-4;
* the value is lnL_dmarg's and the distance row's derivative is 0; a sample
  whose distance peak lies far inside the prior has a finite value and
  derivative, and one whose every node falls outside the prior has value
  -inf and derivative 0.
"""
import numpy as np

from paper_2609_37393_amd import synth

D_MIN, D_MAX = 10.0, 1000.0


def _samples(oracle_mod, pt, n, seed):
    th, _ = synth.weighted_samples(40 * n, seed)
    l = oracle_mod.lnL(pt, th)
    best = th[:, np.argsort(l)[-n:]]
    c = best.copy()
    c[3] = np.cos(c[3])
    c[6] = np.log(c[6])
    return c


def test_grad_dmarg_is_the_derivative(oracle_mod):
    pt = synth.make_point(3, 9, 2000, 16384.0, 100.0, 71)
    c = _samples(oracle_mod, pt, 12, 72)
    ld, g = oracle_mod.grad_dmarg(pt, c, D_MIN, D_MAX, 64)
    want = oracle_mod.lnL_dmarg(pt, oracle_mod._to_physical(c), D_MIN, D_MAX, 64)
    assert np.allclose(ld, want, rtol=1e-13, atol=1e-12)
    assert np.all(g[6] == 0.0)
    h = np.array([1e-6, 1e-6, 1e-6, 1e-6, 1e-6, 1e-8, 0.0])
    for a in range(6):
        cp, cm = c.copy(), c.copy()
        cp[a] += h[a]
        cm[a] -= h[a]
        fp = oracle_mod.lnL_dmarg(pt, oracle_mod._to_physical(cp), D_MIN, D_MAX, 64)
        fm = oracle_mod.lnL_dmarg(pt, oracle_mod._to_physical(cm), D_MIN, D_MAX, 64)
        fd = (fp - fm) / (2 * h[a])
        scale = np.abs(g[a]) + 1e-3 * np.sqrt(np.sum(g[:6] ** 2, axis=0)) + 1e-6
        assert np.all(np.abs(fd - g[a]) <= 1e-4 * scale), (a, np.max(np.abs(fd - g[a]) / scale))


def test_grad_dmarg_edges(oracle_mod):
    pt = synth.make_point(3, 9, 2000, 16384.0, 60.0, 73)
    c = _samples(oracle_mod, pt, 12, 74)
    th = oracle_mod._to_physical(c)
    th[6] = pt["d_ref"]
    K, R = oracle_mod.lnL_terms(pt, th)
    xs, sg = K / R, 1.0 / np.sqrt(R)
    inner = (xs - 10 * sg > pt["d_ref"] / D_MAX) & (xs + 10 * sg < pt["d_ref"] / D_MIN)
    assert inner.sum() >= 6
    c, K, R = c[:, inner], K[inner], R[inner]
    ld, g = oracle_mod.grad_dmarg(pt, c, D_MIN, D_MAX, 20)
    assert np.all(np.isfinite(ld)) and np.all(np.isfinite(g))
    # the same samples with a prior box that excludes the peak far away
    ld2, g2 = oracle_mod.grad_dmarg(pt, c, 1e6, 2e6, 20)
    xs = K / R
    xi_max = np.polynomial.hermite_e.hermegauss(20)[0].max()
    far = pt["d_ref"] / 1e6 < xs - xi_max / np.sqrt(R)  # every node above the box's x range
    assert far.all()
    assert np.all(np.isneginf(ld2)) and np.all(g2 == 0.0)


SIG = np.array([1e-3, 1e-3, 5e-3, 5e-3, 5e-3, 3e-6, 5e-3])
BOX = (-0.01, 0.01, 10.0, 1000.0)


def test_hmc_on_the_distance_marginal(oracle_mod):
    """HMC on L_d p (the distance row frozen): the energy error of a
    trajectory falls as eps^2 (a gradient inconsistent with the marginal
    would leave it O(eps)), the distance row does not move, and NUTS at depth
    one is the one-step HMC transition on the same target."""
    pt = synth.make_point(3, 9, 2000, 16384.0, 100.0, 75)
    c = _samples(oracle_mod, pt, 16, 76)
    # states whose distance peak lies far inside the prior (there the rule's
    # derivative is the integral's; near an edge they differ by the rule's
    # error, and so would the energy)
    th = oracle_mod._to_physical(c)
    th[6] = pt["d_ref"]
    K, R = oracle_mod.lnL_terms(pt, th)
    xs, sg = K / R, 1.0 / np.sqrt(R)
    inner = (xs - 10 * sg > pt["d_ref"] / D_MAX) & (xs + 10 * sg < pt["d_ref"] / D_MIN)
    c = c[:, inner][:, :6]
    assert c.shape[1] == 6
    dm = (D_MIN, D_MAX, 32)
    rng = np.random.default_rng(5)
    z = rng.normal(size=c.shape)
    errs = []
    for eps in (0.02, 0.01):
        p0 = z / SIG[:, None]
        p0[6] = 0.0
        _, U0, _ = oracle_mod.hmc_potential(pt, c, *BOX, dmarg=dm)
        c1, p1, _, U1 = oracle_mod.hmc_trajectory(pt, c, p0, SIG, eps, int(0.2 / eps), *BOX, dmarg=dm)
        H0 = U0 + 0.5 * np.sum(SIG[:, None] ** 2 * p0 ** 2, 0)
        H1 = U1 + 0.5 * np.sum(SIG[:, None] ** 2 * p1 ** 2, 0)
        errs.append(np.abs(H1 - H0))
        assert np.array_equal(c1[6], c[6])
    ratio = errs[0] / errs[1]
    fin = np.isfinite(ratio)
    assert fin.sum() >= 4
    assert np.all((ratio[fin] > 2.5) & (ratio[fin] < 6.0)), ratio
    u = rng.uniform(size=6)
    got = oracle_mod.nuts_step(pt, c, z, np.full((1, 6), 0.75), u[None, :], rng.uniform(size=(1, 6)), SIG, 0.3, 1,
                               *BOX, dmarg=dm)
    want = oracle_mod.hmc_step(pt, c, z, u, SIG, 0.3, 1, *BOX, dmarg=dm)
    assert np.allclose(got[0], want[0], rtol=0, atol=1e-12 * np.abs(c).max())
    assert np.array_equal(got[0][6], c[6])
