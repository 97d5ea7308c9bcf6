"""Pins of the oracle's joint marginal over phiref and psi by exact
reconstruction (ERAI, Eqs. (ap:angleharm), (ap:nyquist)) against what the
mathematics fixes, not against the oracle itself:

* the reconstructed finite harmonic model reproduces the oracle's own lnL at
  angles off the sampling grid; with modes of odd m the paper's count
  N_phi = 2 m_max + 1 does not (the data term then carries odd harmonics,
  so 4 m_max + 1 angles are needed), while with even m alone it would;
* a fine grid equal to the sampling grid returns the mean of e^{lnL} over
  the sampled angles exactly;
* one angle in phiref is the periodic trapezoid rule over psi alone, the
  oracle's polarisation marginal evaluated directly at each angle;
* the rule converges to adaptive two-dimensional quadrature of e^{lnL} over
  the torus.
"""
import numpy as np
from scipy import integrate

from paper_2609_37393_amd import synth

from ._helpers import lnL_scale


def _point(M, snr, seed, lm=None):
    return synth.make_point(3, M, 2000, 16384.0, snr, seed, lm=lm)


def _model(C, alpha, u):
    Nf, Np = C.shape[1:]
    qf = np.fft.fftfreq(Nf, 1.0 / Nf)
    pf = np.fft.fftfreq(Np, 1.0 / Np)
    return np.einsum("nqp,nq,np->n", C, np.exp(1j * np.outer(alpha, qf)), np.exp(1j * np.outer(u, pf))).real


def test_reconstruction_off_grid(oracle_mod):
    pt = _point(9, 40.0, 3)  # modes up to (3, +-3), odd m present
    th = synth.prior_samples(40, 4)
    C, _ = oracle_mod.angle_coefficients(pt, th)
    assert C.shape == (40, 13, 5)
    rng = np.random.default_rng(5)
    alpha = rng.uniform(0, 2 * np.pi, 40)
    u = rng.uniform(0, 2 * np.pi, 40)
    th2 = th.copy()
    th2[4] += alpha
    th2[2] += u / 2
    want = oracle_mod.lnL(pt, th2)
    S = lnL_scale(oracle_mod, pt, th2)
    assert np.all(np.abs(_model(C, alpha, u) - want) <= 1e-10 * S)


def test_paper_count_needs_even_modes(oracle_mod):
    """The count 2 m_max + 1 in phiref: enough with even m only, not with odd."""
    rng = np.random.default_rng(6)
    for lm, enough in (([(2, 2), (2, -2), (2, 0), (4, 4), (4, -4), (4, 2)], True),
                       ([(2, 2), (2, -2), (2, 1), (3, 3)], False)):
        pt = _point(len(lm), 40.0, 7, lm=lm)
        m_max = max(abs(m) for _, m in lm)
        th = synth.prior_samples(12, 8)
        Nf = 2 * m_max + 1
        al = 2 * np.pi * np.arange(Nf) / Nf
        uc = 2 * np.pi * np.arange(5) / 5
        big = np.repeat(th, Nf * 5, axis=1)
        big[4] += np.tile(np.repeat(al, 5), th.shape[1])
        big[2] += np.tile(np.tile(uc / 2, Nf), th.shape[1])
        L = oracle_mod.lnL(pt, big).reshape(th.shape[1], Nf, 5)
        C = np.fft.fft2(L, axes=(1, 2)) / (Nf * 5)
        # with q even only, the samples over [0, 2 pi) alias q onto q mod Nf:
        # compare at offsets where that matters
        alpha = rng.uniform(0, 2 * np.pi, th.shape[1])
        u = rng.uniform(0, 2 * np.pi, th.shape[1])
        th2 = th.copy()
        th2[4] += alpha
        th2[2] += u / 2
        want = oracle_mod.lnL(pt, th2)
        S = lnL_scale(oracle_mod, pt, th2)
        if enough:
            # even harmonics up to 2 m_max: the model in 2 phi has degree
            # m_max, so Nf angles over [0, pi) would do; over [0, 2 pi) the
            # even coefficients c_q (|q| <= 2 m_max) fold pairwise, so use the
            # half-period grid
            al2 = np.pi * np.arange(Nf) / Nf
            big = np.repeat(th, Nf * 5, axis=1)
            big[4] += np.tile(np.repeat(al2, 5), th.shape[1])
            big[2] += np.tile(np.tile(uc / 2, Nf), th.shape[1])
            L2 = oracle_mod.lnL(pt, big).reshape(th.shape[1], Nf, 5)
            C2 = np.fft.fft2(L2, axes=(1, 2)) / (Nf * 5)
            got = _model(C2, 2 * alpha, u)  # the model's variable is 2 phi
            assert np.all(np.abs(got - want) <= 1e-10 * S)
        else:
            err = np.abs(_model(C, alpha, u) - want) / S
            assert err.max() > 1e-3


def test_fine_grid_equal_to_sampling_grid(oracle_mod):
    pt = _point(9, 30.0, 9)
    th = synth.prior_samples(20, 10)
    Nf, Np = oracle_mod.erai_grid(pt)
    _, L = oracle_mod.angle_coefficients(pt, th)
    got = oracle_mod.lnL_erai(pt, th, Nf, Np)
    m = L.reshape(20, -1).max(axis=1)
    want = m + np.log(np.mean(np.exp(L.reshape(20, -1) - m[:, None]), axis=1))
    assert np.all(np.abs(got - want) <= 1e-11 * (1 + np.abs(want)))


def test_one_phase_angle_is_the_polarisation_trapezoid(oracle_mod):
    pt = _point(9, 60.0, 11)
    th = synth.prior_samples(25, 12)
    got = oracle_mod.lnL_erai(pt, th, 1, 64)
    want = oracle_mod.lnL_pmarg(pt, th, "trapezoid", 64)
    S = lnL_scale(oracle_mod, pt, th)
    assert np.all(np.abs(got - want) <= 1e-10 * S)


def test_converges_to_quadrature_over_the_torus(oracle_mod):
    pt = _point(4, 12.0, 13)
    th = synth.weighted_samples(200, 14)[0][:, :3]
    C, _ = oracle_mod.angle_coefficients(pt, th)
    for i in range(th.shape[1]):
        c = C[i:i + 1]

        def f(u, a):
            return np.exp(_model(c, np.array([a]), np.array([u]))[0])

        val, _ = integrate.dblquad(f, 0.0, 2 * np.pi, 0.0, 2 * np.pi, epsabs=0, epsrel=1e-12)
        want = np.log(val / (4 * np.pi ** 2))
        got = oracle_mod.lnL_erai(pt, th[:, i:i + 1], 96, 96)[0]
        assert abs(got - want) <= 1e-9 * max(1.0, abs(want)), (i, got, want)
