"""Pins of the oracle's composite-index (generalised-response) likelihood,
Sec. "A generalized detector response", against what the paper and the
mathematics fix, not against the oracle itself:

* the sidereal harmonics: F_k over the Greenwich hour angle is a trigonometric
  polynomial of degree 2 whose five coefficients reproduce it at every angle
  (Eq. (slowrot:Fharm));
* the rotation coefficients with the arrival-time post-phase: the composite
  template sum_n C~_n chi_n placed at t_k equals F_k(t) h(t - t_k) at every
  time t, with the modulation of the bank referenced to the template's own
  time (Eqs. (slowrot:master), (slowrot:commutator), (slowrot:postphase));
* the delay-drift coefficients (Path B): the composite template of order P
  equals the order-P Taylor series of the strain with the drifting delay (to
  the rounding of its terms), and order 0 is Path A;
* the finite-arm coefficients: sum_p b_p W_p reproduces the Michelson response
  built from the arm transfer function, with W_p the Taylor coefficients of
  the residual transfer in u = a.n (Eqs. (slowrot:armtransfer), (fsize:FA),
  (fsize:Dhat), (fsize:Wp), (fsize:bp)), and b_0 is the static antenna factor;
* the widened contraction: it equals the direct noise-weighted inner products
  <h_k|d> - 1/2 <h_k|h_k> of h_k = Re[sum_A c_A T_{t_k} chi_A] built from the
  bank's spectra (Eq. (slowrot:lnL:Decomposed) from Eq. (resp:static:ip));
* the regression limits: zero rotation rate and the arms' zeroth order give
  the static likelihood exactly (Sec. "Earth rotation...": Omega -> 0; Sec.
  "Long arms...": p_max = 0);
* lnL <= 1/2 <d|d> (Cauchy-Schwarz) and exact quadratic dependence on
  x = D_ref / D.
"""
import numpy as np
import pytest

from paper_2609_37393_amd import synth

from ._helpers import response


def _rand_det(rng):
    x = rng.normal(size=3)
    x /= np.linalg.norm(x)
    y = rng.normal(size=3)
    y -= x * x.dot(y)
    y /= np.linalg.norm(y)
    return x, y, 0.5 * (np.outer(x, x) - np.outer(y, y))


def test_rotation_harmonics_reproduce_the_antenna_factor(oracle_mod):
    rng = np.random.default_rng(1)
    for _ in range(20):
        _, _, D = _rand_det(rng)
        dec = np.arcsin(rng.uniform(-1, 1))
        psi = rng.uniform(0, np.pi)
        A = oracle_mod.rotation_harmonics(D, dec, psi)
        for g in rng.uniform(-10, 10, size=7):
            F, _ = oracle_mod.antenna(D, 0.0, dec, psi, g)  # hour angle g = gmst - ra
            want = np.sum(A * np.exp(1j * np.arange(-2, 3) * g))
            assert abs(F - want) < 1e-13, (F, want)
        # psi enters as e^{-2 i psi} on every harmonic (the polarisation law)
        A2 = oracle_mod.rotation_harmonics(D, dec, psi + 0.3)
        assert np.allclose(A2, A * np.exp(-2j * 0.3), atol=1e-14)


@pytest.mark.parametrize("omega", [synth.SIDEREAL_RATE, 40.0])
def test_rotation_template_identity(oracle_mod, omega):
    """sum_n C~_n e^{i n W (t - t_k)} = F_k(g(t)) for every t: the bank holds
    chi_n(t) = e^{i n W t} h(t) in the template's own time, placed at t_k; the
    physical response is F_k(t) h(t - t_k).  A large W magnifies any error in
    the post-phase (which is a W (t_k - t_ref) rotation of each harmonic)."""
    pt = synth.make_point_wide(3, 2, 5, 400, 4096.0, 20.0, 3, response="rotation", omega=omega)
    rng = np.random.default_rng(2)
    th = synth.prior_samples(10, 7)
    for i in range(th.shape[1]):
        C, tk = oracle_mod.wide_coef(pt, th[:, i])
        ra, dec, psi, tref = th[0, i], th[1, i], th[2, i], th[5, i]
        for k in range(3):
            # the arrival time uses the sky frame at t_ref
            want_tk = oracle_mod.arrival_time(pt["det_pos"][k], ra, dec, pt["gmst"] + omega * tref, tref)
            assert abs(tk[k] - want_tk) < 1e-15
            for t in tref + rng.uniform(-0.05, 0.05, size=5):
                F, _ = oracle_mod.antenna(pt["det_tensor"][k], ra, dec, psi, pt["gmst"] + omega * t)
                got = np.sum(C[k] * np.exp(1j * np.arange(-2, 3) * omega * (t - tk[k])))
                assert abs(got - F) < 1e-12, (omega, k, got, F)


@pytest.mark.parametrize("omega", [synth.SIDEREAL_RATE * 3e3, 40.0])
def test_delay_drift_template(oracle_mod, omega):
    """Path B (Eq. (slowrot:delay) composed with Eq. (slowrot:Fharm) into
    Eq. (slowrot:master)).  For a pure tone h(t) = e^{i w t}, whose p-th
    derivative is (i w)^p h, the composite template placed at t_k,
      sum_{p <= P, n} C~_(p,n) e^{i n W (t - t_k)} (i w)^p e^{i w (t - t_k)},
    equals F_k(t) e^{i w (t - t_k)} sum_{p <= P} (-i w dt(t))^p / p!,
    with F_k(t) the antenna factor at the sidereal angle of time t and dt(t)
    the drift of the arrival-time delay since t_ref (the sky frame at each
    t): the order-P Taylor series of the strain F_k(t) h(t - t_k - dt(t)).
    Order 0 is the rotation coefficients (Path A)."""
    th = synth.prior_samples(6, 8)
    pts = {n_a: synth.make_point_wide(3, 2, n_a, 400, 4096.0, 20.0, 3, response="rotation_delay", omega=omega)
           for n_a in (5, 12, 21, 32)}
    rot = synth.make_point_wide(3, 2, 5, 400, 4096.0, 20.0, 3, response="rotation", omega=omega)
    for i in range(th.shape[1]):
        C0, _ = oracle_mod.wide_coef(pts[5], th[:, i])
        Cr, _ = oracle_mod.wide_coef(rot, th[:, i])
        assert np.allclose(C0, Cr, rtol=0, atol=1e-14)
        ra, dec, psi, tref = th[0, i], th[1, i], th[2, i], th[5, i]
        for P, n_a in ((1, 12), (2, 21), (3, 32)):
            pt = pts[n_a]
            C, tk = oracle_mod.wide_coef(pt, th[:, i])
            for k in range(3):
                ts = tref + np.linspace(-0.05, 0.05, 9)
                dts = np.array([oracle_mod.arrival_time(pt["det_pos"][k], ra, dec, pt["gmst"] + omega * t, t) - t
                                for t in ts]) - (tk[k] - tref)
                w = 0.7 / max(np.abs(dts).max(), 1e-9)  # w |dt| up to 0.7
                for t, dt in zip(ts, dts):
                    F, _ = oracle_mod.antenna(pt["det_tensor"][k], ra, dec, psi, pt["gmst"] + omega * t)
                    want = F * sum((-1j * w * dt) ** p / np.prod(np.arange(1, p + 1)) for p in range(P + 1))
                    got, a, scale = 0.0j, 0, 0.0
                    for p in range(P + 1):
                        for nt in range(-(2 + p), 3 + p):
                            term = C[k, a] * np.exp(1j * nt * omega * (t - tk[k])) * (1j * w) ** p
                            got += term
                            scale += abs(term)
                            a += 1
                    # the harmonic form of (-dt)^p cancels: its coefficients are
                    # of size (|r| cos dec)^p while dt^p is far smaller, so the
                    # rounding of the sum is relative to its terms' magnitudes
                    assert abs(got - want) <= 1e-13 * scale + 1e-12 * abs(F), (omega, P, k, got, want, scale)


def _dhat(u, x):
    """Residual arm transfer e^{2 i x} D~(u, x) of Eq. (fsize:Dhat), from the
    two-leg transfer function of Eq. (slowrot:armtransfer) with x = pi f T."""
    def sinc(z):
        return np.sinc(z / np.pi)  # sin(z) / z
    dt = 0.5 * np.exp(-2j * x) * (np.exp(1j * x * (1 - u)) * sinc(x * (1 + u)) +
                                  np.exp(-1j * x * (1 + u)) * sinc(x * (1 - u)))
    return np.exp(2j * x) * dt


@pytest.mark.parametrize("fT", [0.02, 0.2, 0.6])
def test_arm_coefficients_reproduce_the_michelson_response(oracle_mod, fT):
    """sum_p b_p W_p(x) = 1/2 [Dhat(x.N) e:xx - Dhat(y.N) e:yy] (the complex
    response F = F+ + i Fx with the common light-crossing shift removed), with
    W_p the Taylor coefficients of Dhat in u from a Chebyshev fit."""
    x = np.pi * fT
    P = 26
    nodes = np.cos(np.pi * (np.arange(64) + 0.5) / 64)
    cheb = np.polynomial.chebyshev.Chebyshev.fit(nodes, _dhat(nodes, x).real, P) , \
        np.polynomial.chebyshev.Chebyshev.fit(nodes, _dhat(nodes, x).imag, P)
    Wp = cheb[0].convert(kind=np.polynomial.Polynomial).coef + 1j * cheb[1].convert(kind=np.polynomial.Polynomial).coef
    assert abs(Wp[0] - np.sin(x) / x * np.cos(x)) < 1e-12  # W_0 = sinc(x) cos(x)
    net = synth.network(2, 9)
    base = synth.make_point(2, 2, 64, 4096.0, 10.0, 9, net=net)
    pt = synth.widen_static(base, P + 1, response="arms")
    th = synth.prior_samples(12, 8)
    for i in range(th.shape[1]):
        b, _ = oracle_mod.wide_coef(pt, th[:, i])
        ra, dec, psi = th[0, i], th[1, i], th[2, i]
        for k in range(2):
            F0, N = oracle_mod.antenna(pt["det_tensor"][k], ra, dec, psi, pt["gmst"])
            assert abs(b[k, 0] - F0) < 1e-14  # b_0 is the static antenna factor
            ax, ay = pt["det_arms"][k]
            # e : a a = (X.a + i Y.a)^2, with F(psi) = e : D for D = (x x - y y)/2
            Fx, _ = oracle_mod.antenna(np.outer(ax, ax), ra, dec, psi, pt["gmst"])
            Fy, _ = oracle_mod.antenna(np.outer(ay, ay), ra, dec, psi, pt["gmst"])
            want = 0.5 * (_dhat(ax @ N, x) * Fx - _dhat(ay @ N, x) * Fy)
            got = np.sum(b[k] * Wp)
            assert abs(got - want) < 1e-9, (fT, k, got, want)


def _direct_wide(sp, C, tk, Y, x):
    """sum_k <h_k|d> - 1/2 <h_k|h_k> with h_k = Re[sum_A c_A T_{t_k} chi_A],
    c_(a,lm) = C~_(k,a) Y_lm, built in the frequency domain from the bank's
    spectra (no factorisation)."""
    f, G, w, d = sp["f"], sp["G"], sp["w"], sp["d"]
    tot = 0.0
    for k in range(C.shape[0]):
        c = (C[k][:, None] * Y[None, :]).reshape(-1) * x
        hc = c @ G
        hk = 0.5 * np.exp(-2j * np.pi * f * tk[k]) * (hc + np.conj(hc[::-1]))
        tot += np.real(np.sum(w[k] * np.conj(hk) * d[k])) - 0.5 * np.sum(w[k] * np.abs(hk) ** 2)
    return tot


@pytest.mark.parametrize("resp,n_a", [("rotation", 5), ("arms", 3), ("rotation_delay", 12)])
def test_wide_likelihood_equals_direct_inner_products(oracle_mod, resp, n_a):
    pt = synth.make_point_wide(3, 4, n_a, 6554, 32768.0, 60.0, 21, response=resp, keep_spectra=True)
    sp = pt["spectra"]
    th = synth.prior_samples(25, 6)
    got = oracle_mod.lnL_wide(pt, th)
    for i in range(th.shape[1]):
        C, tk = oracle_mod.wide_coef(pt, th[:, i])
        Y = np.array([oracle_mod.ylm(l, m, th[3, i], th[4, i]) for l, m in pt["lm"]])
        want = _direct_wide(sp, C, tk, Y, pt["d_ref"] / th[6, i])
        # the residual is the four-point cubic's read of the 32768 Hz table
        assert abs(got[i] - want) < 2e-6 * (abs(want) + 60.0 ** 2), (i, got[i], want)


def test_zero_rotation_and_zeroth_arm_order_give_the_static_likelihood(oracle_mod):
    base = synth.make_point(3, 9, 2000, 32768.0, 150.0, 31)
    th = np.concatenate([synth.prior_samples(300, 32), synth.weighted_samples(100, 33)[0]], axis=1)
    want = oracle_mod.lnL(base, th)
    S = np.abs(want) + 1.0
    rot = synth.widen_static(base, 5, response="rotation")  # omega = 0: chi_n = h for every n
    got = oracle_mod.lnL_wide(rot, th)
    assert np.all(np.abs(got - want) <= 1e-11 * S * 40), np.abs(got - want).max()
    arms = synth.widen_static(base, 1, response="arms")
    got = oracle_mod.lnL_wide(arms, th)
    assert np.all(np.abs(got - want) <= 1e-12 * S * 40), np.abs(got - want).max()


@pytest.mark.parametrize("resp,n_a", [("rotation", 5), ("arms", 4), ("rotation_delay", 12)])
def test_wide_cauchy_schwarz_and_distance(oracle_mod, resp, n_a):
    pt = synth.make_point_wide(3, 4, n_a, 3000, 32768.0, 200.0, 41, response=resp)
    th = synth.prior_samples(3000, 42)
    l = oracle_mod.lnL_wide(pt, th)
    assert l.max() <= pt["half_dd"] * (1 + 1e-9)
    # lnL(x) = K x - R x^2 / 2 exactly: three distances determine the fourth
    t = th[:, :50].copy()
    vals = []
    for dist in (50.0, 100.0, 200.0, 400.0):
        t[6] = dist
        vals.append(oracle_mod.lnL_wide(pt, t))
    x = 100.0 / np.array([50.0, 100.0, 200.0, 400.0])
    L = np.array(vals)
    # fit K, R on the first three, predict the fourth
    Amat = np.stack([x[:3], -0.5 * x[:3] ** 2], axis=1)
    for j in range(50):
        kr = np.linalg.solve(Amat[:2], L[:2, j])
        assert abs(Amat[2] @ kr - L[2, j]) < 1e-9 * (abs(L[:, j]).max() + 1)
        assert abs(np.array([x[3], -0.5 * x[3] ** 2]) @ kr - L[3, j]) < 1e-9 * (abs(L[:, j]).max() + 1)
