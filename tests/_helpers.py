"""Shared test helpers: consistent injections built with the oracle's own
response (the generator itself holds no response arithmetic), and the scale
S_i = |x data| + |x^2 quad| used by the FP64 parity bar."""
import numpy as np

from paper_2609_37393_amd import synth


def response(oracle_mod, pt, th):
    ra, dec, psi, inc, phi, tref, dist = th
    K = pt["Q"].shape[0]
    F = np.zeros(K, complex)
    tk = np.zeros(K)
    for k in range(K):
        F[k], _ = oracle_mod.antenna(pt["det_tensor"][k], ra, dec, psi, pt["gmst"])
        tk[k] = oracle_mod.arrival_time(pt["det_pos"][k], ra, dec, pt["gmst"], tref)
    Y = np.array([oracle_mod.ylm(l, m, inc, phi) for l, m in pt["lm"]])
    return F, tk, Y, pt["d_ref"] / dist


def consistent_point(oracle_mod, K, M, n_t, fs, snr, seed, theta_true, on_node=True, noise=False,
                     lm=None):
    """Injection made with the oracle's response at theta_true (optionally with
    detector positions nudged along N so each t_k lands on a grid node).
    Returns (point, theta_true with the distance the amplitude scaling implies)."""
    net = synth.network(K, seed)
    ra, dec, psi, inc, phi, tref, dist = theta_true
    _, N = oracle_mod.antenna(net["det_tensor"][0], ra, dec, psi, net["gmst"])
    dt = 1.0 / fs
    t0 = -(n_t // 2) * dt
    if on_node:
        for k in range(K):
            tk = tref - net["det_pos"][k] @ N
            node = t0 + dt * round((tk - t0) / dt)
            net["det_pos"][k] = net["det_pos"][k] + (tk - node) * N
    F = np.zeros(K, complex)
    tk = np.zeros(K)
    for k in range(K):
        F[k], _ = oracle_mod.antenna(net["det_tensor"][k], ra, dec, psi, net["gmst"])
        tk[k] = oracle_mod.arrival_time(net["det_pos"][k], ra, dec, net["gmst"], tref)
    modes = synth.modes(M) if lm is None else np.asarray(lm, np.int32)
    Y = np.array([oracle_mod.ylm(l, m, inc, phi) for l, m in modes])
    x = 100.0 / dist
    inj = {"z": x * F[:, None] * Y[None, :], "tk": tk}
    pt = synth.make_point(K, M, n_t, fs, snr, seed, injection=inj, net=net, noise=noise,
                          keep_spectra=True, lm=modes)
    th = np.array(theta_true, dtype=np.float64).copy()
    th[6] = dist / pt["inj_scale"]
    return pt, th


def lnL_scale(oracle_mod, pt, th):
    """S_i = |x K_i| + |x^2 R_i / 2| from lnL(x) = K x - R x^2 / 2 (two extra
    oracle evaluations at x = 1 and x = 2)."""
    t1 = th.copy()
    t1[6] = pt["d_ref"]
    t2 = th.copy()
    t2[6] = pt["d_ref"] / 2.0
    L1 = oracle_mod.lnL(pt, t1)
    L2 = oracle_mod.lnL(pt, t2)
    Kc = (4 * L1 - L2) / 2
    R = 2 * L1 - L2
    x = pt["d_ref"] / th[6]
    return np.abs(Kc * x) + np.abs(R * x * x / 2)
