"""The importance-sampling normalisation through the C ABI (rift_ile_moments,
rift_ile_mixture_is) against the oracle on the same random inputs (Eq.
(sampler-menu:is); the defensive mixture of Sec. "Mode coverage, adaptive
clouds, and evidence").

Bars (written here):
* moments: |d mean_j| <= 1e-12 sum_i W_i |c_ij| and |d cov_jk| <= 1e-12
  sum_i W_i |d_ij d_ik| (the rounding of a weighted sum of n terms, far above
  the sqrt(n) eps of either side's summation order);
* draws: the component exactly wherever u lies more than 1e-14 from every
  selection threshold; the states in the sampler coordinates to 1e-13 (|mu_j|
  + sum_k |L_jk z_k|) for a component draw (the two Cholesky factors differ
  in rounding), 1e-14 (1 + |c_j|) for a prior draw (asin, log), the periodic
  rows compared modulo their period;
* weights: -inf on the same draws (those within 1e-12 of the box's edge left
  out), else |d lnw| <= 1e-11 (1 + |ln p| + |ln q|): the quadratic forms'
  rounding through factors of condition below 1e3; the library keeps the
  images within 9 marginal widths, the oracle every image within 6 periods,
  and the difference is below 1e-18 of the density for draws of the mixture.
"""
import numpy as np
import pytest

from paper_2609_37393_amd import synth

pytestmark = pytest.mark.gpu

BOX = (-0.01, 0.01, 10.0, 1000.0)
PERIODIC = ((0, 2 * np.pi), (2, np.pi), (4, 2 * np.pi))


@pytest.fixture(scope="module")
def ile():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_37393_amd import ile as m

    m.load()
    return m


def _dev(a):
    import torch

    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("n", [1, 7, 1000, 100_003])
@pytest.mark.parametrize("weighted", [False, True])
def test_moments_match_oracle(ile, oracle_mod, n, weighted):
    rng = np.random.default_rng(n + 11 * weighted)
    c = rng.normal(size=(7, n)) * np.array([0.3, 0.1, 0.2, 0.1, 0.5, 0.003, 0.4])[:, None]
    c += np.array([6.1, 0.3, 1.0, -0.2, 3.0, 0.001, 5.5])[:, None]
    lnw = None
    if weighted:
        lnw = rng.normal(size=n) * 3
        if n > 10:
            lnw[::13] = -np.inf
            c[:, ::13] = np.nan  # zero-weight samples are not read
    print(f"moments n={n} weighted={weighted}", flush=True)
    want_m, want_C = oracle_mod.cloud_moments(c, lnw)
    got_m, got_C = ile.moments(_dev(c), None if lnw is None else _dev(lnw))
    got_m, got_C = got_m.cpu().numpy(), got_C.cpu().numpy()
    W = np.full(n, 1.0 / n) if lnw is None else np.exp(lnw - oracle_mod._lse(lnw))
    keep = W > 0
    cs = c[:, keep]
    Wk = W[keep]
    assert np.all(np.abs(got_m - want_m) <= 1e-12 * np.sum(Wk * np.abs(cs), axis=1))
    d = cs - want_m[:, None]
    bar = 1e-12 * np.einsum("i,ji,ki->jk", Wk, np.abs(d), np.abs(d)) + 1e-300
    assert np.all(np.abs(got_C - want_C) <= bar), np.max(np.abs(got_C - want_C) / bar)
    assert np.array_equal(got_C, got_C.T)


def test_moments_edges(ile):
    import torch

    m, C = ile.moments(torch.empty((7, 0), dtype=torch.float64, device="cuda"))
    assert torch.isnan(m).all() and torch.isnan(C).all()
    c = _dev(np.ones((7, 5)))
    m, C = ile.moments(c, _dev(np.full(5, -np.inf)))
    assert torch.isnan(m).all() and torch.isnan(C).all()
    m, C = ile.moments(c, _dev(np.r_[0.0, np.nan, 0.0, 0.0, 0.0]))
    assert torch.isnan(m).all() and torch.isnan(C).all()
    m, C = ile.moments(c)
    assert torch.equal(m, torch.ones(7, dtype=torch.float64, device="cuda")) and not C.any()


def _cov(s, rho=0.0):
    s = np.asarray(s, np.float64)
    R = np.eye(7)
    R[0, 2] = R[2, 0] = rho
    R[1, 6] = R[6, 1] = -rho / 2
    return np.outer(s, s) * R


MIXES = {
    "three": (0.2, [0.5, 0.3, 0.2],
              [[1.0, 0.0, 1.5, 0.2, 3.0, 0.0, 5.5], [1.2, 0.1, 1.5, 0.3, 3.0, 0.0, 5.5],
               [4.0, -0.5, 1.0, -0.5, 1.0, 0.0, 6.0]],
              [_cov([0.15, 0.3, 0.6, 0.15, 1.0, 0.006, 0.8], 0.5)] * 3, 1.5),
    # across the ra boundary, with wide periodic rows (images out to K = 4)
    "wrapped": (0.0, [0.6, 0.4],
                [[6.2, 0.2, 3.0, 0.1, 0.1, 0.0, 5.0], [-0.3, -0.2, 0.2, -0.1, 6.0, 0.002, 6.2]],
                [_cov([0.4, 0.2, 0.7, 0.2, 2.0, 0.004, 0.5], 0.6), _cov([1.2, 0.1, 0.3, 0.3, 0.8, 0.003, 0.3])], 2.0),
    "prior": (1.0, [], [], [], 1.0),
    "half": (0.5, [1.0], [[3.0, 0.4, 2.0, 0.0, 2.0, -0.004, 6.5]], [_cov([0.1, 0.1, 0.1, 0.4, 0.2, 0.005, 0.3], 0.3)],
             3.0),
}


def _run(ile, oracle_mod, name, n, seed, rows=0x7F):
    alpha, a, means, covs, scale = MIXES[name]
    rng = np.random.default_rng(seed)
    z = rng.normal(size=(7, n))
    v = rng.uniform(size=(7, n))
    u = rng.uniform(size=n)
    means = np.asarray(means, np.float64).reshape(len(a), 7)
    covs = np.asarray(covs, np.float64).reshape(len(a), 7, 7)
    th, lnw, comp, status = ile.mixture_is(alpha, a, _dev(means), _dev(covs), scale, BOX, _dev(z), _dev(v), _dev(u),
                                           rows=rows)
    return (alpha, a, means, covs, scale, z, v, u, rows), (th.cpu().numpy(), lnw.cpu().numpy(), comp.cpu().numpy(),
                                                           int(status.cpu().numpy()[0]))


def _compare(oracle_mod, args, got, cols=None):
    alpha, a, means, covs, scale, z, v, u, rows = args
    S = [j for j in range(7) if (rows >> j) & 1]
    th, lnw, comp, status = got
    assert status == 0
    if cols is not None:
        z, v, u = z[:, cols], v[:, cols], u[cols]
        th, lnw, comp = th[:, cols], lnw[cols], comp[cols]
    want_th, want_w, want_comp = oracle_mod.mixture_is(alpha, a, means, covs, scale, *BOX, z, v, u, rows=rows)
    # the selection, where u is firm
    T = alpha + (1.0 - alpha) * np.cumsum(a) if len(a) else np.zeros(0)
    firm = np.all(np.abs(u[:, None] - np.r_[alpha, T][None, :]) > 1e-14, axis=1)
    assert firm.sum() >= u.size - 2
    assert np.array_equal(comp[firm], want_comp[firm])
    same = firm & (comp == want_comp)
    # states in the sampler coordinates
    cg, cw = th.copy(), want_th.copy()
    for c in (cg, cw):
        c[3] = np.cos(c[3])
        c[6] = np.log(c[6])
    bound = np.empty_like(cw)
    pri = want_comp == -1
    bound[:, pri] = 1e-14 * (1 + np.abs(cw[:, pri]))
    for m in range(len(a)):
        sel = want_comp == m
        L = np.linalg.cholesky(scale * covs[m][np.ix_(S, S)])
        bound[:, sel] = 1e-14 * (1 + np.abs(cw[:, sel]))  # the rows left to the prior
        bound[np.ix_(S, sel)] = 1e-13 * (np.abs(means[m][S])[:, None] + np.abs(L) @ np.abs(z[np.ix_(S, sel)])) + 1e-15
    diff = cg - cw
    for j, P in PERIODIC:
        diff[j] -= P * np.round(diff[j] / P)
    inside = np.isfinite(want_w)
    # clamped rows of draws outside the box compare as clamped values
    assert np.all(np.abs(diff[:, same]) <= bound[:, same] + 1e-15), np.max(np.abs(diff[:, same]) / bound[:, same])
    # weights: the box decision away from its edges, then the values
    c_or = cw
    edge = (np.abs(c_or[5] - BOX[0]) < 1e-12) | (np.abs(c_or[5] - BOX[1]) < 1e-12) | \
        (np.abs(c_or[6] - np.log(BOX[2])) < 1e-12) | (np.abs(c_or[6] - np.log(BOX[3])) < 1e-12) | \
        (np.abs(np.abs(c_or[3]) - 1) < 1e-12) | (np.abs(np.abs(c_or[1]) - np.pi / 2) < 1e-12)
    for j, P in PERIODIC:
        edge |= (np.abs(c_or[j]) < 1e-12) | (np.abs(c_or[j] - P) < 1e-12)
    ok = same & ~edge
    assert np.array_equal(np.isneginf(lnw[ok]), np.isneginf(want_w[ok]))
    fin = ok & inside
    lp = oracle_mod.is_log_prior(c_or[:, fin], *BOX, rows=rows)
    lq = lp - want_w[fin]
    bar = 1e-11 * (1 + np.abs(lp) + np.abs(lq))
    err = np.abs(lnw[fin] - want_w[fin])
    assert np.all(err <= bar), np.max(err / bar)
    return inside


@pytest.mark.parametrize("name", list(MIXES))
def test_mixture_is_matches_oracle(ile, oracle_mod, name):
    print(f"mixture {name}", flush=True)
    args, got = _run(ile, oracle_mod, name, 3000, 7 + len(name))
    inside = _compare(oracle_mod, args, got)
    assert inside.mean() > 0.3
    if name == "prior":
        assert np.all(got[1][np.isfinite(got[1])] == 0.0) and np.all(got[2] == -1)


@pytest.mark.parametrize("name,rows", [("three", 0b0101111), ("wrapped", 0b0111011), ("half", 0b1000010)],
                         ids=["three-no-phiref-lnD", "wrapped-no-psi-lnD", "half-dec-lnD"])
def test_mixture_is_over_sampled_rows(ile, oracle_mod, name, rows):
    """The weights of a likelihood marginalised over the rows left out: the
    components sample the masked rows, the others are prior draws."""
    print(f"mixture {name} rows={rows:07b}", flush=True)
    args, got = _run(ile, oracle_mod, name, 3000, 17 + rows)
    _compare(oracle_mod, args, got)


def test_mixture_is_full_size_sampled(ile, oracle_mod):
    """One million draws (the benchmark's size): sampled columns against the
    oracle one by one; the weights' mean is 1 within its sampling error (the
    defensive prior share bounds p / q by 1 / alpha)."""
    args, got = _run(ile, oracle_mod, "three", 1_000_000, 99)
    cols = np.random.default_rng(3).choice(1_000_000, 2000, replace=False)
    _compare(oracle_mod, args, got, cols)
    w = np.exp(got[1])
    assert abs(w.mean() - 1.0) < 5 * w.std() / np.sqrt(w.size)


def test_mixture_refuses_and_edges(ile, oracle_mod):
    import torch

    rng = np.random.default_rng(8)
    n = 100
    z, v, u = _dev(rng.normal(size=(7, n))), _dev(rng.uniform(size=(7, n))), _dev(rng.uniform(size=n))
    good = _cov([0.1, 0.1, 0.1, 0.1, 0.1, 0.001, 0.1])
    mean = np.array([[1.0, 0.0, 1.0, 0.0, 1.0, 0.0, 5.0]] * 2)
    notpd = good.copy()
    notpd[0, 0] = -0.01
    broad = good.copy()
    broad[4, 4] = 3.3 ** 2  # wider than half of phiref's period
    nanm = mean.copy()
    nanm[1, 3] = np.nan
    for covs, means, which in ((np.stack([good, notpd]), mean, 2), (np.stack([broad, good]), mean, 1),
                               (np.stack([good, good]), nanm, 2)):
        print(f"refused component {which}", flush=True)
        th, lnw, comp, st = ile.mixture_is(0.1, [0.5, 0.5], _dev(means), _dev(covs), 1.0, BOX, z, v, u)
        assert int(st.cpu()[0]) == which
        assert torch.isnan(lnw).all() and torch.isnan(th).all()
    # a valid call after a refused one, and n = 0 still reports the status
    th, lnw, comp, st = ile.mixture_is(0.1, [0.5, 0.5], _dev(mean), _dev(np.stack([good, good])), 1.0, BOX, z, v, u)
    assert int(st.cpu()[0]) == 0 and torch.isfinite(th).all()
    e = torch.empty((7, 0), dtype=torch.float64, device="cuda")
    _, _, _, st = ile.mixture_is(0.1, [0.5, 0.5], _dev(mean), _dev(np.stack([good, notpd])), 1.0, BOX, e, e.clone(),
                                 torch.empty(0, dtype=torch.float64, device="cuda"))
    assert int(st.cpu()[0]) == 2
    with pytest.raises(RuntimeError):
        ile.mixture_is(0.1, [0.5, 0.6], _dev(mean), _dev(np.stack([good, good])), 1.0, BOX, z, v, u)


def _kish(t):
    w = np.exp(t - np.max(t))
    return w.sum() ** 2 / np.sum(w * w)


def test_mixture_is_lnZ_end_to_end(ile, oracle_mod):
    """Fit a component to the likelihood's peak from prior draws (moments on
    the device), draw from the defensive mixture on the device, and take ln Z
    through rift_ile_lnZ with the draws' weights: equal to the oracle's ln Z
    on the oracle's draws and weights within the likelihood's FP64 bar, and to
    the prior Monte-Carlo ln Z of 2e6 prior draws within five joint standard
    errors (relative error of each mean about 1 / sqrt(its Kish size)).  At
    SNR 4 the posterior is broad enough for one Gaussian; above that the sky
    is multimodal and a proposal needs a component per mode."""
    pt = synth.make_point(3, 9, 2000, 16384.0, 4.0, 61)
    th_p = synth.prior_samples(2_000_000, 62, tref_s=0.01)
    lp = ile.lnL(pt, th_p).cpu().numpy()
    z_prior, _ = oracle_mod.lnZ(lp)
    best = np.argsort(lp)[-4000:]
    c = th_p[:, best].copy()
    c[3] = np.cos(c[3])
    c[6] = np.log(c[6])
    lw = lp[best] - lp[best].max()
    mean, cov = ile.moments(_dev(c), _dev(lw))
    mean_h, cov_h = mean.cpu().numpy(), cov.cpu().numpy()
    m_or, _ = oracle_mod.cloud_moments(c, lw)
    assert np.all(np.abs(mean_h - m_or) <= 1e-12 * (1 + np.abs(m_or)))
    # keep every periodic width within half its period: C -> D C D
    scale = 1.5
    f = np.ones(7)
    for j, P in PERIODIC:
        f[j] = min(1.0, 0.45 * P / np.sqrt(scale * cov_h[j, j]))
    cov_h = f[:, None] * cov_h * f[None, :]
    n = 200_000
    rng = np.random.default_rng(63)
    z, v, u = rng.normal(size=(7, n)), rng.uniform(size=(7, n)), rng.uniform(size=n)
    th, lnw, comp, st = ile.mixture_is(0.3, [1.0], _dev(mean_h[None]), _dev(cov_h[None]), scale, BOX, _dev(z),
                                       _dev(v), _dev(u))
    assert int(st.cpu()[0]) == 0
    zg, _ = ile.lnZ([pt], th, lnw=lnw)
    zg = float(zg.cpu().numpy()[0])
    want_th, want_w, _ = oracle_mod.mixture_is(0.3, [1.0], mean_h[None], cov_h[None], scale, *BOX, z, v, u)
    l_or = oracle_mod.lnL(pt, want_th)
    z_or, _ = oracle_mod.lnZ(l_or, want_w)
    assert abs(zg - z_or) <= 1e-8 * max(1.0, abs(z_or)), (zg, z_or)
    k_is, k_pr = _kish(l_or + want_w), _kish(lp)
    assert k_is > 300 and k_pr > 300, (k_is, k_pr)
    assert abs(z_or - z_prior) < 5 * np.sqrt(1 / k_is + 1 / k_pr), (z_or, z_prior, k_is, k_pr)


def _kmeans(X, k, iters=50, seed=0):
    rng = np.random.default_rng(seed)
    C = X[rng.choice(len(X), k, replace=False)]
    for _ in range(iters):
        lab = ((X[:, None, :] - C[None]) ** 2).sum(-1).argmin(1)
        for j in range(k):
            if np.any(lab == j):
                C[j] = X[lab == j].mean(0)
    return lab


def test_mixture_is_distance_marginalised_multimode(ile, oracle_mod):
    """SNR 12, the likelihood marginalised over distance in the kernel
    (rift_ile_plan_lnZ_dmarg), and one component per mode: k-means clusters
    of the best pilot draws (host logic, as a sampler's), each fitted by the
    device moments over the six sampled rows.  The IS estimate agrees with
    brute-force prior Monte Carlo of 1e8 draws (drawn by rift_ile_mixture_is
    with alpha = 1) within five joint standard errors, each side's relative
    error about 1 / sqrt(its Kish size)."""
    import torch

    box = BOX
    pt = synth.make_point(3, 9, 2000, 16384.0, 12.0, 61)
    N = 2_000_000
    plan = ile.Plan([pt], [N])
    ll = torch.empty(N, dtype=torch.float64, device="cuda")
    zeros = torch.zeros(N, dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    m_run, s_run, s2_run, pilot = -np.inf, 0.0, 0.0, None
    for it in range(50):
        v = torch.rand((7, N), dtype=torch.float64, device="cuda", generator=gen)
        th, _, _, _ = ile.mixture_is(1.0, [], None, None, 1.0, box, v, v, zeros)
        plan.lnZ_dmarg(th, box[2], box[3], 20, lnL_out=ll)
        lm = float(ll.max())
        w = torch.exp(ll - lm)
        s1, s2 = float(w.sum()), float((w * w).sum())
        m = max(m_run, lm)
        s_run = s_run * np.exp(m_run - m) + s1 * np.exp(lm - m)
        s2_run = s2_run * np.exp(2 * (m_run - m)) + s2 * np.exp(2 * (lm - m))
        m_run = m
        if pilot is None:
            pilot = (th.cpu().numpy(), ll.cpu().numpy())
    z_prior = m_run + np.log(s_run / (50 * N))
    k_prior = s_run ** 2 / s2_run
    thp, lp = pilot
    best = np.argsort(lp)[-8000:]
    c = thp[:, best].copy()
    c[3] = np.cos(c[3])
    c[6] = np.log(c[6])
    lb = lp[best]
    feats = np.stack([np.cos(c[0]) * np.cos(c[1]), np.sin(c[0]) * np.cos(c[1]), np.sin(c[1]), np.cos(c[4]),
                      np.sin(c[4]), np.cos(2 * c[2]), np.sin(2 * c[2]), c[3]], 1)
    lab = _kmeans(feats, 4)
    means, covs, a = [], [], []
    for j in range(4):
        sel = lab == j
        cj = c[:, sel].copy()
        for r, P in PERIODIC:  # unwrap the cluster around its circular mean
            mu = np.arctan2(np.sin(2 * np.pi * cj[r] / P).mean(), np.cos(2 * np.pi * cj[r] / P).mean()) * P / (2 * np.pi)
            cj[r] = mu + ((cj[r] - mu + P / 2) % P) - P / 2
        m, C = ile.moments(_dev(cj), _dev(0.5 * (lb[sel] - lb[sel].max())))
        C = C.cpu().numpy()
        f = np.ones(7)
        for r, P in PERIODIC:
            f[r] = min(1.0, 0.45 * P / np.sqrt(2.0 * C[r, r]))
        means.append(m.cpu().numpy())
        covs.append(f[:, None] * C * f[None, :])
        a.append(np.exp(lb[sel] - lb.max()).sum())
    a = np.array(a) / np.sum(a)
    gen.manual_seed(7)
    z = torch.randn((7, N), dtype=torch.float64, device="cuda", generator=gen)
    v = torch.rand((7, N), dtype=torch.float64, device="cuda", generator=gen)
    u = torch.rand(N, dtype=torch.float64, device="cuda", generator=gen)
    th, lnw, comp, st = ile.mixture_is(0.1, a, _dev(np.array(means)), _dev(np.array(covs)), 2.0, box, z, v, u,
                                       rows=0b0111111)
    assert int(st.cpu()[0]) == 0
    zi, _ = plan.lnZ_dmarg(th, box[2], box[3], 20, lnw=lnw, lnL_out=ll)
    z_is = float(zi.cpu()[0])
    t = (ll + lnw).cpu().numpy()
    t = t[np.isfinite(t)]
    w = np.exp(t - t.max())
    k_is = w.sum() ** 2 / np.sum(w * w)
    plan.close()
    print(f"IS {z_is:.4f} (Kish {k_is:.0f}) prior MC {z_prior:.4f} (Kish {k_prior:.0f})", flush=True)
    assert k_is > 30 and k_prior > 10, (k_is, k_prior)
    assert abs(z_is - z_prior) < 5 * np.sqrt(1 / k_is + 1 / k_prior), (z_is, z_prior, k_is, k_prior)
