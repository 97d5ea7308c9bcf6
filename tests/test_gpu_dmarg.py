"""The distance-marginalised likelihood on the GPU (rift_ile_plan_lnZ_dmarg,
Eqs. (ap:dexp), (ap:dpeak), (ap:dgh)) against the FP64 oracle on the same
seeded inputs.

Bar (written here): |d ln L_d| <= 1e-9 (S* + 10) per sample, with
S* = |x* K| + |x*^2 R| / 2 = 3 K^2 / 2R the likelihood's own scale at the
peak (the FP64 bar of lnL carried through x* = K/R; the log of the node sum
adds a few times its relative error); -inf and NaN must agree exactly;
ln Z_d within 1e-9 max(1, |ln Z_d|), n_eff to 1e-9 relative."""
import math

import numpy as np
import pytest

from paper_2609_37393_amd import synth

from .test_gpu_parity import CASES, _point

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ile():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_37393_amd import ile as m

    m.load()
    return m


def _bar(oracle_mod, pt, th):
    """Per-sample bar, with NaN marking the samples whose model power R is
    within 1e-9 of the batch's largest: there R is set by rounding (the
    model has no power), and x* = K/R and sigma = R^-1/2 with it, so the
    rule's value is not a property of the method."""
    K, R = oracle_mod.lnL_terms(pt, th)
    with np.errstate(divide="ignore", invalid="ignore"):
        S = np.where((R > 0) & np.isfinite(K), 1.5 * K * K / np.where(R > 0, R, 1.0), 0.0)
    bar = 1e-9 * (S + 10.0)
    rmax = np.nanmax(np.where(np.isfinite(R), R, np.nan))
    bar[np.isfinite(th).all(axis=0) & np.isfinite(R) & (R < 1e-9 * rmax)] = np.nan
    return bar


def _compare(got, want, bar, what):
    cond = ~np.isnan(bar)  # ill-conditioned samples are not compared
    fin = np.isfinite(want) & cond
    assert np.array_equal(np.isnan(got[cond]), np.isnan(want[cond])), what
    inf = np.isinf(want) & cond
    bad = np.where(inf & (got != want))[0]
    assert bad.size == 0, (what, bad[:5], got[bad[:5]], want[bad[:5]])
    d = np.abs(got[fin] - want[fin])
    assert np.all(d <= bar[fin]), (what, (d / bar[fin]).max())
    assert np.all(~np.isnan(got[~cond])), what  # never NaN for a finite sample


@pytest.mark.parametrize("case", CASES, ids=[f"K{c[0]}M{c[1]}nt{c[2]}" for c in CASES])
def test_dmarg_matches_oracle(ile, oracle_mod, case):
    import torch

    pt, th = _point(case)
    print(f"case {case}", flush=True)
    near, lnw_near = synth.weighted_samples(th.shape[1] // 2 + 1, case[6] + 70)
    th = np.concatenate([th, near], axis=1)
    lnw = np.concatenate([np.zeros(th.shape[1] - near.shape[1]), lnw_near])
    n = th.shape[1]
    for d_min, d_max, nodes in ((10.0, 1000.0, 20), (1.0, 5000.0, 7)):
        want = oracle_mod.lnL_dmarg(pt, th, d_min, d_max, nodes)
        z_or, ne_or = oracle_mod.lnZ(want, lnw)
        plan = ile.Plan([pt], [n])
        tht = torch.as_tensor(th, device="cuda").contiguous()
        w = torch.as_tensor(lnw, device="cuda").contiguous()
        ll = torch.empty(n, dtype=torch.float64, device="cuda")
        z, ne = plan.lnZ_dmarg(tht, d_min, d_max, nodes, lnw=w, lnL_out=ll)
        got = ll.cpu().numpy()
        _compare(got, want, _bar(oracle_mod, pt, th), (case, d_min, d_max, nodes))
        assert abs(z.item() - z_or) <= 1e-9 * max(1.0, abs(z_or)), (z.item(), z_or)
        assert abs(ne.item() - ne_or) <= 1e-9 * ne_or
        plan.close()


def test_dmarg_binned_launch_forms_and_distance_row(ile, oracle_mod):
    """Binned and unbinned evaluation, one block per tile and the work queue,
    give bitwise the same ln L_d per sample (and ln Z_d to rounding) over an
    uneven batch; the distance row of theta is not read."""
    import torch

    pts = synth.batched_points(3, 29, K=3, nt_range=(400, 6554))
    counts = [4000, 1, 2500]
    th = np.concatenate([synth.prior_samples(c, 800 + i) for i, c in enumerate(counts)], axis=1)
    tht = torch.as_tensor(th, device="cuda").contiguous()
    plan = ile.Plan(pts, counts)
    res = []
    for cfg in (dict(block=256, tile_blocks=4, blocks_per_cu=0, sort=0), dict(block=128, tile_blocks=2, blocks_per_cu=4, sort=1),
                dict(block=256, tile_blocks=1, blocks_per_cu=2, sort=0)):
        plan.config = cfg
        ll = torch.empty(th.shape[1], dtype=torch.float64, device="cuda")
        z, ne = plan.lnZ_dmarg(tht, 10.0, 1000.0, 16, lnL_out=ll)
        res.append((ll.clone(), z.clone(), ne.clone()))
    for r in res[1:]:
        # per-sample values bit for bit; the reductions follow the tiling (rounding order)
        assert torch.equal(r[0], res[0][0])
        assert torch.allclose(r[1], res[0][1], rtol=1e-12, atol=1e-12) and torch.allclose(r[2], res[0][2], rtol=1e-12)
    th2 = th.copy()
    th2[6] = np.random.default_rng(5).uniform(1, 1e4, th.shape[1])
    ll2 = torch.empty(th.shape[1], dtype=torch.float64, device="cuda")
    plan.lnZ_dmarg(torch.as_tensor(th2, device="cuda").contiguous(), 10.0, 1000.0, 16, lnL_out=ll2)
    assert torch.equal(ll2, res[2][0])
    s = 0
    for p, c in enumerate(counts):
        want = oracle_mod.lnL_dmarg(pts[p], th[:, s:s + c], 10.0, 1000.0, 16)
        _compare(res[0][0][s:s + c].cpu().numpy(), want, _bar(oracle_mod, pts[p], th[:, s:s + c]), p)
        s += c
    plan.close()


def test_dmarg_edges(ile, oracle_mod):
    """Non-finite samples give NaN; a prior box far beyond every peak gives
    -inf (no node inside); bad priors are refused on the host."""
    import torch

    pt, th = _point(CASES[2])
    th = th[:, :200].copy()
    th[5, 3] = np.nan
    th[0, 4] = np.inf
    got = ile.lnL_dmarg(pt, th, 10.0, 1000.0, 20).cpu().numpy()
    want = oracle_mod.lnL_dmarg(pt, th, 10.0, 1000.0, 20)
    assert np.isnan(got[3]) and np.isnan(got[4])
    _compare(got, want, _bar(oracle_mod, pt, th), "edges")
    far = ile.lnL_dmarg(pt, th, 1e40, 2e40, 20).cpu().numpy()
    ok = np.isfinite(th).all(axis=0)
    assert np.all(far[ok] == -np.inf)
    plan = ile.Plan([pt], [th.shape[1]])
    tht = torch.as_tensor(th, device="cuda").contiguous()
    for d_min, d_max, nodes in ((0.0, 10.0, 4), (10.0, 10.0, 4), (10.0, 1e61, 4), (1.0, 10.0, 0), (1.0, 10.0, 65),
                                (float("nan"), 10.0, 4)):
        with pytest.raises(RuntimeError):
            plan.lnZ_dmarg(tht, d_min, d_max, nodes)
    plan.close()


def test_dmarg_full_size_sampled(ile, oracle_mod):
    """The headline batch (3 detectors, 21 modes, SNR 600, 1e6 prior
    samples): sampled ln L_d against the oracle one by one, ln Z_d against the
    oracle's over all samples."""
    import torch

    pt = synth.make_point(3, 21, 6554, 32768.0, 600.0, 2)
    th = synth.prior_samples(1_000_000, 2)
    tht = torch.as_tensor(th, device="cuda").contiguous()
    plan = ile.Plan([pt], [th.shape[1]])
    ll = torch.empty(th.shape[1], dtype=torch.float64, device="cuda")
    z, _ = plan.lnZ_dmarg(tht, 10.0, 1000.0, 20, lnL_out=ll)
    ll = ll.cpu().numpy()
    plan.close()
    idx = np.random.default_rng(7).choice(th.shape[1], 3000, replace=False)
    want = oracle_mod.lnL_dmarg(pt, th[:, idx], 10.0, 1000.0, 20)
    _compare(ll[idx], want, _bar(oracle_mod, pt, th[:, idx]), "c2 sampled")
    allw = oracle_mod.lnL_dmarg(pt, th, 10.0, 1000.0, 20)
    z_or, _ = oracle_mod.lnZ(allw)
    assert abs(z.item() - z_or) <= 1e-9 * max(1.0, abs(z_or))
    assert math.isfinite(z.item())


@pytest.mark.parametrize("snr,d_box,nodes", [(30.0, (10.0, 1000.0), 20), (100.0, (10.0, 1000.0), 32),
                                             (60.0, (50.0, 400.0), 20)])
def test_grad_dmarg_matches_oracle(ile, oracle_mod, snr, d_box, nodes):
    """rift_ile_plan_grad_dmarg against oracle.grad_dmarg on the same states
    (samplers' coordinates).  Bars: ln L_d as above (its K and R come from
    lnL at two distances, K = 2 l1 - l2 / 2 and R = 2 l1 - l2, each with the
    FP64 bar of lnL, ~1e-12 S); the gradient within 1e-8 (|g_a| + 1e-3 |g| +
    |<x>| |dK_a| + |<x^2>| |dR_a|) per row, the rounding of the two-distance
    differences carried through the moments; row 6 exactly 0; -inf with a
    zero gradient where no node lies in the prior."""
    import torch

    pt = synth.make_point(3, 9, 2000, 16384.0, snr, 81)
    th, _ = synth.weighted_samples(4000, 82)
    l = oracle_mod.lnL(pt, th)
    th = th[:, np.argsort(l)[-300:]]
    th = np.concatenate([th, synth.prior_samples(200, 83)], axis=1)
    c = th.copy()
    c[3] = np.cos(th[3])
    c[6] = np.log(th[6])
    n = c.shape[1]
    print(f"grad_dmarg snr={snr} box={d_box} nodes={nodes}", flush=True)
    want_l, want_g = oracle_mod.grad_dmarg(pt, c, *d_box, nodes)
    plan = ile.Plan([pt], [n])
    ld, g = plan.grad_dmarg(0, torch.as_tensor(c, device="cuda").contiguous(), *d_box, nodes)
    ld, g = ld.cpu().numpy(), g.cpu().numpy()
    plan.close()
    assert np.array_equal(np.isneginf(ld), np.isneginf(want_l))
    fin = np.isfinite(want_l)
    bar_l = _bar(oracle_mod, pt, oracle_mod._to_physical(np.where(np.arange(7)[:, None] == 6, np.log(pt["d_ref"]), c)))
    ok = fin & np.isfinite(bar_l)
    assert np.all(np.abs(ld[ok] - want_l[ok]) <= bar_l[ok])
    assert np.all(g[6] == 0.0)
    # the two-distance parts, for the bar
    t1 = oracle_mod._to_physical(c)
    t1[6] = pt["d_ref"]
    t2 = t1.copy()
    t2[6] = pt["d_ref"] / 2
    _, g1 = oracle_mod.grad(pt, t1)
    _, g2 = oracle_mod.grad(pt, t2)
    dK, dR = np.abs(2 * g1 - 0.5 * g2), np.abs(2 * g1 - g2)
    x_hi = pt["d_ref"] / d_box[0]
    norm = np.sqrt(np.sum(want_g[:6] ** 2, axis=0))
    for a in range(6):
        bar = 1e-8 * (np.abs(want_g[a]) + 1e-3 * norm + x_hi * dK[a] + x_hi ** 2 * dR[a])
        assert np.all(np.abs(g[a, ok] - want_g[a, ok]) <= bar[ok]), (a, np.max(np.abs(g[a, ok] - want_g[a, ok]) / bar[ok]))
    empty = np.isneginf(want_l)
    assert np.all(g[:, empty] == 0.0)


def test_grad_dmarg_lane_form_sampled(ile, oracle_mod):
    """A batch above 256 samples per CU runs the lane-per-sample form of the
    marginal gradient (k_grad_dm); sampled columns against the oracle, and
    the group form on the same columns (a batch of those alone) within the
    same bars."""
    import torch

    pt = synth.make_point(3, 9, 2000, 16384.0, 60.0, 85)
    n = 70_000
    th = synth.prior_samples(n, 86)
    near, _ = synth.weighted_samples(4000, 87)
    l = oracle_mod.lnL(pt, near)
    th[:, :300] = near[:, np.argsort(l)[-300:]]
    c = th.copy()
    c[3] = np.cos(th[3])
    c[6] = np.log(th[6])
    d_box, nodes = (10.0, 1000.0), 20
    plan = ile.Plan([pt], [n])
    ld, g = plan.grad_dmarg(0, torch.as_tensor(c, device="cuda").contiguous(), *d_box, nodes)
    ld, g = ld.cpu().numpy(), g.cpu().numpy()
    idx = np.r_[np.arange(300), np.random.default_rng(2).choice(np.arange(300, n), 300, replace=False)]
    cs = c[:, idx]
    want_l, want_g = oracle_mod.grad_dmarg(pt, cs, *d_box, nodes)
    ld2, g2 = plan.grad_dmarg(0, torch.as_tensor(cs, device="cuda").contiguous(), *d_box, nodes)
    ld2, g2 = ld2.cpu().numpy(), g2.cpu().numpy()
    plan.close()
    t1 = oracle_mod._to_physical(cs)
    t1[6] = pt["d_ref"]
    bar_l = _bar(oracle_mod, pt, t1)
    ok = np.isfinite(want_l) & np.isfinite(bar_l)
    assert ok.sum() > 500
    assert np.array_equal(np.isneginf(ld[idx]), np.isneginf(want_l))
    for got_l, got_g in ((ld[idx], g[:, idx]), (ld2, g2)):
        assert np.all(np.abs(got_l[ok] - want_l[ok]) <= bar_l[ok])
        t2 = t1.copy()
        t2[6] = pt["d_ref"] / 2
        _, a1 = oracle_mod.grad(pt, t1)
        _, a2 = oracle_mod.grad(pt, t2)
        dK, dR = np.abs(2 * a1 - 0.5 * a2), np.abs(2 * a1 - a2)
        x_hi = pt["d_ref"] / d_box[0]
        norm = np.sqrt(np.sum(want_g[:6] ** 2, axis=0))
        for a in range(6):
            bar = 1e-8 * (np.abs(want_g[a]) + 1e-3 * norm + x_hi * dK[a] + x_hi ** 2 * dR[a])
            assert np.all(np.abs(got_g[a, ok] - want_g[a, ok]) <= bar[ok]), a
        assert np.all(got_g[6] == 0.0)
