"""The likelihood marginalised over geocentric time by the band-limited
full-window rule on the GPU (rift_ile_plan_lnZ_tband, Eq. (ap:tband)) against
the FP64 oracle.

Bar (written here): |d ln L_t| <= 1e-9 (2 + ln n_t) max_j S(t_j) + 1e-12 per
sample, with S(t_j) = |x data(t_j)| + |x^2 quad| the FP64 bar's scale at each
node: each fine exponent is a sinc-weighted sum of the node values, whose
weights sum in magnitude to at most 2 + ln n_t, plus the remainder, and the
log-sum of values each within a bar stays within the largest.  NaN must
agree.  ln Z_t within the largest per-sample bar (plus 1e-12 relative), n_eff
within four times it, relative (each weight moves by at most that factor).
"""
import numpy as np
import pytest

from paper_2609_37393_amd import synth

from ._helpers import lnL_scale
from .test_gpu_parity import CASES, _point

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ile():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_37393_amd import ile as m

    m.load()
    return m


def _bar(oracle_mod, pt, th, t_start, h, n_t):
    n = th.shape[1]
    big = np.repeat(th, n_t, axis=1)
    big[5] = np.tile(t_start + h * np.arange(n_t), n)
    S = lnL_scale(oracle_mod, pt, big).reshape(n, n_t)
    S = np.where(np.isfinite(S), S, 0.0)
    return 1e-9 * (2.0 + np.log(n_t)) * S.max(axis=1) + 1e-12


def _compare(got, want, bar, what):
    assert np.array_equal(np.isnan(got), np.isnan(want)), what
    fin = np.isfinite(want)
    d = np.abs(got[fin] - want[fin])
    assert np.all(d <= bar[fin]), (what, (d / bar[fin]).max())


# (t_start, h, n_t, n_fine): node counts at and across the register-block
# sizes (16, 32, 64), one fine interval (the trapezoid rule on the nodes) up
# to the largest refinement
RULES = [(-0.004, 1.0 / 8192, 64, 8), (-0.002, 1.0 / 8192, 33, 1), (-0.001, 1.0 / 16384, 17, 64),
         (-0.0005, 1.0 / 8192, 2, 3), (-0.003, 1.0 / 4096, 16, 16)]


@pytest.mark.parametrize("case", CASES[:7], ids=[f"K{c[0]}M{c[1]}nt{c[2]}" for c in CASES[:7]])
def test_tband_matches_oracle(ile, oracle_mod, case):
    import torch

    pt, th = _point(case)
    print(f"case {case}", flush=True)
    th = th[:, :300]
    near, lnw_near = synth.weighted_samples(150, case[6] + 90)
    th = np.concatenate([th, near], axis=1)
    lnw = np.concatenate([np.zeros(th.shape[1] - 150), lnw_near])
    lnw[::37] = -np.inf
    n = th.shape[1]
    plan = ile.Plan([pt], [n])
    tht = torch.as_tensor(th, device="cuda").contiguous()
    w = torch.as_tensor(lnw, device="cuda").contiguous()
    for t_start, h, n_t, M in RULES:
        want = oracle_mod.lnL_tband(pt, th, t_start, h, n_t, M)
        z_or, ne_or = oracle_mod.lnZ(want, lnw)
        ll = torch.empty(n, dtype=torch.float64, device="cuda")
        z, ne = plan.lnZ_tband(tht, t_start, h, n_t, M, lnw=w, lnL_out=ll)
        bar = _bar(oracle_mod, pt, th, t_start, h, n_t)
        _compare(ll.cpu().numpy(), want, bar, (case, n_t, M))
        top = bar[np.isfinite(want)].max()
        assert abs(z.item() - z_or) <= top + 1e-12 * abs(z_or), (z.item(), z_or, n_t, M)
        assert abs(ne.item() - ne_or) <= 4 * top * ne_or + 1e-12
        # without a per-sample output the library keeps its own
        z2, _ = plan.lnZ_tband(tht, t_start, h, n_t, M, lnw=w)
        assert z2.item() == z.item()
    plan.close()


def test_tband_launch_forms_binning_and_time_row(ile, oracle_mod):
    import torch

    pts = synth.batched_points(3, 31, K=3, nt_range=(400, 6554))
    counts = [1500, 1, 700]
    th = np.concatenate([synth.prior_samples(c, 900 + i) for i, c in enumerate(counts)], axis=1)
    tht = torch.as_tensor(th, device="cuda").contiguous()
    plan = ile.Plan(pts, counts)
    rule = (-0.003, 1.0 / 8192, 40, 6)
    res = []
    for cfg in (dict(block=256, tile_blocks=4, blocks_per_cu=0, sort=0), dict(block=128, tile_blocks=2, blocks_per_cu=4, sort=1),
                dict(block=64, tile_blocks=1, blocks_per_cu=0, sort=0)):
        plan.config = cfg
        ll = torch.empty(th.shape[1], dtype=torch.float64, device="cuda")
        z, ne = plan.lnZ_tband(tht, *rule, lnL_out=ll)
        res.append((ll.clone(), z.clone(), ne.clone()))
    for r in res[1:]:
        # per-sample values bit for bit; the reductions follow the tiling (rounding order)
        assert torch.equal(r[0], res[0][0])
        assert torch.allclose(r[1], res[0][1], rtol=1e-12, atol=1e-12) and torch.allclose(r[2], res[0][2], rtol=1e-12)
    th2 = th.copy()
    th2[5] = np.random.default_rng(2).uniform(-1, 1, th.shape[1])
    ll2 = torch.empty(th.shape[1], dtype=torch.float64, device="cuda")
    plan.lnZ_tband(torch.as_tensor(th2, device="cuda").contiguous(), *rule, lnL_out=ll2)
    assert torch.equal(ll2, res[2][0])
    s = 0
    for p, c in enumerate(counts):
        want = oracle_mod.lnL_tband(pts[p], th[:, s:s + c], *rule)
        _compare(res[0][0][s:s + c].cpu().numpy(), want, _bar(oracle_mod, pts[p], th[:, s:s + c], *rule[:3]), p)
        s += c
    plan.close()


def test_tband_edges_and_rules(ile, oracle_mod):
    import torch

    pt, th = _point(CASES[2])
    th = th[:, :300].copy()
    th[0, 3] = np.nan
    th[6, 4] = np.inf  # x = 0: no signal term, finite
    th[2, 5] = np.inf
    plan = ile.Plan([pt], [th.shape[1]])
    tht = torch.as_tensor(th, device="cuda").contiguous()
    ll = torch.empty(th.shape[1], dtype=torch.float64, device="cuda")
    plan.lnZ_tband(tht, -0.004, 0.0002, 41, 5, lnL_out=ll)
    got = ll.cpu().numpy()
    want = oracle_mod.lnL_tband(pt, th, -0.004, 0.0002, 41, 5)
    assert np.isnan(got[3]) and np.isnan(got[5])
    _compare(got, want, _bar(oracle_mod, pt, th, -0.004, 0.0002, 41), "edges")
    for rule in ((0.0, 1e-4, 1, 4), (0.0, 1e-4, 65, 4), (0.0, 1e-4, 8, 0), (0.0, 1e-4, 8, 65), (0.0, 0.0, 8, 4),
                 (0.0, -1e-4, 8, 4), (float("nan"), 1e-4, 8, 4), (0.0, float("inf"), 8, 4)):
        with pytest.raises(RuntimeError):
            plan.lnZ_tband(tht, *rule)
    plan.close()


def test_tband_full_size_sampled(ile, oracle_mod):
    """The headline batch (3 detectors, 21 modes, SNR 600, 1e6 samples) on 33
    nodes at 4096 Hz around the prior's time window centre, 16 fine intervals
    each: sampled values one by one."""
    import torch

    pt = synth.make_point(3, 21, 6554, 32768.0, 600.0, 2)
    th = synth.prior_samples(1_000_000, 2)
    rule = (-0.0039, 1.0 / 4096, 33, 16)
    plan = ile.Plan([pt], [th.shape[1]])
    ll = torch.empty(th.shape[1], dtype=torch.float64, device="cuda")
    z, _ = plan.lnZ_tband(torch.as_tensor(th, device="cuda").contiguous(), *rule, lnL_out=ll)
    ll = ll.cpu().numpy()
    plan.close()
    idx = np.random.default_rng(8).choice(th.shape[1], 1000, replace=False)
    want = oracle_mod.lnL_tband(pt, th[:, idx], *rule)
    _compare(ll[idx], want, _bar(oracle_mod, pt, th[:, idx], *rule[:3]), "c2 sampled")
    assert np.isfinite(z.item())
