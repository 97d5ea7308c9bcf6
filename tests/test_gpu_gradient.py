"""Gradient of lnL through the C ABI (hand-written adjoint kernels) against the
FP64 oracle's dual-number gradient and against central differences of the
HIP path's own FP64 lnL (Sec. "The differentiable likelihood").

Bars (written here):
  lnL:            |dlnL_i| <= 1e-9 S_i (the FP64 bar)
  vs the oracle:  |dg_a| <= 1e-7 (|g_a| + 1e-6 S_i + 1e-9) per coordinate a
  vs differences: |g_a - fd_a| <= 1e-6 (|g_a| + |fd_a|) + 4 e_i / (2 h_a),
                  e_i = 1e-12 S_i the rounding allowance of one FP64 lnL,
                  steps h = 1e-6 in rad, cos incl and ln dist, 1e-6 dt in tref;
                  samples whose stencil changes cell between the two points
                  are skipped (the cubic is only C0 at the nodes), and so are
                  |cos incl| > 1 - 1e-9.
The oracle returns d/d(cos incl, ln dist) at a sample given as (incl, dist);
the tests move it into the coordinates under test.
"""
import math

import numpy as np
import pytest

from paper_2609_37393_amd import synth

from ._helpers import consistent_point, lnL_scale

pytestmark = pytest.mark.gpu

SIG_C4 = np.array([1e-3, 1e-3, 5e-3, 5e-3, 5e-3, 3e-6, 5e-3])


@pytest.fixture(scope="module")
def ile():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_37393_amd import ile as m

    m.load()
    return m


def to_coords(th, coords):
    """(incl, dist) sample -> rows 3 and 6 in `coords` (bits 1: cos incl, 2: ln dist)."""
    c = th.copy()
    if coords & 1:
        c[3] = np.cos(th[3])
    if coords & 2:
        c[6] = np.log(th[6])
    return c


def from_coords(c, coords):
    th = c.copy()
    if coords & 1:
        th[3] = np.arccos(c[3])
    if coords & 2:
        th[6] = np.exp(c[6])
    return th


def oracle_in(oracle_mod, pt, th, coords):
    """Oracle lnL and gradient in the coordinates `coords` at th = (.., incl, .., dist)."""
    l, g = oracle_mod.grad(pt, th)
    g = g.copy()
    if not coords & 1:
        g[3] = -np.sin(th[3]) * g[3]  # d/d incl = -sin(incl) d/d cos(incl)
    if not coords & 2:
        g[6] = g[6] / th[6]           # d/d dist = d/d ln(dist) / dist
    return l, g


def check_vs_oracle(l, g, l_or, g_or, S, what):
    assert np.all(np.abs(l - l_or) <= 1e-9 * S + 1e-12), what
    for a in range(7):
        rel = np.abs(g[a] - g_or[a]) / (np.abs(g_or[a]) + 1e-6 * S + 1e-9)
        assert rel.max() < 1e-7, (what, a, rel.max())


def c4_point(oracle_mod, seed=61, snr=600.0):
    th0 = np.array([1.3, -0.4, 0.9, 1.1, 2.2, 0.003, 300.0])
    return consistent_point(oracle_mod, 3, 9, 6554, 32768.0, snr, seed, th0, on_node=False, noise=True)


@pytest.mark.parametrize("coords", [0, 1, 2, 3], ids=["incl,dist", "cos,dist", "incl,ln", "cos,ln"])
def test_gradient_matches_oracle(ile, oracle_mod, coords):
    """C4 shape (K=3, 9 modes, SNR 600) at leapfrog-perturbed and prior points,
    in every coordinate system of theta rows 3 and 6."""
    pt, th0 = c4_point(oracle_mod)
    th = np.concatenate([synth.perturbed_samples(th0, SIG_C4, 600, 62), synth.prior_samples(400, 63)], axis=1)
    th[3] = np.clip(th[3], 0.05, np.pi - 0.05)
    c = to_coords(th, coords)
    thb = from_coords(c, coords)  # the point the kernel evaluates
    l, g = ile.grad(pt, c, coords=coords)
    l_or, g_or = oracle_in(oracle_mod, pt, thb, coords)
    check_vs_oracle(l.cpu().numpy(), g.cpu().numpy(), l_or, g_or, lnL_scale(oracle_mod, pt, thb), coords)


def test_gradient_central_differences(ile, oracle_mod):
    """The HIP gradient against central differences of the HIP FP64 lnL at
    leapfrog-perturbed points of the C4 shape, in the sampler's coordinates
    (ra, dec, psi, cos incl, phiref, tref, ln dist), in both kernel forms."""
    import torch

    pt, th0 = c4_point(oracle_mod, seed=64)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    small = synth.perturbed_samples(th0, SIG_C4, 512, 65)
    c_small = to_coords(small, 3)
    big = np.ascontiguousarray(np.tile(c_small, (1, (256 * n_cu) // 512 + 2)))
    S = lnL_scale(oracle_mod, pt, from_coords(c_small, 3))
    steps = np.array([1e-6, 1e-6, 1e-6, 1e-6, 1e-6, 1e-6 * pt["dt"], 1e-6])
    inside = np.abs(c_small[3]) <= 1.0 - 1e-9
    checked = 0
    for form, c in (("group", c_small), ("lane", big)):
        l, g = ile.grad(pt, c, coords=3)
        g = g.cpu().numpy()[:, :512]
        for a, h in enumerate(steps):
            cp, cm = c_small.copy(), c_small.copy()
            cp[a] += h
            cm[a] -= h
            lp, _ = ile.grad(pt, cp, coords=3)
            lm, _ = ile.grad(pt, cm, coords=3)
            fd = (lp.cpu().numpy() - lm.cpu().numpy()) / (2 * h)
            ok = inside.copy()
            if a in (0, 1, 5):  # the stencil must stay in one cell of every detector's table
                tp, tm = from_coords(cp, 3), from_coords(cm, 3)
                for k in range(3):
                    up = [(oracle_mod.arrival_time(pt["det_pos"][k], tp[0, i], tp[1, i], pt["gmst"], tp[5, i])
                           - pt["t0"]) / pt["dt"] for i in range(512)]
                    um = [(oracle_mod.arrival_time(pt["det_pos"][k], tm[0, i], tm[1, i], pt["gmst"], tm[5, i])
                           - pt["t0"]) / pt["dt"] for i in range(512)]
                    ok &= np.floor(up) == np.floor(um)
            tol = 1e-6 * (np.abs(g[a]) + np.abs(fd)) + 4.0 * 1e-12 * S / (2 * h)
            bad = np.abs(g[a] - fd) > tol
            assert not np.any(bad & ok), (form, a, np.abs(g[a] - fd)[ok].max())
            assert ok.sum() > 400, (a, ok.sum())
            checked += ok.sum()
    assert checked > 0


@pytest.mark.parametrize("case", [(2, 2, 410, 4096.0, 20.0, 1), (5, 21, 13108, 32768.0, 1000.0, 5),
                                  (3, 12, 2000, 32768.0, 80.0, 8)], ids=["K2M2", "K5M21", "l8"])
def test_gradient_all_classes(ile, oracle_mod, case):
    """Both gradient forms per detector and mode class: 400 samples alone (16
    lanes per sample) and as the head of a batch large enough for one lane per
    sample."""
    import torch

    from .test_gpu_parity import _mode_set

    K, M, n_t, fs, snr, seed = case
    lm = _mode_set(M, 8) if M == 12 else None
    pt = synth.make_point(K, M, n_t, fs, snr, seed, lm=lm)
    th = synth.prior_samples(400, seed)
    th[3] = np.clip(th[3], 0.05, np.pi - 0.05)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    reps = (256 * n_cu + 1000) // th.shape[1] + 1
    c = to_coords(th, 3)
    thb = from_coords(c, 3)
    big = np.ascontiguousarray(np.tile(c, (1, reps)))
    l_or, g_or = oracle_in(oracle_mod, pt, thb, 3)
    S = lnL_scale(oracle_mod, pt, thb)
    for form, batch in (("group", c), ("lane", big)):
        l, g = ile.grad(pt, batch, coords=3)
        check_vs_oracle(l.cpu().numpy()[:400], g.cpu().numpy()[:, :400], l_or, g_or, S, form)


def test_plan_gradient_lane_and_group_forms(ile, oracle_mod):
    """Through a plan (rift_ile_plan_grad), a batch too small to give every CU
    256 samples runs 16 lanes per sample, a larger one a lane per sample: both
    match the oracle on the same samples."""
    import torch

    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    n_big = 256 * n_cu + 1000
    pt = synth.make_point(3, 9, 6554, 32768.0, 600.0, 3)
    th = synth.prior_samples(n_big, 71)
    th[3] = np.clip(th[3], 0.05, np.pi - 0.05)
    idx = np.linspace(0, n_big - 1, 400).astype(np.int64)
    for coords in (0, 3):
        c = to_coords(th, coords)
        thb = from_coords(c, coords)
        l_or, g_or = oracle_in(oracle_mod, pt, np.ascontiguousarray(thb[:, idx]), coords)
        S = lnL_scale(oracle_mod, pt, np.ascontiguousarray(thb[:, idx]))
        for name, x in (("lane", c), ("group", np.ascontiguousarray(c[:, idx]))):
            n = x.shape[1]
            plan = ile.Plan([pt], [n])
            xt = torch.as_tensor(x, device="cuda").contiguous()
            ll = torch.empty(n, dtype=torch.float64, device="cuda")
            g = plan.grad(0, xt, lnL_out=ll, coords=coords).cpu().numpy()
            ll = ll.cpu().numpy()
            plan.close()
            if name == "lane":
                g, ll = g[:, idx], ll[idx]
            check_vs_oracle(ll, g, l_or, g_or, S, (coords, name))


def test_autograd_function(ile, oracle_mod):
    """LnL (torch.autograd.Function) in the paper's coordinates (incl, ln dist)
    and in the physical ones (incl, dist): backward is grad_out times the
    kernel's gradient."""
    import torch

    pt = synth.make_point(3, 9, 6554, 32768.0, 600.0, 3)
    th = synth.prior_samples(256, 3)
    th[3] = np.clip(th[3], 0.1, np.pi - 0.1)
    dp = ile.DevicePoint.from_dict(pt)
    for coords, name in ((2, "paper"), (0, "physical")):
        c = to_coords(th, coords)
        thb = from_coords(c, coords)
        t = torch.tensor(c, device="cuda", requires_grad=True)
        w = torch.linspace(0.5, 1.5, 256, dtype=torch.float64, device="cuda")
        l = ile.LnL.apply(t, dp, name)
        (l * w).sum().backward()
        l_or, g_or = oracle_in(oracle_mod, pt, thb, coords)
        got = t.grad.cpu().numpy() / w.cpu().numpy()[None, :]
        check_vs_oracle(l.detach().cpu().numpy(), got, l_or, g_or, lnL_scale(oracle_mod, pt, thb), name)


def test_autograd_face_on_and_face_off(ile, oracle_mod):
    """At incl = 0 and pi (face-on, face-off) the incl-derivative is finite:
    the kernel's value equals a central difference of the oracle's lnL in incl
    through the pole (lnL is smooth in incl there)."""
    import torch

    pt = synth.make_point(3, 9, 6554, 32768.0, 600.0, 3)
    th = synth.prior_samples(64, 9)
    dp = ile.DevicePoint.from_dict(pt)
    for pole in (0.0, np.pi):
        th[3] = pole
        c = to_coords(th, 2)
        t = torch.tensor(c, device="cuda", requires_grad=True)
        l = ile.LnL.apply(t, dp, "paper")
        l.sum().backward()
        gi = t.grad.cpu().numpy()[3]
        assert np.all(np.isfinite(gi))
        h = 1e-6
        tp, tm = th.copy(), th.copy()
        tp[3] += h
        tm[3] -= h
        fd = (oracle_mod.lnL(pt, tp) - oracle_mod.lnL(pt, tm)) / (2 * h)
        S = lnL_scale(oracle_mod, pt, th)
        assert np.all(np.abs(gi - fd) <= 1e-6 * np.abs(fd) + 4e-12 * S / (2 * h)), (pole, np.abs(gi - fd).max())


def test_cos_incl_at_and_beyond_the_poles(ile, oracle_mod):
    """cos incl = +-1 is a valid sample (lnL equals the oracle's at incl = 0, pi;
    the cos-incl derivative is not finite there); |cos incl| > 1 is not a point
    of the sky: NaN lnL and gradient, in both kernel forms."""
    import torch

    pt = synth.make_point(3, 9, 6554, 32768.0, 600.0, 3)
    th = synth.prior_samples(8, 10)
    c = to_coords(th, 3)
    c[3, :4] = [1.0, -1.0, 1.0, -1.0]
    c[3, 4:] = [1.0 + 1e-12, -1.0 - 1e-9, 1.5, -7.0]
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    big = np.ascontiguousarray(np.tile(c, (1, (256 * n_cu) // 8 + 2)))
    ref = th[:, :4].copy()
    ref[3] = [0.0, np.pi, 0.0, np.pi]
    l_or = oracle_mod.lnL(pt, ref)
    S = lnL_scale(oracle_mod, pt, ref)
    for form, x in (("group", c), ("lane", big)):
        l, g = ile.grad(pt, x, coords=3)
        l, g = l.cpu().numpy()[:8], g.cpu().numpy()[:, :8]
        assert np.all(np.abs(l[:4] - l_or) <= 1e-9 * S + 1e-12), form
        assert np.all(np.isfinite(g[[0, 1, 2, 4, 5, 6], :4])), form
        assert not np.any(np.isfinite(g[3, :4])), form  # d/d cos(incl) is not finite at the poles
        assert np.all(np.isnan(l[4:])) and np.all(np.isnan(g[:, 4:])), form


def test_far_outside_the_window_reads_zero(ile, oracle_mod):
    """A finite tref whose stencil lies far outside the stored window (|u| up to
    1e20 samples) reads zeros, as the oracle does: lnL = -x^2 quad, and the
    data-term derivatives vanish.  Non-finite tref stays NaN."""
    pt = synth.make_point(2, 2, 410, 4096.0, 20.0, 1)
    th = synth.prior_samples(12, 12)
    th[5] = [1.0, -1.0, 1e3, -1e3, 1e6, -1e9, 2.5e14, -2.5e16, 0.3, -0.2, np.inf, np.nan]
    l, g = ile.grad(pt, th, coords=0)
    l, g = l.cpu().numpy(), g.cpu().numpy()
    l_or, g_or = oracle_in(oracle_mod, pt, th[:, :10], 0)
    S = lnL_scale(oracle_mod, pt, th[:, :10])
    check_vs_oracle(l[:10], g[:, :10], l_or, g_or, S, "far")
    assert np.all(g[5, :10] == 0.0)  # no data term, no time derivative
    assert np.all(np.isnan(l[10:])) and np.all(np.isnan(g[:, 10:]))
    for prec in ("fp64", "fp32"):
        lv, bv = ile.lnL(pt, th, precision=prec, with_bound=True)
        lv, bv = lv.cpu().numpy(), bv.cpu().numpy()
        assert np.all(np.abs(lv[:10] - l_or) <= bv[:10] + 1e-9 * S + 1e-12), prec
        assert np.all(np.isnan(lv[10:])), prec
    assert math.isnan(ile.lnZ([pt], th)[0].item())
