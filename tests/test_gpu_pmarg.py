"""The likelihood marginalised over polarisation on the GPU
(rift_ile_plan_lnZ_pmarg; Eqs. (ap:psiexp), (ap:psilaplace), (ap:psicells))
against the FP64 oracle.  The kernel takes q(u) from one gather and one
contraction (the complex data term and the two model-norm parts); the oracle
evaluates its own lnL at every angle (trapezoid) or transforms five of them
(Laplace, cells), so the comparison also checks the harmonic decomposition.

Bars (written here): trapezoid, |d ln L_psi| <= 1e-9 max_j S(psi_j) + 1e-12
with S the FP64 bar's scale at each angle of the rule; Laplace and cells, the
same scale at the five angles plus 1e-9 (Laplace: the maximum's curvature A
enters through ln A, whose relative error is that of the coefficients;
cells: the nodes follow the stationary points and curvatures, which move
with the coefficients' rounding, shifting the result by far less than the
rule's own error); NaN must agree; ln Z within 1e-9 max(1, |ln Z|)."""
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


def _bar(oracle_mod, pt, th, n_points, five):
    n = th.shape[1]
    m = 5 if five else n_points
    big = np.repeat(th, m, axis=1)
    big[2] = big[2] + np.tile(np.pi * np.arange(m) / m, n)
    S = lnL_scale(oracle_mod, pt, big).reshape(n, m)
    S = np.where(np.isfinite(S), S, 0.0)
    return 1e-9 * S.max(axis=1) + (1e-9 if five else 1e-12)


def _compare(got, want, bar, what):
    assert np.array_equal(np.isnan(got), np.isnan(want)), what
    fin = np.isfinite(want)
    d = np.abs(got[fin] - want[fin])
    assert np.all(d <= bar[fin]), (what, (d / bar[fin]).max())


@pytest.mark.parametrize("case", CASES[:7], ids=[f"K{c[0]}M{c[1]}nt{c[2]}" for c in CASES[:7]])
def test_pmarg_matches_oracle(ile, oracle_mod, case):
    import torch

    pt, th = _point(case)
    print(f"case {case}", flush=True)
    th = th[:, :500]
    near, lnw_near = synth.weighted_samples(200, case[6] + 110)
    th = np.concatenate([th, near], axis=1)
    lnw = np.concatenate([np.zeros(th.shape[1] - 200), lnw_near])
    n = th.shape[1]
    tht = torch.as_tensor(th, device="cuda").contiguous()
    w = torch.as_tensor(lnw, device="cuda").contiguous()
    for method, n_points in (("trapezoid", 64), ("trapezoid", 7), ("laplace", 0), ("cells", 0)):
        want = oracle_mod.lnL_pmarg(pt, th, method, n_points)
        z_or, ne_or = oracle_mod.lnZ(want, lnw)
        plan = ile.Plan([pt], [n])
        ll = torch.empty(n, dtype=torch.float64, device="cuda")
        z, ne = plan.lnZ_pmarg(tht, method, n_points, lnw=w, lnL_out=ll)
        five = method != "trapezoid"
        _compare(ll.cpu().numpy(), want, _bar(oracle_mod, pt, th, n_points, five), (case, method))
        assert abs(z.item() - z_or) <= 1e-9 * max(1.0, abs(z_or)) + (1e-9 if five else 0.0)
        assert abs(ne.item() - ne_or) <= 1e-8 * ne_or
        plan.close()


def test_pmarg_launch_forms_binning_and_psi_row(ile, oracle_mod):
    import torch

    pts = synth.batched_points(3, 37, K=3, nt_range=(400, 6554))
    counts = [2500, 1, 900]
    th = np.concatenate([synth.prior_samples(c, 950 + i) for i, c in enumerate(counts)], axis=1)
    tht = torch.as_tensor(th, device="cuda").contiguous()
    plan = ile.Plan(pts, counts)
    for method, n_points in (("trapezoid", 32), ("laplace", 0), ("cells", 0)):
        res = []
        for cfg in (dict(block=256, tile_blocks=4, blocks_per_cu=0, sort=0), dict(block=128, tile_blocks=2, blocks_per_cu=4, sort=1),
                    dict(block=64, tile_blocks=1, blocks_per_cu=0, sort=0)):
            plan.config = cfg
            ll = torch.empty(th.shape[1], dtype=torch.float64, device="cuda")
            z, ne = plan.lnZ_pmarg(tht, method, n_points, lnL_out=ll)
            res.append((ll.clone(), z.clone(), ne.clone()))
        for r in res[1:]:
            # per-sample values bit for bit; the reductions follow the tiling (rounding order)
            assert torch.equal(r[0], res[0][0])
            assert torch.allclose(r[1], res[0][1], rtol=1e-12, atol=1e-12)
            assert torch.allclose(r[2], res[0][2], rtol=1e-12)
        s = 0
        for p, c in enumerate(counts):
            want = oracle_mod.lnL_pmarg(pts[p], th[:, s:s + c], method, n_points)
            _compare(res[0][0][s:s + c].cpu().numpy(), want,
                     _bar(oracle_mod, pts[p], th[:, s:s + c], n_points, method != "trapezoid"), (p, method))
            s += c
    # Laplace and cells do not depend on where the points start
    th2 = th.copy()
    th2[2] += np.random.default_rng(4).uniform(0, np.pi, th.shape[1])
    plan.config = dict(block=256, tile_blocks=4, blocks_per_cu=0, sort=0)
    for method in ("laplace", "cells"):
        a = torch.empty(th.shape[1], dtype=torch.float64, device="cuda")
        b = torch.empty(th.shape[1], dtype=torch.float64, device="cuda")
        plan.lnZ_pmarg(tht, method, 0, lnL_out=a)
        plan.lnZ_pmarg(torch.as_tensor(th2, device="cuda").contiguous(), method, 0, lnL_out=b)
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.all(np.abs(a - b) <= 1e-9 * (np.abs(a) + 1.0)), method
    plan.close()


def test_pmarg_edges_and_rules(ile, oracle_mod):
    import torch

    pt, th = _point(CASES[2])
    th = th[:, :200].copy()
    th[0, 3] = np.nan
    th[5, 4] = np.inf
    plan = ile.Plan([pt], [th.shape[1]])
    tht = torch.as_tensor(th, device="cuda").contiguous()
    ll = torch.empty(th.shape[1], dtype=torch.float64, device="cuda")
    plan.lnZ_pmarg(tht, "trapezoid", 16, lnL_out=ll)
    got = ll.cpu().numpy()
    assert np.isnan(got[3]) and np.isnan(got[4])
    _compare(got, oracle_mod.lnL_pmarg(pt, th, "trapezoid", 16), _bar(oracle_mod, pt, th, 16, False), "edges")
    lib = ile.load()
    for rule in ((3, 16), (0, 0), (0, 65537), (-1, 4)):
        with pytest.raises(RuntimeError):
            pr = ile.CPsiRule(*rule)
            ile._check(lib.rift_ile_plan_lnZ_pmarg(plan.handle, tht.data_ptr(), None, pr, ll.data_ptr(), None, None,
                                                   ile._stream(torch.device("cuda"))), "pmarg")
    plan.close()


def test_pmarg_full_size_sampled(ile, oracle_mod):
    """The headline batch (3 detectors, 21 modes, SNR 600, 1e6 samples):
    sampled values one by one, both rules."""
    import torch

    pt = synth.make_point(3, 21, 6554, 32768.0, 600.0, 2)
    th = synth.prior_samples(1_000_000, 2)
    tht = torch.as_tensor(th, device="cuda").contiguous()
    plan = ile.Plan([pt], [th.shape[1]])
    idx = np.random.default_rng(9).choice(th.shape[1], 1000, replace=False)
    for method, n_points in (("trapezoid", 64), ("laplace", 0), ("cells", 0)):
        ll = torch.empty(th.shape[1], dtype=torch.float64, device="cuda")
        z, _ = plan.lnZ_pmarg(tht, method, n_points, lnL_out=ll)
        want = oracle_mod.lnL_pmarg(pt, th[:, idx], method, n_points)
        _compare(ll.cpu().numpy()[idx], want, _bar(oracle_mod, pt, th[:, idx], n_points, method != "trapezoid"),
                 method)
        assert np.isfinite(z.item())
    plan.close()
