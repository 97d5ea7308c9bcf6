"""One Metropolis-adjusted HMC transition per chain through the C ABI
(rift_ile_plan_hmc) against the oracle's transition on the same random
inputs (Sec. "Sampling the differentiable extrinsic likelihood").

The chains first take a few oracle transitions so that they sit in the
posterior's bulk, where the energy error H0 - H1 takes both signs; the
uniforms are drawn in (0.8, 1) so that about half of the proposals are
rejected on energy, and one case narrows the time box so that others are
rejected by the prior.

Bars (written here): the accept decision is compared exactly, except for
chains whose ln u lies within 1e-4 of the oracle's H0 - H1 (both sides
decide in FP64 but on energies about 2e3 whose rounding and gradient
differences move them by far less than that); the returned states to
1e-6 sigma_a per coordinate (the oracle's gradient bar of 1e-7 relative,
carried through L kicks of size eps and drifts eps sigma^2, stays below
it at eps L <= 3); lnL to 1e-6 (1 + sum_a sigma_a |dlnL/dc_a|), the
value change that state bar allows, plus the FP64 bar.
"""
import numpy as np
import pytest

from paper_2609_37393_amd import synth

pytestmark = pytest.mark.gpu

SIG = np.array([1e-3, 1e-3, 5e-3, 5e-3, 5e-3, 3e-6, 5e-3])
BOX = (-0.01, 0.01, 10.0, 1000.0)


@pytest.fixture(scope="module")
def ile():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_37393_amd import ile as m

    m.load()
    return m


def _chains(oracle_mod, pt, n, seed, burn=4, eps=0.3, L=8):
    th, _ = synth.weighted_samples(40 * n, seed)
    best = th[:, np.argmax(oracle_mod.lnL(pt, th))]
    c = synth.perturbed_samples(best, SIG, n, seed + 1)
    c[3] = np.cos(c[3])
    c[6] = np.log(c[6])
    rng = np.random.default_rng(seed + 2)
    for _ in range(burn):
        c, _, _ = oracle_mod.hmc_step(pt, c, rng.normal(size=c.shape), rng.uniform(size=n), SIG, eps, L, *BOX)
    return c


def _oracle_dH(oracle_mod, pt, c0, z, eps, L, box):
    p0 = z / SIG[:, None]
    _, U0, _ = oracle_mod.hmc_potential(pt, c0, *box)
    H0 = U0 + 0.5 * np.sum(SIG[:, None] ** 2 * p0 * p0, axis=0)
    _, p, _, U1 = oracle_mod.hmc_trajectory(pt, c0, p0, SIG, eps, L, *box)
    return H0 - (U1 + 0.5 * np.sum(SIG[:, None] ** 2 * p * p, axis=0))


def _to_phys(c):
    t = c.copy()
    t[3] = np.arccos(np.clip(c[3], -1.0, 1.0))
    t[6] = np.exp(c[6])
    return t


def _compare(ile, oracle_mod, pt, plan, point, c0, z, u, eps, L, box):
    import torch

    want_c, want_l, want_acc = oracle_mod.hmc_step(pt, c0, z, u, SIG, eps, L, *box)
    with np.errstate(invalid="ignore"):
        dH = _oracle_dH(oracle_mod, pt, c0, z, eps, L, box)
        firm = ~(np.abs(np.log(u) - dH) < 1e-4)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    tc = dev(c0)
    l, acc = plan.hmc(point, tc, dev(z), dev(u), SIG, eps, L, box)
    got_c, got_l, got_acc = tc.cpu().numpy(), l.cpu().numpy(), acc.cpu().numpy().astype(bool)
    assert np.array_equal(got_acc[firm], want_acc[firm])
    ok = firm
    assert np.all(np.abs(got_c[:, ok] - want_c[:, ok]) <= 1e-6 * SIG[:, None]), \
        np.abs((got_c[:, ok] - want_c[:, ok]) / SIG[:, None]).max()
    _, g = oracle_mod.grad(pt, _to_phys(want_c[:, ok]))
    bar = 1e-6 * (1.0 + np.sum(SIG[:, None] * np.abs(g), axis=0)) + 1e-9 * np.abs(want_l[ok])
    assert np.all(np.abs(got_l[ok] - want_l[ok]) <= bar), np.abs(got_l[ok] - want_l[ok]).max()
    # rejected chains are returned unchanged, bit for bit
    rej = ~got_acc
    assert np.array_equal(got_c[:, rej], c0[:, rej])
    return got_c, got_acc, firm


@pytest.mark.parametrize("eps,L", [(0.3, 8), (0.1, 3), (0.5, 1)])
def test_hmc_matches_oracle(ile, oracle_mod, eps, L):
    pt = synth.make_point(3, 9, 6554, 32768.0, 100.0, 41)
    n = 300
    c0 = _chains(oracle_mod, pt, n, 42)
    rng = np.random.default_rng(int(eps * 100) + L)
    z = rng.normal(size=c0.shape)
    u = rng.uniform(0.8, 1.0, n)
    print(f"hmc eps={eps} L={L} n={n}", flush=True)
    plan = ile.Plan([pt], [n])
    _, acc, firm = _compare(ile, oracle_mod, pt, plan, 0, c0, z, u, eps, L, BOX)
    assert firm.sum() >= n - 3
    if L == 8:
        assert 0.2 < acc.mean() < 0.95, acc.mean()


def test_hmc_prior_box_rejects(ile, oracle_mod):
    """A time box whose upper edge is the proposals' median time: proposals
    beyond it are rejected by the prior and come back unchanged; starts
    beyond it (H0 infinite) take any proposal inside it."""
    pt = synth.make_point(3, 9, 6554, 32768.0, 100.0, 43)
    n = 256
    c0 = _chains(oracle_mod, pt, n, 44)
    rng = np.random.default_rng(5)
    z = rng.normal(size=c0.shape)
    u = rng.uniform(size=n)
    p0 = z / SIG[:, None]
    c1, _, _, _ = oracle_mod.hmc_trajectory(pt, c0, p0, SIG, 0.3, 4, *BOX)
    box = (BOX[0], float(np.median(c1[5])), BOX[2], BOX[3])
    print("hmc box", box, flush=True)
    plan = ile.Plan([pt], [n])
    _, acc, _ = _compare(ile, oracle_mod, pt, plan, 0, c0, z, u, 0.3, 4, box)
    assert 0.1 < acc.mean() < 0.9


def test_hmc_two_points_and_three_transitions(ile, oracle_mod):
    """Chains of the second point of a two-point plan, three transitions in a
    row, each checked against the oracle from the previous HIP state."""
    pts = [synth.make_point(3, 9, 6554, 32768.0, 100.0, 45), synth.make_point(3, 9, 6554, 32768.0, 120.0, 46)]
    n = 200
    c = _chains(oracle_mod, pts[1], n, 47, burn=2)
    plan = ile.Plan(pts, [64, n])
    rng = np.random.default_rng(9)
    for it in range(3):
        z = rng.normal(size=c.shape)
        u = rng.uniform(0.8, 1.0, n)
        print(f"hmc transition {it}", flush=True)
        got_c, _, firm = _compare(ile, oracle_mod, pts[1], plan, 1, c, z, u, 0.3, 8, BOX)
        c = got_c[:, firm]
        n = c.shape[1]


def test_hmc_edge_cases(ile, oracle_mod):
    import torch

    pt = synth.make_point(2, 4, 2000, 16384.0, 50.0, 48)
    plan = ile.Plan([pt], [10])
    empty = torch.empty((7, 0), dtype=torch.float64, device="cuda")
    l, acc = plan.hmc(0, empty, empty.clone(), torch.empty(0, dtype=torch.float64, device="cuda"), SIG, 0.1, 2, BOX)
    assert l.numel() == 0 and acc.numel() == 0
    c0 = _chains(oracle_mod, pt, 10, 49, burn=0)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    z, u = dev(np.zeros((7, 10))), dev(np.full(10, 0.5))
    for bad in (dict(eps=0.0), dict(L=0), dict(sig=np.r_[SIG[:6], 0.0]), dict(box=(0.0, -1.0, 10.0, 1000.0)),
                dict(box=(BOX[0], BOX[1], 0.0, 1000.0)), dict(box=(BOX[0], BOX[1], 10.0, np.inf))):
        with pytest.raises(RuntimeError):
            plan.hmc(0, dev(c0), z, u, bad.get("sig", SIG), bad.get("eps", 0.1), bad.get("L", 2),
                     bad.get("box", BOX))
    # a start outside the distance box (H0 = +inf) and a proposal that stays
    # outside it (H1 = +inf): the same decision as the oracle's
    c_out = c0.copy()
    c_out[6] = np.log(2000.0)
    want_c, _, want_acc = oracle_mod.hmc_step(pt, c_out, np.zeros((7, 10)), np.full(10, 0.5), SIG, 0.1, 2, *BOX)
    tc = dev(c_out)
    _, acc = plan.hmc(0, tc, z, u, SIG, 0.1, 2, BOX)
    assert np.array_equal(acc.cpu().numpy().astype(bool), want_acc)


def _dm_chains(oracle_mod, pt, n, seed, d_box):
    """States near the posterior whose distance peak lies well inside the
    distance prior (the marginal's gradient is the rule's there)."""
    th, _ = synth.weighted_samples(60 * n, seed)
    l = oracle_mod.lnL(pt, th)
    th = th[:, np.argsort(l)[-6 * n:]]
    t1 = th.copy()
    t1[6] = pt["d_ref"]
    K, R = oracle_mod.lnL_terms(pt, t1)
    xs, sg = K / R, 1.0 / np.sqrt(R)
    inner = (xs - 10 * sg > pt["d_ref"] / d_box[1]) & (xs + 10 * sg < pt["d_ref"] / d_box[0])
    th = th[:, inner][:, :n]
    c = th.copy()
    c[3] = np.cos(th[3])
    c[6] = np.log(th[6])
    return c


def test_hmc_and_nuts_on_the_distance_marginal(ile, oracle_mod):
    """rift_ile_plan_hmc_dmarg and rift_ile_plan_nuts_dmarg against
    oracle.hmc_step / nuts_step with dmarg (same bars as the untempered
    transitions; the distance row returned unchanged bit for bit)."""
    import torch

    pt = synth.make_point(3, 9, 2000, 16384.0, 100.0, 91)
    dm = (10.0, 1000.0, 24)
    n = 40
    c0 = _dm_chains(oracle_mod, pt, n, 92, dm)
    assert c0.shape[1] == n
    rng = np.random.default_rng(93)
    z = rng.normal(size=c0.shape)
    u = rng.uniform(0.5, 1.0, n)
    plan = ile.Plan([pt], [n])
    for eps, L, beta in ((0.3, 4, 1.0), (0.2, 6, 0.5)):
        print(f"hmc dmarg eps={eps} L={L} beta={beta}", flush=True)
        want_c, want_l, want_a = oracle_mod.hmc_step(pt, c0, z, u, SIG, eps, L, *BOX, beta=beta, dmarg=dm)
        tc = torch.as_tensor(c0, device="cuda").contiguous()
        l, acc = plan.hmc(0, tc, torch.as_tensor(z, device="cuda").contiguous(),
                          torch.as_tensor(u, device="cuda").contiguous(), SIG, eps, L, BOX, beta=beta, dmarg=dm)
        got_c, got_l, got_a = tc.cpu().numpy(), l.cpu().numpy(), acc.cpu().numpy().astype(bool)
        # energy difference of the oracle, to leave out decisions at the threshold
        p0 = z / SIG[:, None]
        p0[6] = 0.0
        _, U0, _ = oracle_mod.hmc_potential(pt, c0, *BOX, beta=beta, dmarg=dm)
        _, p1, _, U1 = oracle_mod.hmc_trajectory(pt, c0, p0, SIG, eps, L, *BOX, beta=beta, dmarg=dm)
        dH = (U0 + 0.5 * np.sum(SIG[:, None] ** 2 * p0 ** 2, 0)) - (U1 + 0.5 * np.sum(SIG[:, None] ** 2 * p1 ** 2, 0))
        firm = ~(np.abs(np.log(u) - dH) < 1e-4)
        assert firm.sum() >= n - 2
        assert np.array_equal(got_a[firm], want_a[firm])
        assert np.all(np.abs(got_c[:, firm] - want_c[:, firm]) <= 1e-6 * SIG[:, None])
        assert np.array_equal(got_c[6], c0[6])
        _, g = oracle_mod.grad_dmarg(pt, want_c, *dm)
        bar = 1e-6 * (1.0 + np.sum(SIG[:, None] * np.abs(g), axis=0)) + 1e-9 * np.abs(want_l)
        assert np.all(np.abs(got_l[firm] - want_l[firm]) <= bar[firm])
    # NUTS
    D = 4
    dirs, merges = rng.uniform(size=(D, n)), rng.uniform(size=(D, n))
    leaves = rng.uniform(size=(2 ** D - 1, n))
    print("nuts dmarg", flush=True)
    want = oracle_mod.nuts_step(pt, c0, z, dirs, merges, leaves, SIG, 0.3, D, *BOX, dmarg=dm)
    tc = torch.as_tensor(c0, device="cuda").contiguous()
    dev = (lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda"))
    l, info = plan.nuts(0, tc, dev(z), dev(dirs), dev(merges), dev(leaves), SIG, 0.3, D, BOX, dmarg=dm)
    got_c, info = tc.cpu().numpy(), info.cpu().numpy()
    assert np.array_equal(info[0], want[2]) and np.array_equal(info[1], want[3])
    assert np.all(np.abs(got_c - want[0]) <= 1e-6 * SIG[:, None])
    assert np.array_equal(got_c[6], c0[6])
    assert info[1].mean() > 2
    with pytest.raises(RuntimeError):
        plan.hmc(0, dev(c0), dev(z), dev(u), SIG, 0.3, 4, BOX, dmarg=(10.0, 5.0, 24))
    plan.close()
