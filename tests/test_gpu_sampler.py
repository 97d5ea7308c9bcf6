"""The leapfrog drift with the reflecting cos-incl boundary through the C ABI
against a NumPy statement of the same update: theta + step p, then
c -> 1 - |((c + 1) mod 4) - 2| for |c| > 1 with p_c negated after an odd
number of folds.  Bar: the product theta + step p may be contracted to one
FMA on the device, so values agree to a few ulps of the operands' scale;
which momenta flip is compared exactly."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _drift_ref(theta, p, step):
    q = theta + step[:, None] * p
    p = p.copy()
    c = q[3]
    out = np.isfinite(c) & (np.abs(c) > 1.0)
    r = np.mod(c[out] + 1.0, 4.0)
    c[out] = 1.0 - np.abs(r - 2.0)
    idx = np.where(out)[0][r > 2.0]
    p[3, idx] = -p[3, idx]
    return q, p


@pytest.mark.parametrize("n", [1, 255, 256, 257, 100_003])
def test_drift_matches_reference(n):
    import torch

    from paper_2609_37393_amd import ile

    rng = np.random.default_rng(n)
    th = rng.normal(size=(7, n))
    th[3] = rng.uniform(-1, 1, n)
    p = rng.normal(size=(7, n)) * 50.0
    p[3, : n // 3] *= 40.0  # pushes a third far past the boundary, some several folds
    step = np.array([1e-3, 2e-3, 3e-3, 0.05, 1e-3, 3e-6, 2e-3])
    if n > 10:
        th[3, :4] = [1.0, -1.0, np.inf, np.nan]
    want_q, want_p = _drift_ref(th, p, step)
    tq = torch.as_tensor(th, device="cuda").contiguous()
    tp = torch.as_tensor(p, device="cuda").contiguous()
    ile.leapfrog_drift(tq, tp, step)
    got_q = tq.cpu().numpy()
    got_p = tp.cpu().numpy()
    fin = np.isfinite(want_q)
    assert np.array_equal(np.isfinite(got_q), fin)
    scale = np.abs(th) + np.abs(step[:, None] * p) + 1.0
    assert np.all(np.abs(got_q[fin] - want_q[fin]) <= 8e-16 * scale[fin])
    assert np.all(np.abs(got_q[3][fin[3]]) <= 1.0)
    # the sign of p_c decides which fold a state sits in: exact
    assert np.array_equal(np.signbit(got_p[3]), np.signbit(want_p[3]))
    assert np.array_equal(np.delete(got_p, 3, axis=0), np.delete(p, 3, axis=0))
