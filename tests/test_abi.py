"""The C ABI on the CPU: the library loads, exports every entry point that
include/rift_ile.h declares, and its host-side validation rejects bad
arguments before any HIP call (no GPU needed for these paths)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rift_ile.h")
EINVAL = -1
EUNSUPPORTED = -4


@pytest.fixture(scope="module")
def lib():
    from paper_2609_37393_amd import ile

    if not os.path.exists(ile.LIB_PATH):
        from paper_2609_37393_amd import build

        build.build()
    return ile.load()


def test_exports_every_declared_symbol(lib):
    decl = set(re.findall(r"\b(rift_ile_\w+)\s*\(", open(HEADER).read()))
    assert {"rift_ile_lnL", "rift_ile_lnZ", "rift_ile_grad"} <= decl
    for name in sorted(decl):
        assert hasattr(lib, name), name


def test_version_and_strerror(lib):
    assert lib.rift_ile_version() == 2
    assert lib.rift_ile_strerror(0) == b"ok"
    assert lib.rift_ile_strerror(EINVAL) == b"invalid argument"
    assert lib.rift_ile_strerror(-99) == b"unknown status"


def _point(ile, **over):
    lm = np.array([[2, 2], [2, -2]], np.int32)
    D = np.zeros((2, 3, 3))
    R = np.zeros((2, 3))
    keep = (lm, D, R)
    f = dict(n_det=2, n_modes=2, n_t=410, lm=lm.ctypes.data, t0=-0.05, dt=1 / 4096, Q=0x1000,
             U=0x2000, V=0x3000, det_tensor=D.ctypes.data, det_pos=R.ctypes.data, gmst_rad=0.1,
             d_ref=100.0)
    f.update(over)
    return ile.CPoint(**f), keep


BAD = [
    dict(n_det=0), dict(n_det=9), dict(n_modes=0), dict(n_modes=26), dict(n_t=3), dict(n_t=(1 << 26) + 1),
    dict(dt=0.0), dict(dt=-1e-3), dict(dt=float("nan")), dict(t0=float("inf")),
    dict(d_ref=0.0), dict(gmst_rad=float("nan")), dict(Q=None), dict(U=None), dict(V=None),
    dict(lm=None), dict(det_tensor=None), dict(det_pos=None), dict(Q=0x1004),
]


@pytest.mark.parametrize("over", BAD)
def test_invalid_point_rejected_on_host(lib, over):
    from paper_2609_37393_amd import ile

    cp, keep = _point(ile, **over)
    assert lib.rift_ile_lnL(ctypes.byref(cp), 10, 0x4000, 0x5000, None, 0, None) == EINVAL
    assert lib.rift_ile_grad(ctypes.byref(cp), 10, 0x4000, 0, 0x5000, 0x6000, 0, None) == EINVAL
    n = np.array([10], np.int64)
    assert lib.rift_ile_lnZ(ctypes.byref(cp), 1, n.ctypes.data, 0x4000, None, 0x5000, None, None, 0,
                            None) == EINVAL


@pytest.mark.parametrize("lm", [[[1, 0], [2, 2]], [[2, 3], [2, 2]], [[9, 0], [2, 2]], [[2, 2], [2, 2]]])
def test_invalid_modes_rejected(lib, lm):
    from paper_2609_37393_amd import ile

    arr = np.array(lm, np.int32)
    cp, keep = _point(ile, lm=arr.ctypes.data)
    assert lib.rift_ile_lnL(ctypes.byref(cp), 10, 0x4000, 0x5000, None, 0, None) == EINVAL


def test_invalid_detector_geometry_rejected(lib):
    from paper_2609_37393_amd import ile

    D = np.zeros((2, 3, 3))
    D[1, 0, 0] = np.nan
    cp, keep = _point(ile, det_tensor=D.ctypes.data)
    assert lib.rift_ile_lnL(ctypes.byref(cp), 10, 0x4000, 0x5000, None, 0, None) == EINVAL


def test_invalid_call_arguments_rejected(lib):
    from paper_2609_37393_amd import ile

    cp, keep = _point(ile)
    # negative n, null or misaligned sample / output pointers, bad precision
    assert lib.rift_ile_lnL(ctypes.byref(cp), -1, 0x4000, 0x5000, None, 0, None) == EINVAL
    assert lib.rift_ile_lnL(ctypes.byref(cp), 10, None, 0x5000, None, 0, None) == EINVAL
    assert lib.rift_ile_lnL(ctypes.byref(cp), 10, 0x4000, None, None, 0, None) == EINVAL
    assert lib.rift_ile_lnL(ctypes.byref(cp), 10, 0x4001, 0x5000, None, 0, None) == EINVAL
    assert lib.rift_ile_lnL(ctypes.byref(cp), 10, 0x4000, 0x5000, 0x6004, 0, None) == EINVAL
    assert lib.rift_ile_lnL(ctypes.byref(cp), 10, 0x4000, 0x5000, None, 3, None) == EINVAL
    assert lib.rift_ile_grad(ctypes.byref(cp), 10, 0x4000, 0, 0x5000, None, 0, None) == EINVAL
    assert lib.rift_ile_grad(ctypes.byref(cp), 10, 0x4000, 4, 0x5000, 0x6000, 0, None) == EINVAL
    assert lib.rift_ile_grad(ctypes.byref(cp), 10, 0x4000, -1, 0x5000, 0x6000, 0, None) == EINVAL
    # the gradient is FP64 only: a valid request this library does not implement
    assert lib.rift_ile_grad(ctypes.byref(cp), 10, 0x4000, 0, 0x5000, 0x6000, 1, None) == EUNSUPPORTED
    assert lib.rift_ile_grad(ctypes.byref(cp), 10, 0x4000, 0, 0x5000, 0x6000, 2, None) == EUNSUPPORTED
    # RIFT_FP32 is an rift_ile_lnL-only precision
    n1 = np.array([10], np.int64)
    assert lib.rift_ile_lnZ(ctypes.byref(cp), 1, n1.ctypes.data, 0x4000, None, 0x5000, None, None, 2,
                            None) == EINVAL
    n = np.array([10], np.int64)
    assert lib.rift_ile_lnZ(ctypes.byref(cp), 0, n.ctypes.data, 0x4000, None, 0x5000, None, None, 0,
                            None) == EINVAL
    assert lib.rift_ile_lnZ(ctypes.byref(cp), 1, None, 0x4000, None, 0x5000, None, None, 0,
                            None) == EINVAL
    n0 = np.array([0], np.int64)
    assert lib.rift_ile_lnZ(ctypes.byref(cp), 1, n0.ctypes.data, 0x4000, None, 0x5000, None, None, 0,
                            None) == EINVAL
    h = ctypes.c_void_p()
    assert lib.rift_ile_plan_create(ctypes.byref(cp), 1, n.ctypes.data, 7, None, ctypes.byref(h)) == EINVAL
    assert lib.rift_ile_plan_destroy(None) == EINVAL
    assert lib.rift_ile_plan_lnZ(None, 0x4000, None, 0x5000, None, None, None, None, None) == EINVAL
    assert lib.rift_ile_plan_grad(None, 0, 1, 0x4000, 0, None, 0x5000, None) == EINVAL


def test_zero_samples_is_a_validated_noop(lib):
    from paper_2609_37393_amd import ile

    cp, keep = _point(ile)
    assert lib.rift_ile_lnL(ctypes.byref(cp), 0, None, None, None, 0, None) == 0
    bad, keep2 = _point(ile, n_det=0)
    assert lib.rift_ile_lnL(ctypes.byref(bad), 0, None, None, None, 0, None) == EINVAL


def test_product_path_has_no_oracle_dependency():
    """The package never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2609_37393_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "liboracle" not in txt, f


def _point_wide(ile, **over):
    lm = np.array([[2, 2], [2, -2]], np.int32)
    D = np.zeros((2, 3, 3))
    R = np.zeros((2, 3))
    A = np.zeros((2, 2, 3))
    keep = (lm, D, R, A)
    f = dict(n_det=2, n_modes=2, n_t=410, lm=lm.ctypes.data, t0=-0.05, dt=1 / 4096, response=1, n_terms=5,
             Q=0x1000, U=0x2000, V=0x3000, det_tensor=D.ctypes.data, det_pos=R.ctypes.data,
             det_arms=A.ctypes.data, gmst_rad=0.1, omega=7.292115e-5, d_ref=100.0)
    f.update(over)
    return ile.CPointWide(**f), keep


BAD_WIDE = BAD + [
    dict(response=0), dict(response=4), dict(n_terms=4), dict(omega=float("nan")),
    dict(response=3, n_terms=7), dict(response=3, n_terms=32), dict(response=3, omega=float("inf")),
    dict(response=2, n_terms=9),
    dict(response=2, n_terms=0), dict(response=2, n_terms=33), dict(response=2, det_arms=None),
]


@pytest.mark.parametrize("over", BAD_WIDE)
def test_invalid_wide_point_rejected_on_host(lib, over):
    from paper_2609_37393_amd import ile

    cp, keep = _point_wide(ile, **over)
    assert lib.rift_ile_wide_lnL(ctypes.byref(cp), 0, None, None, None) == EINVAL
    assert lib.rift_ile_wide_lnZ(ctypes.byref(cp), 10, 0x4000, None, 0x5000, None, None, None) == EINVAL


def test_wide_call_arguments(lib):
    from paper_2609_37393_amd import ile

    cp, keep = _point_wide(ile)
    assert lib.rift_ile_wide_lnL(ctypes.byref(cp), 0, None, None, None) == 0
    cp2, keep2 = _point_wide(ile, response=2, n_terms=4)
    assert lib.rift_ile_wide_lnL(ctypes.byref(cp2), 0, None, None, None) == 0
    assert lib.rift_ile_wide_lnL(ctypes.byref(cp), -1, 0x4000, 0x5000, None) == EINVAL
    assert lib.rift_ile_wide_lnL(ctypes.byref(cp), 10, None, 0x5000, None) == EINVAL
    assert lib.rift_ile_wide_lnL(ctypes.byref(cp), 10, 0x4000, None, None) == EINVAL
    assert lib.rift_ile_wide_lnL(ctypes.byref(cp), 10, 0x4004, 0x5000, None) == EINVAL
    # ln Z of no samples is undefined; a null ln Z output is refused
    assert lib.rift_ile_wide_lnZ(ctypes.byref(cp), 0, 0x4000, None, 0x5000, None, None, None) == EINVAL
    assert lib.rift_ile_wide_lnZ(ctypes.byref(cp), 10, 0x4000, None, None, None, None, None) == EINVAL


def test_leapfrog_drift_arguments(lib):
    step = np.full(7, 1e-3)
    s = step.ctypes.data
    assert lib.rift_ile_leapfrog_drift(0, None, None, s, None) == 0
    assert lib.rift_ile_leapfrog_drift(-1, 0x4000, 0x5000, s, None) == EINVAL
    assert lib.rift_ile_leapfrog_drift(10, 0x4000, 0x5000, None, None) == EINVAL
    assert lib.rift_ile_leapfrog_drift(10, None, 0x5000, s, None) == EINVAL
    assert lib.rift_ile_leapfrog_drift(10, 0x4000, 0x5004, s, None) == EINVAL
    bad = step.copy()
    bad[3] = np.inf
    assert lib.rift_ile_leapfrog_drift(10, 0x4000, 0x5000, bad.ctypes.data, None) == EINVAL


def test_hmc_arguments(lib):
    """The HMC transition validates its host arguments before any device
    work; n = 0 is a validated no-op (the plan is not touched then)."""
    from paper_2609_37393_amd import ile

    sig = np.array([1e-3, 1e-3, 5e-3, 5e-3, 5e-3, 3e-6, 5e-3])
    box = ile.CHmcPrior(-0.01, 0.01, 10.0, 1000.0)
    fake = 0x1000  # never dereferenced on these paths

    def call(plan=fake, n=0, sigma=sig, eps=0.1, L=4, prior=box):
        return lib.rift_ile_plan_hmc(plan, 0, n, None, None, None, None if sigma is None else sigma.ctypes.data,
                                     eps, L, None if prior is None else ctypes.byref(prior), None, None, None)

    assert call() == 0
    assert call(plan=None) == EINVAL
    assert call(n=-1) == EINVAL
    assert call(sigma=None) == EINVAL
    assert call(prior=None) == EINVAL
    assert call(eps=0.0) == EINVAL and call(eps=float("nan")) == EINVAL
    assert call(L=0) == EINVAL and call(L=10001) == EINVAL
    assert call(sigma=np.r_[sig[:5], -1.0, sig[6]]) == EINVAL
    assert call(prior=ile.CHmcPrior(0.01, -0.01, 10.0, 1000.0)) == EINVAL
    assert call(prior=ile.CHmcPrior(-0.01, 0.01, 0.0, 1000.0)) == EINVAL
    assert call(prior=ile.CHmcPrior(-0.01, 0.01, 10.0, float("inf"))) == EINVAL
    assert call(n=10) == EINVAL  # null state and random-number pointers


def test_importance_arguments(lib):
    """The moments and the mixture draws validate their host arguments before
    any device work."""
    from paper_2609_37393_amd import ile

    fake = 0x1000  # never dereferenced on these paths
    assert lib.rift_ile_moments(-1, fake, None, fake, fake, None) == EINVAL
    assert lib.rift_ile_moments(10, None, None, fake, fake, None) == EINVAL
    assert lib.rift_ile_moments(10, fake, None, None, fake, None) == EINVAL
    assert lib.rift_ile_moments(10, fake, 0x1004, fake, fake, None) == EINVAL
    box = ile.CHmcPrior(-0.01, 0.01, 10.0, 1000.0)
    a = np.array([0.25, 0.75])

    def call(n=4, nc=2, alpha=0.1, scale=1.5, w=a, prior=box, z=fake, comp=None, status=None, rows=0x7F):
        mix = ile.CMixture(nc, alpha, scale, None if w is None else w.ctypes.data, fake, fake, rows)
        return lib.rift_ile_mixture_is(n, ctypes.byref(mix), None if prior is None else ctypes.byref(prior), z, fake,
                                       fake, fake, fake, comp, status, None)

    assert call(n=-1) == EINVAL
    assert call(nc=-1) == EINVAL and call(nc=33) == EINVAL
    assert call(nc=0, alpha=0.5) == EINVAL
    assert call(alpha=-0.1) == EINVAL and call(alpha=1.5) == EINVAL and call(alpha=float("nan")) == EINVAL
    assert call(scale=0.0) == EINVAL and call(scale=float("inf")) == EINVAL
    assert call(w=None) == EINVAL
    assert call(w=np.array([0.25, 0.7])) == EINVAL  # not summing to 1
    assert call(w=np.array([0.0, 1.0])) == EINVAL  # a component of zero weight
    assert call(prior=None) == EINVAL
    assert call(prior=ile.CHmcPrior(0.01, -0.01, 10.0, 1000.0)) == EINVAL
    assert call(prior=ile.CHmcPrior(-0.01, 0.01, 0.0, 1000.0)) == EINVAL
    assert call(z=None) == EINVAL and call(z=0x1004) == EINVAL
    assert call(comp=0x1002) == EINVAL and call(status=0x1001) == EINVAL
    assert call(rows=0) == EINVAL and call(rows=0x80) == EINVAL
    assert lib.rift_ile_mixture_is(4, None, ctypes.byref(box), fake, fake, fake, fake, fake, None, None, None) \
        == EINVAL


def test_rwm_arguments(lib):
    from paper_2609_37393_amd import ile

    box = ile.CHmcPrior(-0.01, 0.01, 10.0, 1000.0)
    fake = 0x1000  # never dereferenced on these paths

    def call(plan=fake, n=4, cov=fake, scale=0.5, prior=box, beta=1.0, lnL=fake, acc=None, status=None):
        return lib.rift_ile_plan_rwm(plan, 0, n, fake, fake, fake, cov, scale,
                                     None if prior is None else ctypes.byref(prior), beta, lnL, acc, status, None)

    assert call(plan=None) == EINVAL and call(n=-1) == EINVAL and call(cov=None) == EINVAL
    assert call(scale=0.0) == EINVAL and call(scale=float("nan")) == EINVAL
    assert call(beta=-0.5) == EINVAL and call(beta=2.0) == EINVAL and call(prior=None) == EINVAL
    assert call(prior=ile.CHmcPrior(0.01, -0.01, 10.0, 1000.0)) == EINVAL
    assert call(lnL=None) == EINVAL and call(acc=0x1002) == EINVAL and call(status=0x1001) == EINVAL


def test_tband_null_plan(lib):
    from paper_2609_37393_amd import ile

    rule = ile.CBandRule(-0.004, 1.0 / 8192, 64, 8)
    assert lib.rift_ile_plan_lnZ_tband(None, 0x4000, None, ctypes.byref(rule), 0x5000, None, None, None) == EINVAL
    assert lib.rift_ile_plan_lnZ_tband(0x1000, 0x4000, None, None, 0x5000, None, None, None) == EINVAL


def test_erai_null_plan(lib):
    from paper_2609_37393_amd import ile

    rule = ile.CAngleRule(32, 16)
    assert lib.rift_ile_plan_lnZ_erai(None, 0x4000, None, ctypes.byref(rule), 0x5000, None, None, None) == EINVAL
    assert lib.rift_ile_plan_lnZ_erai(0x1000, 0x4000, None, None, 0x5000, None, None, None) == EINVAL


def test_wide_rotation_rate_limit(lib):
    """Under rotation the turn over the light-travel time, |omega| |r_k|, must
    stay within one radian."""
    from paper_2609_37393_amd import ile

    R = np.array([[0.02, 0.0, 0.0], [0.0, -0.01, 0.0]])
    ok, keep = _point_wide(ile, det_pos=R.ctypes.data, omega=40.0)
    assert lib.rift_ile_wide_lnL(ctypes.byref(ok), 0, None, None, None) == 0
    bad, keep2 = _point_wide(ile, det_pos=R.ctypes.data, omega=60.0)
    assert lib.rift_ile_wide_lnL(ctypes.byref(bad), 0, None, None, None) == EINVAL
    # the arms response has no rotation
    arms, keep3 = _point_wide(ile, det_pos=R.ctypes.data, omega=60.0, response=2, n_terms=3)
    assert lib.rift_ile_wide_lnL(ctypes.byref(arms), 0, None, None, None) == 0
