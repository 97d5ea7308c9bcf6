"""rift_ile_lnZ_noalloc (the allocation-free variant of rift_ile_lnZ) through
the C ABI: on the same inputs it returns what rift_ile_lnZ returns -- the same
kernels and launch shape, so the same values -- on two calls in a row, the
second with a smaller batch (the fixed scratch keeps the first call's
contents), in FP64 and mixed precision; a request beyond the scratch is
refused before anything is written.  Bar: FP64 lnL and ln Z to 1e-9 relative of
rift_ile_lnZ's (and in fact bitwise equal); mixed ln Z within 1e-3 and bitwise
equal."""
import ctypes

import numpy as np
import pytest

from paper_2609_37393_amd import synth

pytestmark = pytest.mark.gpu

ESCRATCH = -5


@pytest.fixture(scope="module")
def ile():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_37393_amd import ile as m

    lib = m.load()
    vp, i32, ci = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
    lib.rift_ile_lnZ_noalloc.argtypes = [ctypes.POINTER(m.CPoint), i32, vp, vp, vp, vp, vp, vp, ci, vp]
    return m


def _call(ile, fn, pts, counts, th, lnw, prec):
    import torch

    cps = (ile.CPoint * len(pts))(*[p.cstruct() for p in pts])
    c = np.asarray(counts, np.int64)
    N = int(c.sum())
    z = torch.full((len(pts),), 7.0, dtype=torch.float64, device="cuda")
    ne = torch.full((len(pts),), 7.0, dtype=torch.float64, device="cuda")
    ll = torch.full((N,), 7.0, dtype=torch.float64, device="cuda")
    rc = fn(cps, len(pts), c.ctypes.data, th.data_ptr(), None if lnw is None else lnw.data_ptr(), z.data_ptr(),
            ne.data_ptr(), ll.data_ptr(), ile.PRECISIONS[prec], ile._stream(th.device))
    torch.cuda.synchronize()
    return rc, z.cpu().numpy(), ne.cpu().numpy(), ll.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_lnZ_twice_then_smaller(ile, prec):
    import torch

    lib = ile.load()
    big = [ile.DevicePoint.from_dict(p) for p in synth.batched_points(3, 41, K=3, nt_range=(2000, 6554))]
    big_counts = [40000, 25000, 35000]
    small = [ile.DevicePoint.from_dict(synth.make_point(2, 4, 800, 32768.0, 300.0, 42))]
    small_counts = [3000]
    for pts, counts, seed in ((big, big_counts, 43), (small, small_counts, 44)):
        N = sum(counts)
        th = torch.as_tensor(np.concatenate([synth.prior_samples(c, seed + i) for i, c in enumerate(counts)], axis=1),
                             device="cuda").contiguous()
        lnw = torch.as_tensor(np.random.default_rng(seed).normal(0, 1, N), device="cuda").contiguous()
        print(f"noalloc {prec}: {len(pts)} points, {N} samples", flush=True)
        rc0, z0, ne0, l0 = _call(ile, lib.rift_ile_lnZ, pts, counts, th, lnw, prec)
        rc1, z1, ne1, l1 = _call(ile, lib.rift_ile_lnZ_noalloc, pts, counts, th, lnw, prec)
        assert rc0 == 0 and rc1 == 0, (rc0, rc1)
        if prec == "fp64":
            assert np.all(np.abs(l1 - l0) <= 1e-9 * np.maximum(1.0, np.abs(l0)))
            assert np.all(np.abs(z1 - z0) <= 1e-9 * np.maximum(1.0, np.abs(z0)))
            assert np.all(np.abs(ne1 - ne0) <= 1e-9 * ne0)
        else:
            assert np.all(np.abs(z1 - z0) <= 1e-3)
        # same kernels, same launch shape, fixed-order reductions
        assert np.array_equal(z1, z0) and np.array_equal(ne1, ne0) and np.array_equal(l1, l0)


def test_noalloc_refuses_beyond_its_scratch(ile):
    import torch

    lib = ile.load()
    # 5 detectors, 21 modes, 13108 samples per series: ~23 MB of FP64 table per
    # point, so three points exceed the 64 MiB scratch
    p = ile.DevicePoint.from_dict(synth.make_point(5, 21, 13108, 32768.0, 300.0, 45))
    pts, counts = [p, p, p], [100, 100, 100]
    th = torch.as_tensor(synth.prior_samples(300, 46), device="cuda").contiguous()
    rc, z, ne, ll = _call(ile, lib.rift_ile_lnZ_noalloc, pts, counts, th, None, "fp64")
    assert rc == ESCRATCH
    assert np.all(z == 7.0) and np.all(ne == 7.0) and np.all(ll == 7.0)  # nothing written
    assert lib.rift_ile_strerror(ESCRATCH).decode().startswith("request exceeds the fixed scratch")
    # one such point fits, and gives rift_ile_lnZ's result
    rc0, z0, _, l0 = _call(ile, lib.rift_ile_lnZ, [p], [100], th[:, :100].contiguous(), None, "fp64")
    rc1, z1, _, l1 = _call(ile, lib.rift_ile_lnZ_noalloc, [p], [100], th[:, :100].contiguous(), None, "fp64")
    assert rc0 == 0 and rc1 == 0 and np.array_equal(z0, z1) and np.array_equal(l0, l1)
