"""The Fourier refinement of the correlation series on the GPU
(rift_ile_pregrid, Eq. (q-time-pregrid)) against the oracle's FFT
implementation of the same chain (reflect, zero-pad the spectrum with the
Nyquist bin halved, transform back).

Bar (written here): per series, |fine_GPU - fine_oracle| <= 8 n u Lambda max|q|
with u = 2^-53 and Lambda = (2/pi) ln(2n) + 2, the growth bound of a periodic
sinc interpolant (its Lebesgue constant), for the n-term sum of the kernel;
the nodes j = a r must equal q[a] bit for bit (the operator is the identity
there), and r = 1 is the identity."""
import math

import numpy as np
import pytest

from paper_2609_37393_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ile():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2609_37393_amd import ile as m

    m.load()
    return m


def _bar(q, n):
    lam = 2.0 / math.pi * math.log(2 * n) + 2.0
    return 8 * n * 2.0 ** -53 * lam * np.abs(q).max(axis=-1, keepdims=True)


CASES = [(3, 37, 8), (1, 2, 8), (9, 20, 3), (2, 100, 1), (17, 64, 5), (4, 500, 16), (3, 2500, 2), (11, 65, 7)]


@pytest.mark.parametrize("S,n,r", CASES)
def test_pregrid_matches_oracle(ile, oracle_mod, S, n, r):
    rng = np.random.default_rng(S * 1000 + n + r)
    q = rng.normal(size=(S, n)) + 1j * rng.normal(size=(S, n))
    q[0] *= 1e3  # a series on another scale
    got = ile.pregrid(q, r).cpu().numpy()
    want = oracle_mod.pregrid(q, r)
    assert got.shape == want.shape == (S, (n - 1) * r + 1)
    assert np.all(np.abs(got - want) <= _bar(q, n))
    assert np.array_equal(got[:, ::r], q)  # the nodes, exactly


@pytest.mark.parametrize("K,M,n", [(3, 21, 820), (5, 21, 1639)])
def test_pregrid_table_shapes(ile, oracle_mod, K, M, n):
    """The native-rate tables of the headline and the five-detector points
    (4096 Hz, refined x8 to 32768 Hz)."""
    pt = synth.make_point(K, M, n, 4096.0, 600.0, 7 + K)
    q = pt["Q"]
    got = ile.pregrid(q, 8).cpu().numpy()
    want = oracle_mod.pregrid(q, 8)
    assert np.all(np.abs(got - want) <= _bar(q, n)[..., :])
    assert np.array_equal(got[..., ::8], q)


def test_pregrid_identity_and_arguments(ile):
    import torch

    rng = np.random.default_rng(3)
    q = rng.normal(size=(5, 33)) + 1j * rng.normal(size=(5, 33))
    assert np.array_equal(ile.pregrid(q, 1).cpu().numpy(), q)
    lib = ile.load()
    qt = torch.as_tensor(q, device="cuda")
    out = torch.empty((5, 33 * 8), dtype=torch.complex128, device="cuda")
    assert lib.rift_ile_pregrid(qt.data_ptr(), 0, 33, 8, out.data_ptr(), None) == 0
    for n, r in ((1, 8), (33, 0), (33, 65)):
        assert lib.rift_ile_pregrid(qt.data_ptr(), 5, n, r, out.data_ptr(), None) == -1
    assert lib.rift_ile_pregrid(None, 5, 33, 8, out.data_ptr(), None) == -1
