"""CPU checks of the integer index maps the likelihood kernel's data term is
built on (restated here from their definitions; the GPU parity tests check the
kernel's results):

- the Q table groups W internal modes per padded time row;
- detectors are processed in groups of two or three;
- the cooperative stencil read: lane l = 8 q + c' of read t fetches chunk
  c' ^ key(j) of the 128-byte block of lane j = 8 t + q into LDS at
  t * 1024 + 16 l; lane j reads chunk c at j * 128 + ((c ^ key(j)) << 4).
"""
import itertools

import pytest


def key(j):
    return (j >> 1) & 7


def det_group_size(kt, j):
    n3, r = kt // 3, kt % 3
    if r == 1:
        n3, r = n3 - 1, 4
    if j < n3:
        return 3
    jj = j - n3
    if r == 2:
        return 2 if jj == 0 else 0
    if r == 4:
        return 2 if jj < 2 else 0
    return 0


@pytest.mark.parametrize("kt", [2, 3, 4, 5, 6, 7, 8])
def test_detector_groups_partition(kt):
    sizes = [det_group_size(kt, j) for j in range(4)]
    assert sum(sizes) == kt
    assert all(s in (0, 2, 3) for s in sizes)
    # nonzero groups first, at most three of them
    nz = [s for s in sizes if s]
    assert sizes[: len(nz)] == nz and len(nz) <= 3


@pytest.mark.parametrize("m,w", [(1, 2), (2, 2), (21, 2), (25, 2), (1, 4), (21, 4), (25, 4)])
def test_mode_groups_cover_modes(m, w):
    ng = (m + w - 1) // w
    slots = [(g, s) for g in range(ng) for s in range(w)]
    modes = [g * w + s for g, s in slots if g * w + s < m]
    assert modes == list(range(m))
    assert ng * w - m < w


def test_cooperative_read_lands_where_read():
    lds = {}
    for t, l in itertools.product(range(8), range(64)):
        q, cp = l >> 3, l & 7
        j = 8 * t + q
        # the kernel's form of the key for read t
        assert key(j) == (((t & 1) << 2) | (q >> 1))
        dst = t * 1024 + 16 * l
        assert dst not in lds
        lds[dst] = (j, cp ^ key(j))
    assert len(lds) == 512
    for j in range(64):
        rbase = j * 128 + (key(j) << 4)
        for c in range(8):
            assert lds[rbase ^ (c << 4)] == (j, c)


@pytest.mark.parametrize("lanes_per_pass", [4, 8, 16])
def test_own_block_reads_conflict_free(lanes_per_pass):
    """64 banks of 4 bytes: the 16-byte reads of one pass hit distinct 16-byte
    bank columns."""
    for c in range(8):
        for base in range(0, 64, lanes_per_pass):
            cols = {((j * 128 + ((c ^ key(j)) << 4)) % 256) // 16 for j in range(base, base + lanes_per_pass)}
            assert len(cols) == lanes_per_pass
