"""The measurement's own arithmetic (no GPU): the canonical word count behind the
algorithmic bytes, the bounding box of a launch's states, the expansion kernel filter
and the choice of the counter passes' calibration copies."""
import numpy as np
import pytest

import bench


def key(x, y, z, ia, ie, n):
    return (((z * n + y) * n + x) << 16) | (ia << 8) | ie


def test_canonical_words_against_a_dense_bitset():
    """The words counted are the non-zero 64-bit words of a dense bitset laid out as
    [o][z][y][x/64] (o = ia * na + ie), built state by state."""
    rng = np.random.default_rng(7)
    for n, na in ((20, 6), (70, 4), (130, 3)):
        wpr = (n + 63) // 64
        states = rng.integers(0, [n, n, n, na, na], size=(400, 5))
        keys = np.array([key(*map(int, s), n) for s in states], np.uint64)
        bits = np.zeros(na * na * n * n * wpr * 64, bool)
        for x, y, z, ia, ie in states:
            o = ia * na + ie
            bits[(((o * n + z) * n + y) * wpr) * 64 + x] = True
        words = np.flatnonzero(bits.reshape(-1, 64).any(1))
        assert np.array_equal(bench.canonical_words(keys, n, na), words)


def test_canonical_words_merge_neighbours_in_x():
    n, na = 128, 2
    same = [key(x, 5, 6, 1, 0, n) for x in (0, 1, 63)]     # one word
    other = [key(64, 5, 6, 1, 0, n), key(0, 5, 6, 0, 1, n)]  # next word in x; another orientation
    assert len(bench.canonical_words(np.array(same, np.uint64), n, na)) == 1
    assert len(bench.canonical_words(np.array(same + other, np.uint64), n, na)) == 3


def test_box_of():
    n = 50
    a = np.array([key(3, 4, 5, 0, 0, n), key(10, 2, 7, 1, 1, n)], np.uint64)
    b = np.array([key(1, 9, 6, 0, 2, n)], np.uint64)
    lo, hi = bench.box_of([a, np.array([], np.uint64), b], n)
    assert list(lo) == [1, 2, 5] and list(hi) == [10, 9, 7]
    lo, hi = bench.box_of([np.array([], np.uint64)], n)
    assert hi[0] < 0   # no states: an empty box


@pytest.mark.parametrize("name,expect", [
    ("msc::k_expand_fwd(unsigned long const*, unsigned long, msc::SetView)", True),
    ("void msc::k_expand_bwd<3, true>(unsigned long const*)", True),
    ("void msc::k_expand_bwd<4, false>(unsigned long const*)", True),
    ("msc::k_expand_bwd_set(unsigned long const*, unsigned long)", True),
    ("msc::k_compact(msc::SetView, unsigned long*)", False),
    ("msc::k_meet(unsigned long const*)", False),
    ("msc::k_unexpand_bwd(unsigned long const*)", False),
])
def test_is_expansion(name, expect):
    assert bench.is_expansion(name) == expect


def test_calibration_copies_are_the_largest_grid():
    """The three 1 GiB copies are found by their grid, also when the library's small
    uploads (copies too) come after them."""
    d = [(1, "k_raster", 4096), (4, "__amd_rocclr_copyBuffer", 512), (7, "__amd_rocclr_copyBuffer", 512),
         (10, "__amd_rocclr_copyBuffer", 131072), (11, "__amd_rocclr_copyBuffer", 131072),
         (12, "__amd_rocclr_copyBuffer", 131072), (13, "msc::k_expand_fwd", 65536),
         (20, "__amd_rocclr_copyBuffer", 512), (21, "msc::k_tube_blk", 64)]
    assert bench.calibration_copies(d) == [10, 11, 12]
    with pytest.raises(RuntimeError):
        bench.calibration_copies(d[:5])   # two large copies only
