"""The tensor build's line order without a GPU.

The last axis of a 3D build on a box with equal sides takes the lines of the
contiguous axis 0 in the order of c = a1^2 + a2^2, ties by a1 (k_row_order
in csrc/fsa_tensor.hip).  The kernel ranks every line in closed form: the
lines before (a1, a2) are, column by column b1, the b2 with
b2^2 < c - b1^2, which number ceil(sqrt(c - b1^2)), plus the tie
b2^2 = c - b1^2 when b1 < a1.  This restates that count with numpy, with the
kernel's integer square root (an FP32 root corrected in integers), and
checks that it is a permutation that sorts the lines by (c, a1): a count
that missed or doubled a line would leave part of the tensor unwritten.  The
kernel itself runs in the GPU tensor tests (tests/test_gpu_parity.py), whose
cubic boxes take this path.
"""
import numpy as np
import pytest


def isqrt_f32(x):
    """floor(sqrt(x)) for integers 0 <= x < 2^24, as the kernel computes it."""
    s = np.sqrt(x.astype(np.float32)).astype(np.int64)
    s = np.where(s * s > x, s - 1, s)
    s = np.where((s + 1) * (s + 1) <= x, s + 1, s)
    return s


def ranks(d1, d2, a1, a2):
    c = a1 * a1 + a2 * a2
    rank = np.zeros_like(c)
    for b1 in range(d1):
        x = c - b1 * b1
        live = x >= 0
        xs = np.where(live, x, 0)
        s = isqrt_f32(xs)
        square = s * s == xs
        lt = np.where(square, s, s + 1)
        rank += np.where(live, np.minimum(lt, d2), 0)
        rank += np.where(live & square & (b1 < a1) & (s < d2), 1, 0)
    return rank


@pytest.mark.parametrize("d1,d2", [(1, 1), (2, 3), (17, 17), (17, 25), (33, 9), (65, 129),
                                   (257, 257)])
def test_line_ranks_are_a_sorting_permutation(d1, d2):
    r = np.arange(d1 * d2, dtype=np.int64)
    a1, a2 = r % d1, r // d1
    rk = ranks(d1, d2, a1, a2)
    assert np.array_equal(np.sort(rk), r)           # every rank once
    order = np.empty_like(r)
    order[rk] = r                                   # rows[rank] = line
    keys = (a1[order] ** 2 + a2[order] ** 2) * d1 + a1[order]
    assert np.all(np.diff(keys) > 0)                # increasing (c, a1)


def test_line_ranks_at_the_largest_grid_sampled():
    """D = 2049 (N = 2048): sampled lines against a brute-force count over
    every line, in exact integers."""
    d = 2049
    rng = np.random.default_rng(11)
    a1 = rng.integers(0, d, 40)
    a2 = rng.integers(0, d, 40)
    got = ranks(d, d, a1, a2)
    b1, b2 = np.meshgrid(np.arange(d), np.arange(d), indexing="ij")
    cb = b1 * b1 + b2 * b2
    for i in range(len(a1)):
        c = a1[i] ** 2 + a2[i] ** 2
        want = np.count_nonzero(cb < c) + np.count_nonzero((cb == c) & (b1 < a1[i]))
        assert got[i] == want


def test_tiles_of_ordered_lines_span_little_c():
    """What the order buys: 8 consecutive lines of it span c by a few tens
    at 257 x 257, 8 adjacent lines by up to 14 a1."""
    d = 257
    r = np.arange(d * d, dtype=np.int64)
    a1, a2 = r % d, r // d
    order = np.empty_like(r)
    order[ranks(d, d, a1, a2)] = r
    c = a1[order] ** 2 + a2[order] ** 2
    spans = c[7::8][: len(c) // 8] - c[0::8][: len(c) // 8]
    assert np.mean(spans) < 20
