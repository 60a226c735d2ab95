"""Column coverage of the SR solve's vectorised matrix-vector product (host check).

`sr_matvec_kernel` (csrc/sr.hip) gives each wave one row and splits the row's
column range [lo, hi) -- all columns (mode 0), k <= row (mode 1, lower
triangle) or k >= row (mode 2, upper triangle) -- into a head of single
columns up to the first multiple of four, a body read four columns at a time
and a tail of single columns.  This replays that index arithmetic for the 64
lanes of a wave and checks that every column of [lo, hi) is read exactly once,
for unaligned row starts and small n."""
import itertools

import pytest


def _columns(n, row, mode, vec, lanes=64):
    lo = row if mode == 2 else 0
    hi = row + 1 if mode == 1 else n
    seen = []
    k0 = lo
    if vec:
        a = min(hi, (lo + 3) & ~3)
        seen += [lo + lane for lane in range(lanes) if lo + lane < a]          # head
        n4 = (hi - a) >> 2
        for lane in range(lanes):                                               # body
            for q in range(lane, n4, lanes):
                c = a + 4 * q
                seen += [c, c + 1, c + 2, c + 3]
        k0 = a + (n4 << 2)
    for lane in range(lanes):                                                   # tail
        seen += list(range(k0 + lane, hi, lanes))
    return lo, hi, seen


@pytest.mark.parametrize("mode,vec", list(itertools.product((0, 1, 2), (0, 1))))
def test_every_column_once(mode, vec):
    sizes = list(range(1, 10)) + [63, 64, 65, 127, 128, 129, 255, 256, 257, 300, 1000]
    for n in sizes:
        rows = sorted(set(list(range(min(n, 9))) + [n // 2, n - 2, n - 1]) - {-1})
        for row in rows:
            lo, hi, seen = _columns(n, row, mode, vec)
            assert sorted(seen) == list(range(lo, hi)), (n, row, mode, vec)


def test_head_never_exceeds_the_lanes():
    # the head holds at most three columns, so one pass of the 64 lanes covers it
    for lo in range(0, 200):
        a = (lo + 3) & ~3
        assert 0 <= a - lo <= 3
