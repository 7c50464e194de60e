"""Host model of the batch kernels' tile dealing over the eight XCDs.

Workgroup b of a launch runs on XCD b mod 8; the batch kernels give it tile
number start(x) + b div 8 of the x-th contiguous eighth of the ACTIVE tile
total, or none when b div 8 is past that eighth (the device function
xcd_remap_active in csrc/common.h).  These cases check the formula's
arithmetic: for every grid at or above the total, the numbers handed out
are exactly 0 .. total-1, once each, and every XCD's share differs from the
others' by at most one tile.  The device code's outputs are checked by the
active-subset and bounded-graph tests of the batched path."""
import random

import pytest

XCD = 8


def deal(b, total):
    x, idx = b % XCD, b // XCD
    q, rem = divmod(total, XCD)
    if idx >= q + (1 if x < rem else 0):
        return -1
    return (x * (q + 1) if x < rem else rem * (q + 1) + (x - rem) * q) + idx


def totals():
    rng = random.Random(7)
    return list(range(0, 70)) + [rng.randint(70, 30000) for _ in range(12)]


@pytest.mark.parametrize("total", totals())
def test_dealing_is_a_bijection_onto_the_active_total(total):
    for grid in sorted({total, total + 1, total + 7, total + 8, total + 13, 2 * total + 3,
                        max(total, 1), 5 * total + 11}):
        got = [deal(b, total) for b in range(grid)]
        taken = sorted(g for g in got if g >= 0)
        assert taken == list(range(total)), (total, grid)
        per_xcd = [0] * XCD
        for b in range(grid):
            per_xcd[b % XCD] += got[b] >= 0
        assert max(per_xcd) - min(per_xcd) <= 1
        # each XCD's numbers are contiguous and rise with the dispatch order
        for x in range(XCD):
            mine = [got[b] for b in range(x, grid, XCD) if got[b] >= 0]
            assert mine == list(range(mine[0], mine[0] + len(mine))) if mine else True


def test_full_grid_equals_the_plain_dealing():
    # with no idle workgroups the dealing is the single-frame kernels' one
    for total in (1, 8, 9, 255, 4096, 30001):
        q, rem = divmod(total, XCD)
        for b in range(0, total, max(1, total // 97)):
            x, idx = b % XCD, b // XCD
            plain = (x * (q + 1) if x < rem else rem * (q + 1) + (x - rem) * q) + idx
            assert deal(b, total) == plain
