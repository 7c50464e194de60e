"""Pins for the oracle's mesh extraction (T, T_map and HE of Sec. 4.2).

The oracle computes T and T_map from their definition (valid triangles of
T_FC ranked in GID order) and HE from the twin definition (the half-edge of
the reversed point pair).  Each check ties it to something other than itself:
the paper's printed triangle counts, the neighbour rules by which Alg. 2
builds HE, a brute-force pair search, closed-form counts, and geometric facts
(winding, twin involution).
"""
import os

import numpy as np
import pytest

from synth import random_grid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.txt")


def full_grid(M, N):
    v, u = np.meshgrid(np.arange(N, dtype=np.float32), np.arange(M, dtype=np.float32))
    return np.stack([v, u, np.ones_like(u)], axis=-1)


def alg2_twins(tri_map, M, N):
    """HE as Alg. 2 builds it from T_map alone (Sec. 4.2): the first triangle
    of quad (u, v) meets the second triangle of its Right (u, v+1) and Top
    (u-1, v) neighbours across its edges 0 and 1, the second triangle meets
    the first triangle of its Left (u, v-1) and Bottom (u+1, v) neighbours
    across its edges 0 and 1, and the two share edge 2 across the cut; a
    neighbour off the grid or missing gives -1.  Vectorised over the quads."""
    Mq, Nq = M - 1, N - 1
    tm = tri_map.reshape(Mq, Nq, 2).astype(np.int64)
    pad = np.full((Mq + 2, Nq + 2, 2), -1, dtype=np.int64)
    pad[1:-1, 1:-1] = tm
    F, S = tm[..., 0], tm[..., 1]
    right = pad[1:-1, 2:, 1]
    top = pad[:-2, 1:-1, 1]
    left = pad[1:-1, :-2, 0]
    bottom = pad[2:, 1:-1, 0]
    n = int((tm >= 0).sum())
    he = np.full(3 * n, -1, dtype=np.int64)

    def link(src, j, dst, k):
        ok = (src >= 0) & (dst >= 0)
        he[3 * src[ok] + j] = 3 * dst[ok] + k

    link(F, 0, right, 0)
    link(F, 1, top, 1)
    link(F, 2, S, 2)
    link(S, 0, left, 0)
    link(S, 1, bottom, 1)
    link(S, 2, F, 2)
    return he.astype(np.int32)


def hashmap_twins(tris):
    """Brute-force form of the twin definition (Sec. 3, Sec. 4.3): key every
    half-edge by its ordered point pair in a dictionary; the twin of (a, b) is
    the half-edge keyed (b, a)."""
    table = {}
    for t, tri in enumerate(tris):
        for j in range(3):
            a, b = int(tri[j]), int(tri[(j + 1) % 3])
            assert (a, b) not in table
            table[(a, b)] = 3 * t + j
    he = np.full(3 * len(tris), -1, dtype=np.int32)
    for (a, b), h in table.items():
        he[h] = table.get((b, a), -1)
    return he


def test_paper_printed_counts(orc):
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert rows
    for M, N, count in rows:
        M, N, count = int(M), int(N), int(count)
        tri_map, tris = orc.mesh(full_grid(M, N))
        assert len(tris) == count
        assert np.array_equal(tri_map, np.arange(count, dtype=np.int32))


@pytest.mark.parametrize("M,N", [(2, 2), (2, 3), (3, 2), (7, 7), (5, 11)])
def test_full_grid_border_halfedges(orc, M, N):
    tri_map, tris = orc.mesh(full_grid(M, N))
    he = orc.halfedges(tri_map, M, N, len(tris))
    assert len(tris) == 2 * (M - 1) * (N - 1)
    assert int((he == -1).sum()) == 2 * (M - 1) + 2 * (N - 1)


def test_7x7_counts(orc):
    tri_map, tris = orc.mesh(full_grid(7, 7))
    he = orc.halfedges(tri_map, 7, 7, len(tris))
    assert len(tris) == 72 and int((he == -1).sum()) == 24


@pytest.mark.parametrize("where,removed", [
    ((3, 4), 6), ((0, 0), 2), ((0, 9), 1), ((6, 0), 1), ((6, 9), 2), ((0, 4), 3), ((3, 0), 3)])
def test_single_nan_removes(orc, where, removed):
    g = full_grid(7, 10)
    g[where] = np.nan
    _, tris = orc.mesh(g)
    assert 2 * 6 * 9 - len(tris) == removed
    flat = where[0] * 10 + where[1]
    assert not np.any(tris == flat)


@pytest.mark.parametrize("seed", range(40))
def test_halfedges_equal_hashmap(orc, seed):
    rng = np.random.default_rng(seed)
    M, N = int(rng.integers(2, 9)), int(rng.integers(2, 9))
    g = random_grid(M, N, seed, nan_frac=float(rng.uniform(0.0, 0.4)))
    tri_map, tris = orc.mesh(g)
    he = orc.halfedges(tri_map, M, N, len(tris))
    assert np.array_equal(he, hashmap_twins(tris))


@pytest.mark.parametrize("seed", range(40))
def test_halfedges_equal_alg2_neighbour_rules(orc, seed):
    """Alg. 2's Right/Top/Left/Bottom links give the same twins as the
    reversed-pair definition the oracle uses."""
    rng = np.random.default_rng(500 + seed)
    M, N = int(rng.integers(2, 12)), int(rng.integers(2, 12))
    g = random_grid(M, N, 500 + seed, nan_frac=float(rng.uniform(0.0, 0.5)))
    tri_map, tris = orc.mesh(g)
    he = orc.halfedges(tri_map, M, N, len(tris))
    assert np.array_equal(he, alg2_twins(tri_map, M, N))


def test_halfedges_alg2_full_and_holed_frames(orc):
    for M, N, nan in ((2, 2, 0.0), (7, 7, 0.0), (31, 47, 0.2), (60, 9, 0.5)):
        g = random_grid(M, N, M * N, nan_frac=nan)
        tri_map, tris = orc.mesh(g)
        he = orc.halfedges(tri_map, M, N, len(tris))
        assert np.array_equal(he, alg2_twins(tri_map, M, N))


@pytest.mark.parametrize("seed", range(5))
def test_halfedges_equal_hashmap_larger(orc, seed):
    g = random_grid(23, 37, 100 + seed, nan_frac=0.25)
    tri_map, tris = orc.mesh(g)
    he = orc.halfedges(tri_map, 23, 37, len(tris))
    assert np.array_equal(he, hashmap_twins(tris))


@pytest.mark.parametrize("seed", range(10))
def test_structure_invariants(orc, seed):
    M, N = 9, 13
    g = random_grid(M, N, 200 + seed, nan_frac=0.3)
    valid = ~np.isnan(g).any(-1)
    tri_map, tris = orc.mesh(g)
    he = orc.halfedges(tri_map, M, N, len(tris))
    # validity from shifted masks (vectorised, a second route to Alg. 1's test)
    p1, p2 = valid[:-1, :-1], valid[:-1, 1:]
    p3, p4 = valid[1:, 1:], valid[1:, :-1]
    expect = np.stack([p1 & p2 & p3, p1 & p3 & p4], axis=-1).reshape(-1)
    assert np.array_equal(tri_map != -1, expect)
    # ranks are consecutive in GID order
    ranks = tri_map[tri_map != -1]
    assert np.array_equal(ranks, np.arange(len(tris)))
    # each triangle uses only valid points and winds counter-clockwise as
    # displayed (negative signed area in (column, row) coordinates)
    cols, rows = tris % N, tris // N
    assert valid.reshape(-1)[tris].all()
    area2 = ((cols[:, 1] - cols[:, 0]) * (rows[:, 2] - rows[:, 0])
             - (cols[:, 2] - cols[:, 0]) * (rows[:, 1] - rows[:, 0]))
    assert np.all(area2 == -1)
    # twins: involution, reversed endpoints
    for h in np.flatnonzero(he != -1):
        t = he[h]
        assert he[t] == h
        a, b = tris[h // 3][h % 3], tris[h // 3][(h % 3 + 1) % 3]
        c, d = tris[t // 3][t % 3], tris[t // 3][(t % 3 + 1) % 3]
        assert (a, b) == (d, c)


def test_first_triangle_halfedge_order(orc):
    # Sec. 4.2: the first triangle's half-edges are p3->p2, p2->p1, p1->p3.
    g = full_grid(2, 2)
    tri_map, tris = orc.mesh(g)
    p1, p2, p3, p4 = 0, 1, 3, 2
    assert tris.tolist() == [[p3, p2, p1], [p1, p4, p3]]


def test_all_nan_and_degenerate_sizes(orc):
    g = np.full((4, 5, 3), np.nan, dtype=np.float32)
    tri_map, tris = orc.mesh(g)
    assert len(tris) == 0 and np.all(tri_map == -1)
    assert orc.halfedges(tri_map, 4, 5, 0).size == 0
