"""Pins for the oracle's user-mesh half-edges (Sec. 4.3, option 1 for edges
shared by more than two triangles): Alg. 2 on organized meshes (which are
two-manifold), hand-worked non-manifold cases, and a quadratic search
written with plain loops on small random soups."""
import numpy as np
import pytest

from synth import random_grid


def quadratic(tris):
    """For each half-edge: if an earlier one has the same (a, b), no twin;
    else the earliest half-edge (b, a), if any.  a == b: no twin."""
    he = []
    edges = [(int(t[j]), int(t[(j + 1) % 3])) for t in tris for j in range(3)]
    for h, (a, b) in enumerate(edges):
        if a == b or any(edges[g] == (a, b) for g in range(h)):
            he.append(-1)
            continue
        he.append(next((g for g, e in enumerate(edges) if e == (b, a)), -1))
    return np.array(he, dtype=np.int32)


@pytest.mark.parametrize("seed", range(12))
def test_equals_alg2_on_organized_meshes(orc, seed):
    rng = np.random.default_rng(seed)
    M, N = int(rng.integers(2, 30)), int(rng.integers(2, 30))
    g = random_grid(M, N, 300 + seed, nan_frac=float(rng.uniform(0.0, 0.4)))
    tri_map, tris = orc.mesh(g)
    assert np.array_equal(orc.user_halfedges(tris), orc.halfedges(tri_map, M, N, len(tris)))


def test_hand_worked_non_manifold(orc):
    # T0 and T1 share 0-1 with opposite orientations; T2 is a third triangle
    # on that edge (1 -> 0 again); T3 repeats T0's orientation (0 -> 1)
    tris = np.array([[0, 1, 2], [1, 0, 3], [1, 0, 4], [0, 1, 5]])
    he = orc.user_halfedges(tris)
    want = np.full(12, -1)
    want[0], want[3] = 3, 0
    assert he.tolist() == want.tolist()
    # a degenerate triangle: no half-edge from a point to itself has a twin;
    # its 0 -> 1 and 1 -> 0 half-edges pair with each other
    assert orc.user_halfedges(np.array([[0, 0, 1]])).tolist() == [-1, 2, 1]
    # a closed tetrahedron: every half-edge has a twin, reversed
    tet = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [2, 0, 3]])
    he = orc.user_halfedges(tet)
    assert np.all(he >= 0)
    for h in range(12):
        t, j = divmod(h, 3)
        g = he[h]
        u, k = divmod(int(g), 3)
        assert (tet[t][j], tet[t][(j + 1) % 3]) == (tet[u][(k + 1) % 3], tet[u][k])
    assert orc.user_halfedges(np.zeros((0, 3))).shape == (0,)


@pytest.mark.parametrize("seed", range(20))
def test_quadratic_search_on_soups(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    tris = rng.integers(-2, 8, size=(n, 3))           # few points: many shared, fins, repeats
    he = orc.user_halfedges(tris)
    assert np.array_equal(he, quadratic(tris))
    paired = he >= 0
    assert np.array_equal(he[he[paired]], np.flatnonzero(paired))   # a symmetric pairing
