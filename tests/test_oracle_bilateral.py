"""Pins for the oracle's bilateral normal filter (Eqs. 3-6, Sec. 2.3;
Sec. 5.2).

The neighbourhood reading (both triangles of the K*K - 1 other quads of the
quad window; 16 neighbours at K = 3, the count the paper gives) is pinned by
hand-built cases whose answer follows from symmetry or from a hand sum; the
weights by worked examples at exactly one e-fold; the renormalisation by
closed forms; and edge preservation, plane fixed points and equivariance as
the paper states them.
"""
import math

import numpy as np
import pytest

from synth import random_grid


def unit(x):
    x = np.asarray(x, dtype=np.float64)
    return x / np.linalg.norm(x)


def lattice_centroids(Mq, Nq, spacing=0.01):
    c = np.zeros((Mq, Nq, 2, 3))
    for u in range(Mq):
        for v in range(Nq):
            c[u, v, 0] = (spacing * (v + 0.67), spacing * (u + 0.33), 1.0)
            c[u, v, 1] = (spacing * (v + 0.33), spacing * (u + 0.67), 1.0)
    return c


def test_neighbourhood_is_other_quads_both_triangles(orc):
    # 3x3 quads; centre quad (1, 1).  Its own two triangles carry normals that
    # would show up as a y component if they were counted.  The eight other
    # quads give 14 x (0,0,1) + 2 x (1,0,0) -> (1, 0, 7)/sqrt(50).
    n = np.zeros((3, 3, 2, 3))
    n[...] = (0.0, 0.0, 1.0)
    n[0, 0, :] = (1.0, 0.0, 0.0)
    n[1, 1, 0] = (0.0, 1.0, 0.0)
    n[1, 1, 1] = (0.0, -0.6, 0.8)
    c = lattice_centroids(3, 3)
    out = orc.bilateral(n, c, 3, 1e6, 1e6, 1)
    expect = np.array([1.0, 0.0, 7.0]) / math.sqrt(50.0)
    assert np.allclose(out[1, 1, 0], expect, atol=1e-12)
    assert np.allclose(out[1, 1, 1], expect, atol=1e-12)


def test_sixteen_neighbours_at_k3(orc):
    # Give every triangle of a 5x5 quad grid a distinct tilt; with huge sigmas
    # the output is the renormalised plain sum over the neighbourhood, and the
    # number of neighbours shows in how far the result is from the all-sum.
    rng = np.random.default_rng(0)
    n = rng.normal(size=(5, 5, 2, 3))
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    c = lattice_centroids(5, 5)
    out = orc.bilateral(n, c, 3, 1e8, 1e8, 1)
    u, v = 2, 2
    s = n[u - 1:u + 2, v - 1:v + 2].reshape(-1, 2, 3).sum(axis=(0, 1)) - n[u, v].sum(axis=0)
    assert np.allclose(out[u, v, 0], unit(s), atol=1e-9)
    assert np.allclose(out[u, v, 1], unit(s), atol=1e-9)


def test_window_reach_kernel5_and_border(orc):
    n = np.full((5, 5, 2, 3), np.nan)
    c = lattice_centroids(5, 5)
    n[2, 2, 0] = unit([0.1, 0.2, 1.0])
    n[0, 4, 1] = unit([0.5, -0.3, 1.0])        # quad offset (-2, +2)
    out = orc.bilateral(n, c, 5, 1e6, 1e6, 1)
    assert np.allclose(out[2, 2, 0], n[0, 4, 1], atol=1e-12)
    out3 = orc.bilateral(n, c, 3, 1e6, 1e6, 1)
    assert np.array_equal(out3[2, 2, 0], n[2, 2, 0])   # no neighbour at K = 3
    # corner triangle: partial window, off-grid quads are simply absent
    m = np.full((4, 4, 2, 3), np.nan)
    m[0, 0, 0] = unit([0.0, 0.0, 1.0])
    m[1, 1, 1] = unit([0.0, 1.0, 1.0])
    out_c = orc.bilateral(m, lattice_centroids(4, 4), 3, 1e6, 1e6, 1)
    assert np.allclose(out_c[0, 0, 0], m[1, 1, 1], atol=1e-12)


def test_centroid_weight_one_efold(orc):
    # Two neighbours whose normals are mirror images about n_i (same normal
    # term); A sits at n_i's centroid, B at distance sqrt(2) sigma_l, so B's
    # weight is exactly e^-1 times A's.
    sl, th = 0.1, 0.3
    n = np.full((3, 3, 2, 3), np.nan)
    c = np.zeros((3, 3, 2, 3))
    n[1, 1, 0] = (0.0, 0.0, 1.0)
    nA = np.array([math.sin(th), 0.0, math.cos(th)])
    nB = np.array([-math.sin(th), 0.0, math.cos(th)])
    n[0, 1, 0], n[2, 1, 1] = nA, nB
    c[2, 1, 1] = (0.0, math.sqrt(2.0) * sl, 0.0)
    out = orc.bilateral(n, c, 3, sl, 0.5, 1)
    expect = unit(nA + math.exp(-1.0) * nB)
    assert np.allclose(out[1, 1, 0], expect, atol=1e-14)


def test_normal_weight_one_efold(orc):
    # Both neighbours at n_i's centroid; A has n_i's normal, B a normal whose
    # chord to n_i is sqrt(2) sigma_a, so B's weight is e^-1 times A's.
    sa = 0.1
    th = 2.0 * math.asin(math.sqrt(2.0) * sa / 2.0)
    n = np.full((3, 3, 2, 3), np.nan)
    c = np.zeros((3, 3, 2, 3))
    n[1, 1, 1] = (0.0, 0.0, 1.0)
    nB = np.array([0.0, math.sin(th), math.cos(th)])
    n[1, 0, 0] = (0.0, 0.0, 1.0)
    n[0, 2, 1] = nB
    out = orc.bilateral(n, c, 3, 0.3, sa, 1)
    expect = unit(np.array([0.0, 0.0, 1.0]) + math.exp(-1.0) * nB)
    assert np.allclose(out[1, 1, 1], expect, atol=1e-14)


def test_far_neighbourhood_does_not_underflow(orc):
    # All neighbours 5 m away with sigma_l = 0.1: every weight underflows in
    # double precision, yet the renormalised mean is well defined:
    # exp(-(5.01^2 - 5^2)/0.02) = exp(-5.005) relative weight.
    n = np.full((3, 3, 2, 3), np.nan)
    c = np.zeros((3, 3, 2, 3))
    n[1, 1, 0] = (0.0, 0.0, 1.0)
    n[0, 0, 0] = (1.0, 0.0, 0.0)
    n[2, 2, 1] = (0.0, 1.0, 0.0)
    c[0, 0, 0] = (5.0, 0.0, 0.0)
    c[2, 2, 1] = (0.0, 5.01, 0.0)
    out = orc.bilateral(n, c, 3, 0.1, 1e6, 1)
    w = math.exp(-(5.01 ** 2 - 5.0 ** 2) / 0.02)
    assert np.allclose(out[1, 1, 0], unit([1.0, w, 0.0]), atol=1e-15)


def test_edge_preservation(orc):
    # Two half-planes meeting at 90 degrees: chord sqrt(2) between the sides,
    # weight exp(-2 / (2 * 0.1^2)) = e^-100 relative, so each side keeps its
    # normal to ~1e-43.
    Mq, Nq = 6, 10
    n = np.zeros((Mq, Nq, 2, 3))
    n[:, :5] = (0.0, 0.0, 1.0)
    n[:, 5:] = (1.0, 0.0, 0.0)
    c = lattice_centroids(Mq, Nq)
    out = orc.bilateral(n, c, 3, 0.1, 0.1, 2)
    assert np.max(np.abs(out - n)) < 1e-30


@pytest.mark.parametrize("K", [3, 5])
def test_noise_free_plane_fixed_point(orc, K):
    M, N, f = 20, 24, 30.0
    v, u = np.meshgrid(np.arange(N, dtype=np.float64), np.arange(M, dtype=np.float64))
    d = np.stack([(v - 11.5) / f, (u - 9.5) / f, np.ones_like(u)], axis=-1)
    nrm = unit([0.3, -0.2, -1.0])
    g = d * (-2.0 / (d @ nrm))[..., None]
    g[3, 4] = np.nan
    g[10, 15] = np.nan
    n, c = orc.tri_normals(g)
    out = orc.bilateral(n, c, K, 0.1, 0.1, 3)
    assert np.allclose(out, n, atol=1e-13, equal_nan=True)


def test_nan_neighbour_equals_absent(orc):
    g = random_grid(9, 10, 5, nan_frac=0.0, noise=0.05)
    n, c = orc.tri_normals(g)
    n_a, c_b = n.copy(), c.copy()
    n_a[4, 5, 1] = np.nan           # missing normal
    c_b[4, 5, 1] = np.nan           # missing centroid
    out_a = orc.bilateral(n_a, c, 3, 0.1, 0.2, 1)
    out_b = orc.bilateral(n, c_b, 3, 0.1, 0.2, 1)
    mask = np.ones(out_a.shape[:3], dtype=bool)
    mask[4, 5, 1] = False
    assert np.array_equal(out_a[mask], out_b[mask])
    assert np.isnan(out_a[4, 5, 1]).all()
    assert np.array_equal(out_b[4, 5, 1], n[4, 5, 1])   # own centroid NaN: copied


def test_rotation_equivariance(orc):
    g = random_grid(10, 12, 6, nan_frac=0.1, noise=0.05)
    n, c = orc.tri_normals(g)
    a, b = 0.4, -1.1
    Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1.0]])
    Rx = np.array([[1.0, 0, 0], [0, math.cos(b), -math.sin(b)], [0, math.sin(b), math.cos(b)]])
    R = Rz @ Rx
    out = orc.bilateral(n, c, 3, 0.1, 0.3, 2)
    rot = orc.bilateral(n @ R.T, c @ R.T + np.array([1.0, 2.0, 3.0]), 3, 0.1, 0.3, 2)
    assert np.allclose(rot, out @ R.T, atol=1e-12, equal_nan=True)


@pytest.mark.parametrize("K", [3, 5])
def test_half_turn_equivariance_jacobi(orc, K):
    # Turning the image by 180 degrees maps t_{u,v,k} to
    # t_{Mq-1-u, Nq-1-v, 1-k} and keeps every neighbourhood; Jacobi updates
    # commute with it, a raster-order in-place sweep would not.
    g = random_grid(11, 14, 7, nan_frac=0.15, noise=0.05)
    n, c = orc.tri_normals(g)
    out = orc.bilateral(n, c, K, 0.1, 0.3, 3)
    turn = lambda a: np.ascontiguousarray(a[::-1, ::-1, ::-1])
    out_t = orc.bilateral(turn(n), turn(c), K, 0.1, 0.3, 3)
    assert np.allclose(out_t, turn(out), atol=1e-13, equal_nan=True)


def test_outputs_unit_and_nan_preserved(orc):
    g = random_grid(15, 17, 8, nan_frac=0.2, noise=0.05)
    n, c = orc.tri_normals(g)
    out = orc.bilateral(n, c, 5, 0.1, 0.1, 2)
    assert np.array_equal(np.isnan(out), np.isnan(n))
    ok = ~np.isnan(out).any(-1)
    assert np.allclose(np.linalg.norm(out[ok], axis=-1), 1.0, atol=1e-14)
