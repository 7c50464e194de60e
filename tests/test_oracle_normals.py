"""Pins for the oracle's triangle centroids and normals (Sec. 5.2) and the
gather onto the final mesh T."""
import numpy as np
import pytest

from synth import random_grid


def test_axis_aligned_planes_exact(orc):
    v, u = np.meshgrid(np.arange(4.0), np.arange(3.0))
    # plane z = 2 facing a camera that looks down +z (columns -> x, rows -> y)
    g = np.stack([v, u, np.full_like(u, 2.0)], axis=-1)
    n, c = orc.tri_normals(g)
    assert np.all(n == np.array([0.0, 0.0, -1.0]))
    # plane x = 5 with columns -> y and rows -> z: worked by hand for the
    # first triangle (p3, p2, p1): (b-a) = (0,0,-1), (c-a) = (0,-1,-1),
    # cross = (-1, 0, 0)
    g2 = np.stack([np.full_like(u, 5.0), v, u], axis=-1)
    n2, _ = orc.tri_normals(g2)
    assert np.all(n2 == np.array([-1.0, 0.0, 0.0]))
    # rows -> x, columns -> z on the plane y = 0 (mirrored parametrisation):
    # p3 = (1,0,1), p2 = (0,0,1), p1 = (0,0,0); (b-a) = (-1,0,0),
    # (c-a) = (-1,0,-1), cross = (0, -1, 0)
    g3 = np.stack([u, np.zeros_like(u), v], axis=-1)
    n3, _ = orc.tri_normals(g3)
    assert np.all(n3 == np.array([0.0, -1.0, 0.0]))


def test_centroid_is_vertex_mean(orc):
    g = random_grid(5, 6, 1, nan_frac=0.0)
    n, c = orc.tri_normals(g)
    g = g.astype(np.float64)
    # quad (2, 3): first = (p3, p2, p1), second = (p1, p4, p3)
    p1, p2, p3, p4 = g[2, 3], g[2, 4], g[3, 4], g[3, 3]
    assert np.allclose(c[2, 3, 0], (p1 + p2 + p3) / 3, atol=1e-15)
    assert np.allclose(c[2, 3, 1], (p1 + p3 + p4) / 3, atol=1e-15)


def test_normals_unit_and_orthogonal(orc):
    g = random_grid(11, 13, 2, nan_frac=0.0, noise=0.05).astype(np.float64)
    n, _ = orc.tri_normals(g)
    assert np.allclose(np.linalg.norm(n, axis=-1), 1.0, atol=1e-14)
    for u in range(10):
        for v in range(12):
            p1, p2, p3, p4 = g[u, v], g[u, v + 1], g[u + 1, v + 1], g[u + 1, v]
            assert abs(n[u, v, 0] @ (p2 - p3)) < 1e-12 and abs(n[u, v, 0] @ (p1 - p3)) < 1e-12
            assert abs(n[u, v, 1] @ (p4 - p1)) < 1e-12 and abs(n[u, v, 1] @ (p3 - p1)) < 1e-12


def test_normals_face_the_camera(orc):
    # Noise-free pinhole view of a tilted plane: every triangle is front-facing
    # and its normal points back toward the camera at the origin.
    M, N, f = 30, 40, 50.0
    v, u = np.meshgrid(np.arange(N, dtype=np.float64), np.arange(M, dtype=np.float64))
    d = np.stack([(v - 19.5) / f, (u - 14.5) / f, np.ones_like(u)], axis=-1)
    nrm = np.array([0.2, -0.3, -1.0])
    nrm /= np.linalg.norm(nrm)
    t = -2.0 / (d @ nrm)
    g = d * t[..., None]
    n, c = orc.tri_normals(g)
    assert np.all((n * c).sum(-1) < 0)
    assert np.allclose(n, nrm, atol=1e-12)


def test_nan_propagation_and_degenerate(orc):
    g = random_grid(6, 7, 3, nan_frac=0.0).astype(np.float64)
    g[2, 3] = np.nan
    n, c = orc.tri_normals(g)
    bad = np.isnan(n).any(-1)
    # the interior NaN point touches exactly 6 triangles
    assert bad.sum() == 6 and np.array_equal(bad, np.isnan(c).any(-1))
    # collinear vertices: finite centroid, NaN normal
    h = np.zeros((2, 2, 3))
    h[0, 0] = (0, 0, 0); h[0, 1] = (1, 0, 0); h[1, 1] = (2, 0, 0); h[1, 0] = (0, 1, 0)
    n2, c2 = orc.tri_normals(h)
    assert np.isnan(n2[0, 0, 0]).all() and np.isfinite(c2[0, 0, 0]).all()
    assert np.isfinite(n2[0, 0, 1]).all()


def test_gather(orc):
    g = random_grid(8, 9, 4, nan_frac=0.25)
    tri_map, tris = orc.mesh(g)
    n, _ = orc.tri_normals(g)
    nt = orc.gather(n, tri_map, len(tris))
    flat = n.reshape(-1, 3)
    for gid in np.flatnonzero(tri_map != -1):
        assert np.array_equal(nt[tri_map[gid]], flat[gid])
    # the gathered normal belongs to the triangle with those vertices
    gp = g.astype(np.float64).reshape(-1, 3)
    a, b, c = gp[tris[:, 0]], gp[tris[:, 1]], gp[tris[:, 2]]
    x = np.cross(b - a, c - a)
    assert np.allclose(nt, x / np.linalg.norm(x, axis=-1, keepdims=True), atol=1e-12)
