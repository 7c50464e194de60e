"""Pins for the oracle's vertex update (the second stage of the bilateral
mesh denoising the paper cites, Sun et al. 2007; the paper gives no formula
and skips the step, Sec. 5.2).  The restated update is pinned by closed
forms on a plane with known normals and by invariants."""
import numpy as np
import pytest

from synth import random_grid


def plane_grid(M, N, z=2.0, h=0.01):
    v, u = np.meshgrid(np.arange(N, dtype=np.float64), np.arange(M, dtype=np.float64))
    return np.stack([h * v, h * u, np.full_like(u, z)], axis=-1)


def plane_normals(M, N):
    n = np.zeros((M - 1, N - 1, 2, 3))
    n[..., 2] = -1.0          # the grid's triangles face a camera looking down +z
    return n


def test_identity_and_fixed_plane(orc):
    g = plane_grid(7, 9)
    n, _ = orc.tri_normals(g)
    assert np.allclose(n, plane_normals(7, 9), atol=1e-15)
    assert np.array_equal(orc.vertex_update(g, n, 0), g)
    assert np.allclose(orc.vertex_update(g, n, 3), g, atol=1e-15)


def test_displaced_vertex_closed_form(orc):
    """An interior vertex lifted by d off the plane, normals held to the
    plane's: every incident face's centroid is lifted by d/3, so the vertex
    drops to d/3; each of its six mesh neighbours shares two of its six faces
    and rises by (2/6)(d/3) = d/9; nothing else moves."""
    M, N, r, c, d = 9, 11, 4, 5, 0.03
    g = plane_grid(M, N)
    g[r, c, 2] += d
    out = orc.vertex_update(g, plane_normals(M, N), 1)
    dz = out[..., 2] - 2.0
    want = np.zeros((M, N))
    want[r, c] = d / 3
    for dr, dc in ((0, 1), (0, -1), (1, 0), (-1, 0), (1, 1), (-1, -1)):
        want[r + dr, c + dc] = d / 9
    assert np.allclose(dz, want, atol=1e-15)
    assert np.allclose(out[..., :2], g[..., :2], atol=1e-15)
    # a corner vertex drops to d/3 as well (all its faces contain it)
    g = plane_grid(M, N)
    g[0, 0, 2] += d
    out = orc.vertex_update(g, plane_normals(M, N), 1)
    assert abs(out[0, 0, 2] - (2.0 + d / 3)) < 1e-15


def test_tangential_motion_is_kept(orc):
    g = plane_grid(8, 8)
    g[3, 4, :2] += (0.004, -0.003)
    out = orc.vertex_update(g, plane_normals(8, 8), 2)
    assert np.allclose(out, g, atol=1e-15)


def test_rigid_motion_equivariance(orc):
    g = random_grid(12, 15, 3, nan_frac=0.1, noise=0.02).astype(np.float64)
    n, _ = orc.tri_normals(g)
    out = orc.vertex_update(g, n, 2)
    rng = np.random.default_rng(1)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    t = np.array([0.3, -1.2, 4.0])
    out2 = orc.vertex_update(g @ q.T + t, n @ q.T, 2)
    ok = ~np.isnan(out).any(-1)
    assert np.allclose(out2[ok], out[ok] @ q.T + t, atol=1e-12)


def test_invalid_points(orc):
    g = plane_grid(6, 7)
    g[2, 3] = np.nan
    g[3, 3, 2] += 0.02                 # next to the hole
    n, _ = orc.tri_normals(g)
    nn = np.where(np.isnan(n), np.nan, plane_normals(6, 7))
    out = orc.vertex_update(g, nn, 1)
    assert np.isnan(out[2, 3]).all()
    # the lifted vertex loses the faces through the hole but still drops to d/3
    assert abs(out[3, 3, 2] - (2.0 + 0.02 / 3)) < 1e-15
    # a vertex whose every face has a NaN normal is unchanged
    out = orc.vertex_update(g, np.full_like(nn, np.nan), 2)
    assert np.array_equal(np.isnan(out), np.isnan(g)) and np.allclose(out[~np.isnan(g)], g[~np.isnan(g)])
