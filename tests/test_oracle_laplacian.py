"""Pins for the oracle's Laplacian filter (Eqs. 1-2, Sec. 2.3; Sec. 5.1).

Worked examples derived by hand, closed forms, and invariants that any
correct reading must satisfy: lambda = 0 is the identity, coplanar points stay
on their plane, the image border is pinned, NaN pixels never contribute, and
Jacobi iterations commute with flips of the image.
"""
import math

import numpy as np
import pytest

from synth import random_grid


def nan_grid(M, N):
    return np.full((M, N, 3), np.nan, dtype=np.float64)


def test_lambda_zero_identity(orc):
    g = random_grid(12, 17, 1, nan_frac=0.2)
    out = orc.laplacian(g, 3, 0.0, 4)
    assert np.array_equal(out, g.astype(np.float64), equal_nan=True)


def test_zero_iterations_identity(orc):
    g = random_grid(12, 17, 2, nan_frac=0.2)
    assert np.array_equal(orc.laplacian(g, 5, 1.0, 0), g.astype(np.float64), equal_nan=True)


@pytest.mark.parametrize("lam", [0.25, 0.5, 1.0])
def test_lifted_center_closed_form(orc, lam):
    # Flat unit lattice z = 0, centre lifted by h.  All eight neighbours lie on
    # z = 0 and are placed symmetrically, so their weighted mean is the centre's
    # foot point and the output height is (1 - lambda) h.
    h = 0.37
    v, u = np.meshgrid(np.arange(3.0), np.arange(3.0))
    g = np.stack([v, u, np.zeros_like(u)], axis=-1)
    g[1, 1, 2] = h
    out = orc.laplacian(g, 3, lam, 1)
    assert out[1, 1].tolist() == pytest.approx([1.0, 1.0, (1.0 - lam) * h], abs=1e-15)


@pytest.mark.parametrize("lam,expect", [(1.0, (2 / 3, 2 / 3, 0.0)), (0.5, (1 / 3, 1 / 3, 0.0))])
def test_inverse_distance_worked_example(orc, lam, expect):
    # Centre at the origin with two usable neighbours: a = (1,0,0) at distance
    # 1 and b = (0,2,0) at distance 2.  Weights 1 and 1/2 give the mean
    # (a + b/2) / (3/2) = (2/3, 2/3, 0).
    g = nan_grid(3, 3)
    g[1, 1] = (0.0, 0.0, 0.0)
    g[1, 2] = (1.0, 0.0, 0.0)
    g[0, 1] = (0.0, 2.0, 0.0)
    out = orc.laplacian(g, 3, lam, 1)
    assert out[1, 1].tolist() == pytest.approx(list(expect), abs=1e-15)


def test_window_reach_kernel5(orc):
    g = nan_grid(5, 5)
    g[2, 2] = (0.0, 0.0, 0.0)
    g[0, 4] = (3.0, -1.0, 2.0)     # offset (-2, +2): inside the 5x5 window
    assert orc.laplacian(g, 5, 1.0, 1)[2, 2].tolist() == pytest.approx([3.0, -1.0, 2.0], abs=1e-15)
    # outside the 3x3 window: no usable neighbour, the pixel keeps its value
    g7 = nan_grid(7, 7)
    g7[3, 3] = (0.0, 0.0, 0.0)
    g7[1, 5] = (3.0, -1.0, 2.0)
    assert g7[3, 3].tolist() == orc.laplacian(g7, 3, 1.0, 1)[3, 3].tolist()


@pytest.mark.parametrize("bad", [(np.nan, 5.0, 5.0), (5.0, np.nan, 5.0), (5.0, 5.0, np.nan)])
def test_partial_nan_point_is_invalid(orc, bad):
    # A point with any NaN coordinate is invalid and contributes nothing.
    g = nan_grid(3, 3)
    g[1, 1] = (0.0, 0.0, 0.0)
    g[1, 2] = (1.0, 0.0, 0.0)
    g[0, 0] = bad
    assert orc.laplacian(g, 3, 1.0, 1)[1, 1].tolist() == pytest.approx([1.0, 0.0, 0.0], abs=1e-15)


@pytest.mark.parametrize("K", [3, 5])
def test_border_band_pinned(orc, K):
    g = random_grid(14, 19, 3, nan_frac=0.1)
    out = orc.laplacian(g, K, 1.0, 3)
    r = K // 2
    g64 = g.astype(np.float64)
    band = np.ones((14, 19), dtype=bool)
    band[r:14 - r, r:19 - r] = False
    assert np.array_equal(out[band], g64[band], equal_nan=True)
    inner = ~band & ~np.isnan(g).any(-1)
    assert np.all(np.any(out[inner] != g64[inner], axis=-1))


def test_nan_pattern_invariant(orc):
    g = random_grid(20, 25, 4, nan_frac=0.3)
    out = orc.laplacian(g, 5, 0.8, 3)
    assert np.array_equal(np.isnan(out), np.isnan(g))


@pytest.mark.parametrize("K", [3, 5])
def test_coplanar_points_stay_on_plane(orc, K):
    rng = np.random.default_rng(5)
    M, N = 16, 21
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    e1 = np.cross(n, [0.3, 0.5, 0.8])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(n, e1)
    v, u = np.meshgrid(np.arange(N, dtype=np.float64), np.arange(M, dtype=np.float64))
    a = 0.1 * v + rng.uniform(-0.03, 0.03, size=v.shape)
    b = 0.1 * u + rng.uniform(-0.03, 0.03, size=u.shape)
    d0 = 2.5
    g = d0 * n + a[..., None] * e1 + b[..., None] * e2
    g[rng.random((M, N)) < 0.15] = np.nan
    out = orc.laplacian(g, K, 1.0, 5)
    res = np.abs(out @ n - d0)
    assert np.nanmax(res) < 1e-12


def test_affine_lattice_interior_fixed_point(orc):
    # Weights depend only on distance and the full window is point-symmetric,
    # so an affine lattice is a fixed point away from the border.
    M, N = 9, 11
    v, u = np.meshgrid(np.arange(N, dtype=np.float64), np.arange(M, dtype=np.float64))
    o, a, b = np.array([0.1, -0.2, 3.0]), np.array([0.05, 0.01, 0.02]), np.array([-0.01, 0.04, 0.03])
    g = o + v[..., None] * a + u[..., None] * b
    for K in (3, 5):
        out = orc.laplacian(g, K, 1.0, 2)
        assert np.max(np.abs(out - g)) < 1e-13


@pytest.mark.parametrize("K", [3, 5])
def test_flip_equivariance_jacobi(orc, K):
    # Jacobi updates commute with mirroring the image; an in-place sweep in
    # raster order would not.
    g = random_grid(13, 16, 6, nan_frac=0.15, noise=0.05)
    out = orc.laplacian(g, K, 0.9, 3)
    for axis in (0, 1):
        flipped = orc.laplacian(np.flip(g, axis=axis), K, 0.9, 3)
        assert np.allclose(flipped, np.flip(out, axis=axis), rtol=0, atol=1e-13, equal_nan=True)
    tr = orc.laplacian(np.ascontiguousarray(g.transpose(1, 0, 2)), K, 0.9, 3)
    assert np.allclose(tr, out.transpose(1, 0, 2), rtol=0, atol=1e-13, equal_nan=True)


def test_rigid_and_scale_equivariance(orc):
    g = random_grid(12, 14, 7, nan_frac=0.1, noise=0.05).astype(np.float64)
    th = 0.7
    R = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1.0]])
    t = np.array([1.0, -2.0, 0.5])
    out = orc.laplacian(g, 3, 0.7, 3)
    moved = orc.laplacian(g @ R.T * 2.5 + t, 3, 0.7, 3)
    assert np.allclose(moved, out @ R.T * 2.5 + t, atol=1e-12, equal_nan=True)


def test_two_iterations_worked_example(orc):
    # 1x5 interior strip embedded in a 3x5 grid whose outer rows are NaN.
    # Points on a line x = 0, 1, 3, 4, 6 (y = z = 0).  Pixel 1 (x=1) has
    # neighbours at distance 1 and 2: mean (0/1 + 3/2)/(1 + 1/2) = 1.
    # Pixel 2 (x=3): neighbours x=1 (d=2), x=4 (d=1): (1/2 + 4)/(3/2) = 3.
    # Pixel 3 (x=4): neighbours x=3 (d=1), x=6 (d=2): (3 + 3)/(3/2) = 4.
    # In general one neighbour on each side at distances d_l, d_r gives
    # ((x_i - d_l)/d_l + (x_i + d_r)/d_r) / (1/d_l + 1/d_r) = x_i, so the
    # unevenly spaced line is a fixed point (uniform weights would move it).
    g = nan_grid(3, 5)
    g[1, :, 0] = [0.0, 1.0, 3.0, 4.0, 6.0]
    g[1, :, 1:] = 0.0
    out = orc.laplacian(g, 3, 1.0, 2)
    assert np.allclose(out[1, :, 0], [0.0, 1.0, 3.0, 4.0, 6.0], atol=1e-15)
    # Lift pixel 2 by 0.5 in y: both its neighbours lie on y = 0, so one step
    # at lambda = 1 brings it back to y = 0 while its neighbours, which see
    # the lifted pixel, move up.
    g[1, 2, 1] = 0.5
    out1 = orc.laplacian(g, 3, 1.0, 1)
    assert out1[1, 2, 1] == pytest.approx(0.0, abs=1e-15)
    assert out1[1, 1, 1] > 0 and out1[1, 3, 1] > 0
