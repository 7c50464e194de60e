"""GPU parity on the degenerate inputs the paper leaves to a reading:

* a Laplacian neighbour that coincides with the centre (distance 0, Eq. 2
  gives an infinite weight) is skipped, on the 3x3 and 5x5 windows;
* a valid triangle of zero area (collinear corners) has no normal: its
  normal is NaN, it stays in T (validity is the corners' NaN test of
  Alg. 1), the bilateral filter neither uses it as a neighbour nor filters
  it (its NaN is copied through), and the gather puts a NaN row into N_T
  (Sec. 5.2, Eqs. 3-6).

Both are exact events: the grids below place duplicated and collinear
points on a lattice of small dyadic numbers, so the differences and cross
products are exact in float32 and float64 alike, and the GPU and the FP64
oracle meet the same zeros.  Each case runs through the single-frame calls,
the fused single-frame entry and a batch plan, against the oracle.
"""
import os

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def pl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2007_12065_amd as pl
    return pl


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def angle(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(-1, 3)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 3)
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), np.sum(a * b, axis=-1))


def lattice(M, N, seed, nan_frac=0.05):
    """A bumpy surface on a lattice of multiples of 1/64 (exact in float32):
    x = v / 8, y = u / 8, z = 4 + k / 64 with k random in [-8, 8]."""
    rng = np.random.default_rng(seed)
    v, u = np.meshgrid(np.arange(N), np.arange(M))
    z = 4.0 + rng.integers(-8, 9, size=(M, N)) / 64.0
    pts = np.stack([v / 8.0, u / 8.0, z], axis=-1).astype(np.float32)
    if nan_frac:
        pts[rng.random((M, N)) < nan_frac] = np.nan
    return pts


def with_duplicates(pts, seed, count):
    """Copy `count` random pixels onto their right-hand neighbour (the pair
    then coincides exactly)."""
    p = pts.copy()
    rng = np.random.default_rng(seed)
    M, N = p.shape[:2]
    for _ in range(count):
        u, v = int(rng.integers(0, M)), int(rng.integers(0, N - 1))
        p[u, v + 1] = p[u, v]
    return p


def with_collinear(pts, seed, count):
    """Make `count` random quads' first triangle (p3, p2, p1) degenerate:
    p2 = (u, v+1) is moved to the midpoint of p1 = (u, v) and p3 = (u+1, v+1),
    exact on the lattice.  Returns the grid and the quads (u, v) touched."""
    p = pts.copy()
    rng = np.random.default_rng(seed)
    M, N = p.shape[:2]
    quads = set()
    while len(quads) < count:
        u, v = int(rng.integers(1, M - 2)), int(rng.integers(1, N - 2))
        if any(abs(u - a) <= 1 and abs(v - b) <= 1 for a, b in quads):
            continue
        if np.isnan(p[u, v]).any() or np.isnan(p[u + 1, v + 1]).any():
            continue
        p[u, v + 1] = (p[u, v] + p[u + 1, v + 1]) * np.float32(0.5)
        quads.add((u, v))
    return p, sorted(quads)


def check_points(gpu, ref):
    g = gpu.astype(np.float64)
    bad = np.isnan(ref).any(-1)
    assert np.array_equal(np.isnan(g).any(-1), bad)
    err = np.linalg.norm(g[~bad] - ref[~bad], axis=-1) / np.linalg.norm(ref[~bad], axis=-1)
    assert err.max(initial=0.0) <= 1e-5, err.max()


def check_normals(gpu, ref, tol=1e-4):
    g = np.asarray(gpu, dtype=np.float64).reshape(-1, 3)
    r = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
    nan_r = np.isnan(r).any(-1)
    assert np.array_equal(np.isnan(g).any(-1), nan_r)
    a = angle(g[~nan_r], r[~nan_r])
    assert a.max(initial=0.0) <= tol, a.max()


@pytest.mark.parametrize("K", [3, 5])
def test_laplacian_coincident_neighbours(pl, K):
    pts = with_duplicates(lattice(37, 70, 1), 2, 200)
    # the reading is exercised: many valid pixels have an exactly coinciding neighbour
    same = np.all(pts[:, 1:] == pts[:, :-1], axis=-1) & ~np.isnan(pts[:, 1:]).any(-1)
    assert same.sum() >= 150
    for iters in (1, 3):
        print(f"[case] laplacian K{K} x{iters} with coincident neighbours", flush=True)
        got = host(pl.pl_laplacian(to_dev(pts), K, 1.0, iters))
        ref = oracle.laplacian(pts, K, 1.0, iters, THREADS)
        assert np.isfinite(got[~np.isnan(ref).any(-1)]).all()
        check_points(got, ref)


def test_zero_area_triangles_single_calls(pl):
    import torch
    pts, quads = with_collinear(lattice(40, 90, 3), 4, 60)
    n, c = pl.pl_tri_normals(to_dev(pts), torch.float32)
    rn, rc = oracle.tri_normals(pts, THREADS)
    n, c = host(n), host(c)
    # the degenerate triangles: valid corners, finite centroid, NaN normal
    for u, v in quads:
        assert np.isnan(rn[u, v, 0]).all() and np.isfinite(rc[u, v, 0]).all()
        assert np.isnan(n[u, v, 0]).all() and np.isfinite(c[u, v, 0]).all()
    check_normals(n, rn, tol=1e-6)
    ok = ~np.isnan(rc).any(-1)
    assert np.abs(c[ok] - rc[ok]).max() <= 1e-6
    # they stay in T: validity is the corners' NaN test
    m = pl.pl_mesh_opc(to_dev(pts))
    tri_map, tris = oracle.mesh(pts)
    assert np.array_equal(host(m["tri_map"]), tri_map)
    Nq = pts.shape[1] - 1
    gids = [2 * (u * Nq + v) for u, v in quads]
    assert (tri_map[gids] >= 0).all()
    # bilateral on identical float32 inputs, with the gather: the degenerate
    # triangles are skipped as neighbours and copied through as NaN
    n32, c32 = rn.astype(np.float32), rc.astype(np.float32)
    for iters in (1, 2):
        print(f"[case] bilateral x{iters} around zero-area triangles", flush=True)
        out, nT = pl.pl_bilateral(to_dev(n32), to_dev(c32), 3, 0.1, 0.1, iters,
                                  tri_map=to_dev(tri_map))
        ref = oracle.bilateral(n32, c32, 3, 0.1, 0.1, iters, THREADS)
        out = host(out)
        check_normals(out, ref)
        for u, v in quads:
            assert np.isnan(out[u, v, 0]).all()
        t = host(nT)[:len(tris)]
        want = oracle.gather(ref, tri_map, len(tris))
        rows = tri_map[gids]
        assert np.isnan(t[rows]).all() and np.isnan(want[rows]).all()
        check_normals(t, want)


def _spec(pts, kl, il, kb, ib):
    return dict(pts=to_dev(pts), kernel_lap=kl, lam=1.0, iters_lap=il, kernel_bil=kb,
                sigma_length=0.1, sigma_angle=0.1, iters_bil=ib)


@pytest.mark.parametrize("path", ["fused", "batch"])
def test_degenerate_whole_path(pl, path):
    """Zero-area triangles (no Laplacian sweep, so they stay degenerate) and
    coincident points (with sweeps) through the fused single-frame entry and
    a batch plan, against the oracle's whole pipeline."""
    import torch
    deg, quads = with_collinear(lattice(48, 100, 5), 6, 80)
    dup = with_duplicates(lattice(33, 70, 7), 8, 150)
    specs = [(_spec(deg, 3, 0, 3, 2), deg, (3, 0, 3, 2)), (_spec(dup, 5, 2, 5, 1), dup, (5, 2, 5, 1)),
             (_spec(dup, 3, 4, 3, 2), dup, (3, 4, 3, 2))]
    if path == "fused":
        outs = [pl.pl_smooth_frame(s, torch.float32) for s, _, _ in specs]
    else:
        b = pl.Batch([s for s, _, _ in specs], torch.float32)
        b.run()
        outs = b.outputs
    for i, ((s, pts, (kl, il, kb, ib)), o) in enumerate(zip(specs, outs)):
        print(f"[case] {path} degenerate frame {i}", flush=True)
        ref = oracle.pipeline(pts, kl, 1.0, il, kb, 0.1, 0.1, ib, THREADS)
        n = int(host(o["n_tri"])[0])
        assert n == len(ref["triangles"])
        assert np.array_equal(host(o["tri_map"]), ref["tri_map"])
        assert np.array_equal(host(o["triangles"])[:n], ref["triangles"])
        check_points(host(o["points"]), ref["points"])
        nT = host(o["normals_T"])[:n]
        r = ref["normals_T"]
        if i == 0:
            # the zero-area triangles: NaN rows of N_T on both sides
            rows = ref["tri_map"][[2 * (u * (pts.shape[1] - 1) + v) for u, v in quads]]
            assert np.isnan(nT[rows]).all() and np.isnan(r[rows]).all()
        # float32 normals and smoothing upstream of the filter: the NaN pattern
        # matches exactly, the angles follow the end-to-end bound
        nan_r = np.isnan(r).any(-1)
        assert np.array_equal(np.isnan(nT).any(-1), nan_r)
        a = angle(nT[~nan_r], r[~nan_r])
        assert np.median(a) <= 1e-4 and np.percentile(a, 99) <= 1e-3, (np.median(a), a.max())
    if path == "batch":
        b.close()
