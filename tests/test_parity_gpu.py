"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Integer outputs (validity mask, T_map, T, HE, |T|) must match bit for bit.
Floating-point stages are compared stage by stage on identical float32
inputs: vertices within 1e-5 relative (per vertex, Euclidean norm), normals
within 1e-4 rad; invalid pixels / NaN triangles must keep their NaN pattern,
and copied values (border band, invalid pixels) must be bitwise copies.
Sizes span several tiles with ragged tails; the full 120x160, 480x640,
64x1024 and 128x2048 synthetic frames run at their real shapes.
"""
import os

import numpy as np
import pytest

import oracle
from synth import KINDS, config_frame, make_frame, random_grid

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)
VERTEX_RTOL = 1e-5
NORMAL_ATOL = 1e-4


@pytest.fixture(scope="module")
def pl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2007_12065_amd as pl
    return pl


def dev():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*a):
    print("[case]", *a, flush=True)


def angle(a, b):
    """Angle in radians between row vectors (float64, robust near 0)."""
    a = np.asarray(a, dtype=np.float64).reshape(-1, 3)
    b = np.asarray(b, dtype=np.float64).reshape(-1, 3)
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=-1), np.sum(a * b, axis=-1))


def check_points(gpu, ref, inp):
    gpu = gpu.astype(np.float64)
    bad_ref = np.isnan(ref).any(-1)
    assert np.array_equal(np.isnan(gpu).any(-1), bad_ref)
    ok = ~bad_ref
    err = np.linalg.norm(gpu[ok] - ref[ok], axis=-1) / np.maximum(np.linalg.norm(ref[ok], axis=-1), 1e-30)
    assert err.max(initial=0.0) <= VERTEX_RTOL, err.max()
    # untouched pixels are bitwise copies of the input
    same = np.all(ref == inp.astype(np.float64), axis=-1) | bad_ref
    assert np.array_equal(gpu.astype(np.float32).view(np.uint32)[same],
                          inp.view(np.uint32)[same])
    return err.max(initial=0.0)


def check_normals(gpu, ref, tol=NORMAL_ATOL):
    g = np.asarray(gpu, dtype=np.float64).reshape(-1, 3)
    r = np.asarray(ref, dtype=np.float64).reshape(-1, 3)
    nan_r = np.isnan(r).any(-1)
    assert np.array_equal(np.isnan(g).any(-1), nan_r)
    ang = angle(g[~nan_r], r[~nan_r])
    assert ang.max(initial=0.0) <= tol, (ang.max(), np.percentile(ang, 99))
    return ang


# ---------------------------------------------------------------- mesh

MESH_GRIDS = [(2, 2, 0.0), (2, 3, 0.2), (3, 2, 0.2), (7, 7, 0.15), (5, 300, 0.1),
              (300, 5, 0.1), (4, 600, 0.3), (33, 260, 0.05), (2, 1000, 0.5), (17, 513, 0.0),
              (3, 1025, 0.1), (2, 1026, 0.0), (4, 2100, 0.2), (3, 3075, 0.05),
              # one full 256-quad segment; a second segment of one quad
              (4, 257, 0.1), (6, 258, 0.1),
              # 256 x 32 = 8192 row segments of 256 quads: the largest frame
              # meshed by segments; 299 x 28 = 8372 takes the whole-row kernels
              (257, 8193, 0.1), (300, 7000, 0.1)]


def mesh_compare(pl, pts, cap=None):
    say("mesh", pts.shape, "cap", cap)
    r = pl.pl_mesh_opc(to_dev(pts), cap=cap)
    tri_map, tris = oracle.mesh(pts)
    M, N = pts.shape[:2]
    he = oracle.halfedges(tri_map, M, N, len(tris))
    n = int(host(r["n_tri"])[0])
    assert n == len(tris)
    assert np.array_equal(host(r["tri_map"]), tri_map)
    assert np.array_equal(host(r["tri_valid"]), (tri_map != -1).astype(np.uint8))
    k = n if cap is None else min(n, cap)
    assert np.array_equal(host(r["triangles"])[:k], tris[:k])
    if cap is None:
        assert np.array_equal(host(r["halfedges"])[:3 * n], he)
    else:
        assert np.array_equal(host(r["halfedges"])[:3 * k], he[:3 * k])


@pytest.mark.parametrize("M,N,frac", MESH_GRIDS)
def test_mesh_grids(pl, M, N, frac):
    mesh_compare(pl, random_grid(M, N, seed=M * 1000 + N, nan_frac=frac))


@pytest.mark.parametrize("kind", ["rgbd_small", "rgbd", "lidar", "lidar128"])
def test_mesh_frames(pl, kind):
    mesh_compare(pl, make_frame(kind, 11))


def test_mesh_all_nan_and_cap(pl):
    mesh_compare(pl, np.full((6, 9, 3), np.nan, dtype=np.float32))
    g = random_grid(20, 40, 3, nan_frac=0.2)
    mesh_compare(pl, g, cap=100)
    mesh_compare(pl, g, cap=0)
    big = random_grid(300, 7000, 5, nan_frac=0.2)          # whole-row kernels
    mesh_compare(pl, big, cap=123457)
    seg = random_grid(64, 1100, 6, nan_frac=0.2)           # segments, cap inside a segment
    mesh_compare(pl, seg, cap=70001)


@pytest.mark.parametrize("M,N", [(30, 70), (300, 7000)])   # segment and whole-row kernels
def test_mesh_optional_outputs(pl, M, N):
    g = random_grid(M, N, 4, nan_frac=0.2)
    r = pl.pl_mesh_opc(to_dev(g), tri_valid=False, halfedges=False)
    tri_map, tris = oracle.mesh(g)
    assert r["tri_valid"] is None and r["halfedges"] is None
    assert np.array_equal(host(r["tri_map"]), tri_map)
    assert np.array_equal(host(r["triangles"])[:len(tris)], tris)


# ---------------------------------------------------------------- Laplacian

LAP_GRIDS = [(2, 2), (5, 5), (16, 64), (37, 150), (100, 70), (9, 300)]


@pytest.mark.parametrize("M,N", LAP_GRIDS)
@pytest.mark.parametrize("K", [3, 5, 7, 9])
def test_laplacian_grids(pl, M, N, K):
    g = random_grid(M, N, seed=7 * M + N + K, nan_frac=0.12, noise=0.02)
    for iters, lam in [(0, 1.0), (1, 1.0), (2, 0.5), (3, 1.0), (5, 0.7), (9, 1.0)]:
        say("laplacian", (M, N), "K", K, "iters", iters, "lam", lam)
        out = host(pl.pl_laplacian(to_dev(g), K, lam, iters))
        ref = oracle.laplacian(g, K, lam, iters, THREADS)
        check_points(out, ref, g)


@pytest.mark.parametrize("config", [0, 1, 2])
def test_laplacian_frames(pl, config):
    pts, k = config_frame(config)
    say("laplacian frame", config)
    out = host(pl.pl_laplacian(to_dev(pts), k.kernel_lap, k.lam, k.iters_lap))
    ref = oracle.laplacian(pts, k.kernel_lap, k.lam, k.iters_lap, THREADS)
    err = check_points(out, ref, pts)
    print(f"config {config}: max vertex rel err {err:.2e}")


def test_laplacian_lidar128(pl):
    k = KINDS["lidar128"]
    pts = make_frame("lidar128", 21)
    out = host(pl.pl_laplacian(to_dev(pts), k.kernel_lap, k.lam, k.iters_lap))
    check_points(out, oracle.laplacian(pts, k.kernel_lap, k.lam, k.iters_lap, THREADS), pts)


# ---------------------------------------------------------------- normals

@pytest.mark.parametrize("M,N", [(2, 2), (3, 7), (40, 300), (129, 65)])
def test_normals_grids(pl, M, N):
    import torch
    g = random_grid(M, N, seed=M + 3 * N, nan_frac=0.1, noise=0.02)
    say("normals", (M, N))
    n, c = pl.pl_tri_normals(to_dev(g), torch.float32)
    rn, rc = oracle.tri_normals(g)
    check_normals(host(n), rn)
    cc = host(c).astype(np.float64)
    assert np.array_equal(np.isnan(cc), np.isnan(rc))
    ok = ~np.isnan(rc)
    assert np.max(np.abs(cc[ok] - rc[ok])) <= 1e-6 * max(1.0, np.abs(rc[ok]).max())


@pytest.mark.parametrize("kind", ["rgbd_small", "rgbd", "lidar", "lidar128"])
def test_normals_frames(pl, kind):
    import torch
    pts = make_frame(kind, 5)
    say("normals frame", kind)
    n, c = pl.pl_tri_normals(to_dev(pts), torch.float32)
    rn, rc = oracle.tri_normals(pts)
    ang = check_normals(host(n), rn)
    print(f"{kind}: normal angle err p99 {np.percentile(ang, 99):.2e} max {ang.max():.2e}")
    n16, _ = pl.pl_tri_normals(to_dev(pts), torch.float16)
    check_normals(host(n16).astype(np.float32), rn, tol=1e-3)


# ---------------------------------------------------------------- bilateral

def bil_inputs(pts):
    """Normals and centroids from the oracle, rounded to float32: the same
    float32 arrays go to both sides."""
    n, c = oracle.tri_normals(pts, THREADS)
    return n.astype(np.float32), c.astype(np.float32)


BIL_GRIDS = [(2, 2), (3, 3), (9, 33), (30, 100), (17, 70), (50, 20)]


@pytest.mark.parametrize("M,N", BIL_GRIDS)
@pytest.mark.parametrize("K", [3, 5, 7, 9])
def test_bilateral_grids(pl, M, N, K):
    g = random_grid(M, N, seed=11 * M + N + K, nan_frac=0.1, noise=0.02)
    n, c = bil_inputs(g)
    for iters, sl, sa in [(0, 0.1, 0.1), (1, 0.1, 0.1), (2, 0.05, 0.3), (3, 0.1, 0.1)]:
        say("bilateral", (M, N), "K", K, "iters", iters, "sigmas", sl, sa)
        out, _ = pl.pl_bilateral(to_dev(n), to_dev(c), K, sl, sa, iters)
        ref = oracle.bilateral(n, c, K, sl, sa, iters, THREADS)
        check_normals(host(out), ref)
        if iters == 0:
            assert np.array_equal(host(out).view(np.uint32), n.view(np.uint32))


@pytest.mark.parametrize("config", [0, 1, 2])
def test_bilateral_frames(pl, config):
    pts, k = config_frame(config)
    smooth = oracle.laplacian(pts, k.kernel_lap, k.lam, k.iters_lap, THREADS).astype(np.float32)
    n, c = bil_inputs(smooth)
    say("bilateral frame", config)
    tri_map, tris = oracle.mesh(pts)
    out, nT = pl.pl_bilateral(to_dev(n), to_dev(c), k.kernel_bil, k.sigma_length,
                              k.sigma_angle, k.iters_bil, tri_map=to_dev(tri_map))
    ref = oracle.bilateral(n, c, k.kernel_bil, k.sigma_length, k.sigma_angle, k.iters_bil, THREADS)
    ang = check_normals(host(out), ref)
    print(f"config {config}: bilateral angle err p99 {np.percentile(ang, 99):.2e} max {ang.max():.2e}")
    # the gather is a copy of the filtered T_FC normals of the valid GIDs
    o = host(out).reshape(-1, 3)
    t = host(nT)[:len(tris)]
    valid = tri_map >= 0
    assert np.array_equal(t.view(np.uint32), o[valid].view(np.uint32))


def test_bilateral_lidar128(pl):
    k = KINDS["lidar128"]
    pts = make_frame("lidar128", 22)
    n, c = bil_inputs(pts)
    out, _ = pl.pl_bilateral(to_dev(n), to_dev(c), k.kernel_bil, k.sigma_length,
                             k.sigma_angle, k.iters_bil)
    check_normals(host(out), oracle.bilateral(n, c, k.kernel_bil, k.sigma_length,
                                              k.sigma_angle, k.iters_bil, THREADS))


def test_bilateral_far_neighbourhood(pl):
    # every neighbour 5 m away with sigma_length 0.1: all weights underflow
    # unless the exponents are shifted; the renormalised mean is still defined
    n = np.full((3, 3, 2, 3), np.nan, dtype=np.float32)
    c = np.zeros((3, 3, 2, 3), dtype=np.float32)
    n[1, 1, 0] = (0, 0, 1); n[0, 0, 0] = (1, 0, 0); n[2, 2, 1] = (0, 1, 0)
    c[0, 0, 0] = (5.0, 0, 0); c[2, 2, 1] = (0, 5.01, 0)
    out, _ = pl.pl_bilateral(to_dev(n), to_dev(c), 3, 0.1, 1e6, 1)
    ref = oracle.bilateral(n, c, 3, 0.1, 1e6, 1)
    check_normals(host(out), ref)


def test_bilateral_edge_preservation(pl):
    n = np.zeros((6, 10, 2, 3), dtype=np.float32)
    n[:, :5] = (0, 0, 1)
    n[:, 5:] = (1, 0, 0)
    c = np.zeros_like(n)
    v, u = np.meshgrid(np.arange(10), np.arange(6))
    c[..., 0] = 0.01 * v[..., None]
    c[..., 1] = 0.01 * u[..., None]
    out, _ = pl.pl_bilateral(to_dev(n), to_dev(c), 3, 0.1, 0.1, 2)
    assert np.max(np.abs(host(out) - n)) < 1e-6


def test_bilateral_fp16_stagewise(pl):
    # float16 storage, identical float16-rounded inputs on both sides, one
    # sweep: the only differences are float32 arithmetic and the final
    # rounding of the output to float16 (< 2^-11 relative per component).
    import torch
    pts, k = config_frame(1)
    smooth = oracle.laplacian(pts, k.kernel_lap, k.lam, k.iters_lap, THREADS).astype(np.float32)
    n, c = bil_inputs(smooth)
    n16 = n.astype(np.float16)
    ref = oracle.bilateral(n16.astype(np.float64), c, k.kernel_bil, k.sigma_length,
                           k.sigma_angle, 1, THREADS)
    out, _ = pl.pl_bilateral(to_dev(n16), to_dev(c), k.kernel_bil, k.sigma_length,
                             k.sigma_angle, 1)
    assert out.dtype == torch.float16
    ang = check_normals(host(out).astype(np.float32), ref, tol=1e-3)
    print(f"fp16 one sweep: angle err p99 {np.percentile(ang, 99):.2e} max {ang.max():.2e}")


def test_bilateral_fp16_vs_fp64(pl):
    # The float16 path as used (normals stored in float16 between sweeps)
    # against the FP64 oracle on the float32 normals.  Where a window holds
    # two balanced clusters of normals (edges), the filter amplifies input
    # perturbations ~100x, so storage rounding shows up at a few triangles;
    # the distribution is gated at p99 and reported in full.
    import torch
    pts, k = config_frame(1)
    smooth = oracle.laplacian(pts, k.kernel_lap, k.lam, k.iters_lap, THREADS).astype(np.float32)
    n, c = bil_inputs(smooth)
    ref = oracle.bilateral(n, c, k.kernel_bil, k.sigma_length, k.sigma_angle, k.iters_bil, THREADS)
    out, _ = pl.pl_bilateral(to_dev(n).to(torch.float16), to_dev(c), k.kernel_bil,
                             k.sigma_length, k.sigma_angle, k.iters_bil)
    g = host(out).astype(np.float64).reshape(-1, 3)
    r = ref.reshape(-1, 3)
    nan_r = np.isnan(r).any(-1)
    assert np.array_equal(np.isnan(g).any(-1), nan_r)
    ang = angle(g[~nan_r], r[~nan_r])
    # the same amplification in exact arithmetic: FP64 on float16-rounded input
    ref16 = oracle.bilateral(n.astype(np.float16).astype(np.float64), c, k.kernel_bil,
                             k.sigma_length, k.sigma_angle, k.iters_bil, THREADS)
    amp = angle(ref16.reshape(-1, 3)[~nan_r], r[~nan_r])
    print(f"fp16 vs fp64: p50 {np.median(ang):.2e} p99 {np.percentile(ang, 99):.2e} "
          f"max {ang.max():.2e}; exact arithmetic on rounded input: max {amp.max():.2e}")
    assert np.percentile(ang, 99) <= 1e-3


# ---------------------------------------------------------------- whole path

def yardsticks(ref, k, n):
    """The spread exact arithmetic shows on the same path: the FP64 pipeline
    restarted from its own smoothed vertices rounded to float32 (y32), and the
    same with the normals rounded to float16 wherever the float16 mode stores
    them -- the raw normals and each sweep's output (y16).  The bilateral
    weights (sigma_angle = 0.1 on noisy normals) amplify such perturbations
    by 1e2..1e3 where a window holds two balanced clusters of normals."""
    n32, c32 = oracle.tri_normals(ref["points"].astype(np.float32), THREADS)
    f = oracle.bilateral(n32, c32, k.kernel_bil, k.sigma_length, k.sigma_angle, k.iters_bil,
                         THREADS)
    y32 = angle(oracle.gather(f, ref["tri_map"], n), ref["normals_T"])
    g = n32.astype(np.float16).astype(np.float64)
    for _ in range(k.iters_bil):
        g = oracle.bilateral(g, c32, k.kernel_bil, k.sigma_length, k.sigma_angle, 1, THREADS)
        g = g.astype(np.float16).astype(np.float64)
    y16 = angle(oracle.gather(g, ref["tri_map"], n), ref["normals_T"])
    return y32, y16


@pytest.mark.parametrize("dtype_name", ["float32", "float16"])
@pytest.mark.parametrize("config", [0, 1, 2])
def test_end_to_end(pl, config, dtype_name):
    """The whole path against the FP64 oracle.  Integers exact, vertices within
    1e-5; the filtered normals' error distribution is gated in full: the
    median at 1e-4 rad (float32) and the 99th percentile at 1e-3 rad (both
    modes; the float16 target is stated at that percentile), and the largest
    error at three times the largest of the exact-arithmetic yardstick for
    the same storage (plus 1e-4 rad), so the tail has to be the conditioning
    of the filter and not the kernels' arithmetic."""
    import torch
    pts, k = config_frame(config)
    say("end to end", config, dtype_name)
    r = pl.smooth_frame(to_dev(pts), k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil,
                        k.sigma_length, k.sigma_angle, k.iters_bil,
                        normal_dtype=getattr(torch, dtype_name))
    ref = oracle.pipeline(pts, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil,
                          k.sigma_length, k.sigma_angle, k.iters_bil, THREADS)
    n = int(host(r["n_tri"])[0])
    assert n == len(ref["triangles"])
    assert np.array_equal(host(r["triangles"])[:n], ref["triangles"])
    assert np.array_equal(host(r["halfedges"])[:3 * n], ref["halfedges"])
    check_points(host(r["points"]), ref["points"], pts)
    got = host(r["normals_T"])[:n].astype(np.float64)
    nan_r = np.isnan(ref["normals_T"]).any(-1)
    assert np.array_equal(np.isnan(got).any(-1), nan_r)
    ang = angle(got[~nan_r], ref["normals_T"][~nan_r])
    y32, y16 = yardsticks(ref, k, n)
    yard = (y32 if dtype_name == "float32" else y16)[~nan_r]
    print(f"config {config} {dtype_name} end to end: normal angle err p50 {np.median(ang):.2e} "
          f"p99 {np.percentile(ang, 99):.2e} max {ang.max():.2e}; exact arithmetic on the same "
          f"storage: p50 {np.median(yard):.2e} p99 {np.percentile(yard, 99):.2e} "
          f"max {yard.max():.2e}")
    if dtype_name == "float32":
        assert np.median(ang) <= NORMAL_ATOL
    assert np.percentile(ang, 99) <= max(1e-3, 3 * np.percentile(yard, 99))
    assert ang.max() <= 3 * yard.max() + 1e-4, (ang.max(), yard.max())


def test_deterministic(pl):
    pts, k = config_frame(1)
    x = to_dev(pts)
    a = pl.smooth_frame(x, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil,
                        k.sigma_length, k.sigma_angle, k.iters_bil)
    b = pl.smooth_frame(x, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil,
                        k.sigma_length, k.sigma_angle, k.iters_bil)
    n = int(host(a["n_tri"])[0])
    valid_rows = {"triangles": n, "halfedges": 3 * n, "normals_T": n}
    for key in ("tri_map", "triangles", "halfedges", "points", "filtered", "normals_T"):
        x, y = host(a[key]), host(b[key])
        if key in valid_rows:          # rows past |T| are never written
            x, y = x[:valid_rows[key]], y[:valid_rows[key]]
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8)), key


def test_errors_on_device(pl):
    import torch
    x = to_dev(random_grid(10, 12, 1))
    with pytest.raises(pl.PLError, match="PL_ERR_ALIAS"):
        pl.pl_laplacian(x, 3, 1.0, 1, out=x)
    with pytest.raises(pl.PLError, match="PL_ERR_KERNEL"):
        pl.pl_laplacian(x, 4, 1.0, 1)
    n, c = pl.pl_tri_normals(x)
    with pytest.raises(pl.PLError, match="PL_ERR_ALIAS"):
        pl.pl_bilateral(n, c, 3, 0.1, 0.1, 1, out=n)
    with pytest.raises(pl.PLError, match="PL_ERR_ARG"):
        pl.pl_bilateral(n, c, 3, -0.1, 0.1, 1)
    torch.cuda.synchronize()
