"""Pins for the oracle's group assignment (Sec. 7.1, Alg. 4).

Hand-worked triangles, the strict comparisons of Alg. 4 (first maximum wins,
an edge exactly l_max long is kept), an FP64 brute force of the definition
written with numpy, equivariance under permutations, and a two-plane grid
whose labels are known exactly."""
import math

import numpy as np

import synth

DOM = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, 1.0, 0.0]], dtype=np.float32)


def _tri_pts(legs):
    """Right triangles in the plane z = 0, one per leg length, each with its
    own three points: (0,0,0), (a,0,0), (0,a,0) offset along x."""
    pts, tris = [], []
    for i, a in enumerate(legs):
        o = np.array([10.0 * i, 0.0, 0.0])
        pts += [o, o + [a, 0.0, 0.0], o + [0.0, a, 0.0]]
        tris.append([3 * i, 3 * i + 1, 3 * i + 2])
    return np.array(pts, dtype=np.float32), np.array(tris, dtype=np.int32)


def test_hand_worked(orc):
    # legs 0.03: longest edge 0.0424 <= 0.05; legs 0.04: hypotenuse 0.0566 > 0.05
    pts, tris = _tri_pts([0.03, 0.04] + [0.03] * 5)
    s10, c10 = math.sin(math.radians(10)), math.cos(math.radians(10))
    s20, c20 = math.sin(math.radians(20)), math.cos(math.radians(20))
    normals = np.array([
        [0, 0, 1],            # aligned with dominant 1
        [0, 0, 1],            # long edge
        [s10, 0, c10],        # 10 deg off: cos = 0.985 >= 0.96
        [s20, 0, c20],        # 20 deg off: cos = 0.940 < 0.96
        [0, 0, -1],           # antiparallel: best is dominant 0 with 0 < 0.96
        [np.nan, 0, 0],       # NaN normal matches nothing
        [0, 0.96, 0.28],      # closest to dominant 2 (0.96 exactly at the threshold)
    ], dtype=np.float32)
    g = orc.group_assign(pts, tris, normals, DOM, 0.05, 0.96)
    # 0.96 and 0.28 are not exact in float32: the float32 product decides
    exp6 = 2 if np.float32(0.96) * np.float32(1.0) >= np.float32(0.96) else 255
    assert g.tolist() == [1, 255, 1, 255, 255, 255, exp6]
    # with ang_min = -1 nothing is below the threshold: the 20 deg triangle
    # keeps dominant 1 and the antiparallel one its first maximum (0)
    g = orc.group_assign(pts, tris, normals, DOM, 0.05, -1.0)
    assert g.tolist() == [1, 255, 1, 1, 0, 255, 2]


def test_edge_equal_to_l_max_is_kept(orc):
    # edges 0.5, sqrt(0.125), sqrt(0.125): the longest is exactly 0.5
    pts = np.array([[0, 0, 0], [0.5, 0, 0], [0.25, 0.25, 0]], dtype=np.float32)
    tris = np.array([[0, 1, 2]], dtype=np.int32)
    n = np.array([[0, 0, 1]], dtype=np.float32)
    assert orc.group_assign(pts, tris, n, DOM, 0.5, 0.9).tolist() == [1]
    assert orc.group_assign(pts, tris, n, DOM, np.nextafter(np.float32(0.5), 0), 0.9).tolist() == [255]
    # every vertex order of the same triangle gives the same label
    for perm in ([1, 2, 0], [2, 0, 1], [0, 2, 1]):
        assert orc.group_assign(pts, tris[:, perm], n, DOM, 0.5, 0.9).tolist() == [1]


def test_first_maximum_wins(orc):
    pts, tris = _tri_pts([0.01] * 2)
    n = np.array([[0, 0, 1], [1 / math.sqrt(2), 1 / math.sqrt(2), 0]], dtype=np.float32)
    dup = np.array([[0, 1, 0], [0, 0, 1], [0, 0, 1], [0, 0, 1]], dtype=np.float32)
    assert orc.group_assign(pts, tris, n, dup, 1.0, 0.5)[0] == 1
    # (1,1,0)/sqrt2 is equally similar to x and y: the first of them wins
    xy = np.array([[0, 1, 0], [1, 0, 0]], dtype=np.float32)
    assert orc.group_assign(pts, tris, n, xy, 1.0, 0.5)[1] == 0
    assert orc.group_assign(pts, tris, n, xy[::-1].copy(), 1.0, 0.5)[1] == 0


def test_degenerate_inputs(orc):
    pts, tris = _tri_pts([0.01] * 3)
    n = np.tile(np.array([[0, 0, 1]], dtype=np.float32), (3, 1))
    # no dominant normal: every label is the sentinel
    assert orc.group_assign(pts, tris, n, np.zeros((0, 3), np.float32), 1.0, 0.5).tolist() == [255] * 3
    # a vertex index outside the point array gives the sentinel
    bad = tris.copy()
    bad[0, 1] = -1
    bad[2, 2] = len(pts)
    assert orc.group_assign(pts, bad, n, DOM, 1.0, 0.5).tolist() == [255, 1, 255]
    # no triangle
    assert orc.group_assign(pts, tris[:0], n[:0], DOM, 1.0, 0.5).shape == (0,)
    # a NaN vertex makes its edges NaN, which no length test passes
    p2 = pts.copy()
    p2[4] = np.nan
    assert orc.group_assign(p2, tris, n, DOM, 1.0, 0.5).tolist() == [1, 255, 1]


def _random_case(seed, n_tri=20000, l=12):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-0.05, 0.05, size=(3 * n_tri, 3)).astype(np.float32)
    tris = rng.permutation(3 * n_tri).astype(np.int32).reshape(n_tri, 3)
    n = rng.normal(size=(n_tri, 3))
    n = (n / np.linalg.norm(n, axis=1, keepdims=True)).astype(np.float32)
    d = rng.normal(size=(l, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    return pts, tris, n, d


def test_fp64_brute_force(orc):
    """The definition in float64 with numpy (argmax takes the first maximum)
    agrees wherever no comparison is within 1e-5 of its threshold."""
    pts, tris, n, d = _random_case(5)
    l_max, ang_min = 0.08, 0.6
    g = orc.group_assign(pts, tris, n, d, l_max, ang_min)
    P = pts.astype(np.float64)[tris]
    edges = np.stack([np.linalg.norm(P[:, 1] - P[:, 0], axis=1),
                      np.linalg.norm(P[:, 2] - P[:, 1], axis=1),
                      np.linalg.norm(P[:, 0] - P[:, 2], axis=1)], axis=1).max(axis=1)
    sims = n.astype(np.float64) @ d.astype(np.float64).T
    best = sims.max(axis=1)
    second = np.sort(sims, axis=1)[:, -2]
    exp = np.where((edges > np.float64(np.float32(l_max))) | (best < np.float64(np.float32(ang_min))),
                   255, sims.argmax(axis=1))
    clear = ((np.abs(edges - np.float32(l_max)) > 1e-5) & (np.abs(best - np.float32(ang_min)) > 1e-5)
             & (best - second > 1e-5))
    assert clear.mean() > 0.99
    assert np.array_equal(g[clear], exp[clear])
    # every label class occurs
    assert (g == 255).any() and len(np.unique(g)) > d.shape[0] // 2


def test_permutation_equivariance(orc):
    pts, tris, n, d = _random_case(6, n_tri=5000, l=6)
    g = orc.group_assign(pts, tris, n, d, 0.08, 0.3)
    rng = np.random.default_rng(1)
    pt = rng.permutation(len(tris))
    assert np.array_equal(orc.group_assign(pts, tris[pt], n[pt], d, 0.08, 0.3), g[pt])
    pd = rng.permutation(len(d))
    g2 = orc.group_assign(pts, tris, n, d[pd], 0.08, 0.3)
    inv = np.argsort(pd)  # new index k holds old dominant pd[k]; old j sits at inv[j]
    mapped = np.where(g == 255, 255, inv[np.minimum(g, len(d) - 1)])
    sims = np.sort(n.astype(np.float64) @ d.astype(np.float64).T, axis=1)
    no_tie = sims[:, -1] - sims[:, -2] > 1e-6
    assert np.array_equal(g2[no_tie], mapped[no_tie])


def test_two_plane_grid(orc):
    """A 20 x 12 grid at 1 cm spacing: rows 0-9 on the plane z = 2, rows 10-19
    on z = 2.5.  Every triangle within a plane faces the camera, (0, 0, -1);
    the quad row joining the planes has 0.5 m edges."""
    M, N = 20, 12
    v, u = np.meshgrid(np.arange(N, dtype=np.float64), np.arange(M, dtype=np.float64))
    z = np.where(u < 10, 2.0, 2.5)
    g = np.stack([0.01 * v, 0.01 * u, z], axis=-1).astype(np.float32)
    tri_map, T = orc.mesh(g)
    normals, _ = orc.tri_normals(g)
    nT = orc.gather(normals, tri_map, len(T))
    dom = np.array([[0, 1, 0], [0, 0, -1]], dtype=np.float32)
    lab = orc.group_assign(g, T, nT.astype(np.float32), dom, 0.05, 0.96)
    assert len(lab) == 2 * (M - 1) * (N - 1)
    rows = np.arange(len(lab)) // (2 * (N - 1))  # quad row of each triangle (all are valid)
    assert np.all(lab[rows == 9] == 255)
    assert np.all(lab[rows != 9] == 1)


def test_scene_planes_match_smoothed_scene(orc):
    """On the 120x160 scene after smoothing, the floor's normal claims most
    triangles: the orientation of scene_planes agrees with the mesh winding."""
    k = synth.KINDS["rgbd_small"]
    p = synth.make_frame("rgbd_small", 3)
    r = orc.pipeline(p, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil, k.sigma_length,
                     k.sigma_angle, k.iters_bil, threads=4)
    lab = orc.group_assign(r["points"].astype(np.float32), r["triangles"],
                           r["normals_T"].astype(np.float32), synth.scene_planes("rgbd_small", 3),
                           k.l_max, k.ang_min)
    assert np.mean(lab == 0) > 0.9
    # flipping every dominant normal leaves almost nothing assigned
    lab2 = orc.group_assign(r["points"].astype(np.float32), r["triangles"],
                            r["normals_T"].astype(np.float32), -synth.scene_planes("rgbd_small", 3),
                            k.l_max, k.ang_min)
    assert np.mean(lab2 != 255) < 0.01
