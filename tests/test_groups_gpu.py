"""GPU parity of group assignment (Sec. 7.1, Alg. 4) through the C ABI.

The labels are integers decided in float32, so on identical float32 inputs
the HIP kernel must match the oracle bit for bit: on the smoothed synthetic
frames at their real sizes (float32 and float16 normals), on random
triangle soups with 1, 12 and 254 dominant normals and ragged counts, and on
the degenerate cases (no points, no dominant normal, out-of-range indices,
NaN vertices and normals, |T| beyond the capacity or negative).  The whole
GPU path (mesh, smoothing, normals, groups) is also compared with the whole
oracle path wherever no comparison sits within the float32 path's error of
its threshold.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

UNTOUCHED = 77


@pytest.fixture(scope="module")
def pl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2007_12065_amd as pl
    return pl


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def say(*a):
    print("[case]", *a, flush=True)


def gpu_groups(pl, pts, tris, normals, n_tri, dom, l_max, ang_min, cap=None):
    """Labels from the kernel; `out` is prefilled so rows the call must not
    write can be checked."""
    import torch
    cap = len(tris) if cap is None else cap
    out = torch.full((max(cap, 1),), UNTOUCHED, dtype=torch.uint8, device="cuda:0")
    g = pl.pl_group_assign(to_dev(pts), to_dev(tris[:cap]), to_dev(normals[:cap]),
                           to_dev(np.array([n_tri], dtype=np.int32)),
                           None if dom is None or len(dom) == 0 else to_dev(dom),
                           l_max, ang_min, out=out)
    torch.cuda.synchronize()
    return g.cpu().numpy()


def check(pl, pts, tris, normals, n_tri, dom, l_max, ang_min, cap=None):
    cap = len(tris) if cap is None else cap
    got = gpu_groups(pl, pts, tris, normals, n_tri, dom, l_max, ang_min, cap)
    n = min(max(n_tri, 0), cap)
    ref = oracle.group_assign(pts, tris[:n], normals[:n].astype(np.float32),
                              np.zeros((0, 3), np.float32) if dom is None else dom, l_max, ang_min)
    assert np.array_equal(got[:n], ref), f"{np.count_nonzero(got[:n] != ref)} labels differ"
    assert np.all(got[n:cap] == UNTOUCHED)
    return got[:n]


@pytest.mark.parametrize("kind", ["rgbd_small", "rgbd", "lidar", "lidar128"])
def test_scene_parity(pl, orc, kind):
    k = synth.KINDS[kind]
    p = synth.make_frame(kind, 21)
    r = orc.pipeline(p, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil, k.sigma_length,
                     k.sigma_angle, k.iters_bil, threads=8)
    pts = r["points"].astype(np.float32)
    T = r["triangles"]
    dom = synth.scene_planes(kind, 21)
    for nd in (np.float32, np.float16):
        say("groups scene", kind, p.shape, nd.__name__, len(T))
        nT = r["normals_T"].astype(nd)
        g = check(pl, pts, T, nT, len(T), dom, k.l_max, k.ang_min)
        assert (g != 255).mean() > 0.5


@pytest.mark.parametrize("l", [1, 12, 254])
def test_random_parity_ragged(pl, l):
    rng = np.random.default_rng(100 + l)
    cap = 5003
    pts = rng.uniform(-0.05, 0.05, size=(3 * cap, 3)).astype(np.float32)
    pts[rng.choice(len(pts), 40, replace=False)] = np.nan
    tris = rng.integers(0, len(pts), size=(cap, 3)).astype(np.int32)
    bad = rng.choice(cap, 30, replace=False)
    tris[bad[:10], 0] = -1
    tris[bad[10:20], 1] = len(pts)
    tris[bad[20:], 2] = np.iinfo(np.int32).max
    n = rng.normal(size=(cap, 3))
    n = (n / np.linalg.norm(n, axis=1, keepdims=True)).astype(np.float32)
    n[rng.choice(cap, 25, replace=False)] = np.nan
    d = rng.normal(size=(l, 3))
    d = (d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)
    for n_tri in (cap, cap - 1, cap - 2, cap - 3, 4, 3, 1, 0, cap + 10, -5):
        say("groups random l", l, "n_tri", n_tri)
        check(pl, pts, tris, n, n_tri, d, 0.08, 0.2)
    # a capacity that is not a multiple of the four triangles a thread takes
    say("groups random l", l, "cap 4097")
    check(pl, pts, tris, n, 4097, d, 0.08, 0.2, cap=4097)
    for nd in (np.float16,):
        say("groups random f16 l", l)
        check(pl, pts, tris, n.astype(nd), cap, d, 0.08, 0.2)
    say("groups random inf l_max l", l)
    check(pl, pts, tris, n, cap, d, float("inf"), -2.0)


def test_degenerate(pl):
    rng = np.random.default_rng(7)
    pts = rng.uniform(0, 0.01, size=(30, 3)).astype(np.float32)
    tris = rng.integers(0, 30, size=(10, 3)).astype(np.int32)
    n = np.tile(np.array([[0, 0, 1]], np.float32), (10, 1))
    d = np.array([[0, 0, 1]], np.float32)
    say("groups no dominant normal")
    assert np.all(check(pl, pts, tris, n, 10, None, 1.0, 0.5) == 255)
    say("groups no points")
    assert np.all(gpu_groups(pl, pts[:0], tris, n, 10, d, 1.0, 0.5)[:10] == 255)
    say("groups all assigned")
    assert np.all(check(pl, pts, tris, n, 10, d, 1.0, 0.5) == 0)
    say("groups empty capacity")
    import torch
    out = torch.full((1,), UNTOUCHED, dtype=torch.uint8, device="cuda:0")
    pl.pl_group_assign(to_dev(pts), to_dev(tris[:0]), to_dev(n[:0]),
                       to_dev(np.array([5], np.int32)), to_dev(d), 1.0, 0.5, out=out)
    torch.cuda.synchronize()
    assert out.item() == UNTOUCHED


def test_whole_path_against_oracle_path(pl, orc):
    """Mesh, smoothing, normals and groups on the GPU (float32 and float16
    normals) against the same on the oracle: identical T, and identical labels
    on every triangle whose comparisons the differences between the two
    paths cannot flip.  For unit vectors |n.d - n'.d| <= |n - n'|, and an
    edge moves by at most the sum of its endpoints' displacements; a
    triangle counts as decided when, in the oracle's FP64 values, the best
    similarity clears the runner-up and ang_min, and every edge clears l_max,
    by more than those differences (plus 1e-6 for float32 rounding)."""
    import torch
    kind = "rgbd"
    k = synth.KINDS[kind]
    p = synth.make_frame(kind, 1001)
    r = orc.pipeline(p, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil, k.sigma_length,
                     k.sigma_angle, k.iters_bil, threads=8)
    T = r["triangles"]
    dom = synth.scene_planes(kind, 1001)
    P = r["points"].reshape(-1, 3)
    pairs = ((0, 1), (1, 2), (2, 0))
    e = np.stack([np.linalg.norm(P[T[:, a]] - P[T[:, b]], axis=1) for a, b in pairs], axis=1)
    srt = np.sort(r["normals_T"] @ dom.astype(np.float64).T, axis=1)
    lm = float(np.float32(k.l_max))
    amin = float(np.float32(k.ang_min))
    ref = oracle.group_assign(r["points"].astype(np.float32), T,
                              r["normals_T"].astype(np.float32), dom, k.l_max, k.ang_min)
    for nd in (torch.float32, torch.float16):
        say("groups whole path 480x640", nd)
        plan = pl.FramePlan(k.M, k.N, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil,
                            k.sigma_length, k.sigma_angle, k.iters_bil, normal_dtype=nd)
        plan.run(to_dev(p))
        plan.run_groups(to_dev(dom), k.l_max, k.ang_min)
        torch.cuda.synchronize()
        n = int(plan.n_tri.item())
        assert n == len(T)
        assert np.array_equal(plan.triangles[:n].cpu().numpy(), T)
        got = plan.groups[:n].cpu().numpy()
        dp = np.linalg.norm(plan.points.cpu().numpy().reshape(-1, 3).astype(np.float64) - P, axis=1)
        dn = np.linalg.norm(plan.normals_T[:n].cpu().numpy().astype(np.float64) - r["normals_T"],
                            axis=1)
        de = np.stack([dp[T[:, a]] + dp[T[:, b]] for a, b in pairs], axis=1) + 1e-6 * lm
        m = dn + 1e-6
        decided = (np.all(np.abs(e - lm) > de, axis=1) & (srt[:, -1] - srt[:, -2] > 2 * m)
                   & (np.abs(srt[:, -1] - amin) > m))
        assert decided.mean() > 0.98
        assert np.array_equal(got[decided], ref[decided]), np.count_nonzero(got[decided] != ref[decided])


def _batch_specs(with_groups):
    """Mixed frames; every other one asks for group assignment, with 3
    scene planes, none, one or 254 dominant normals."""
    from synth import KINDS, make_frame, random_grid, scene_planes
    rng = np.random.default_rng(5)
    specs = []
    frames = [("rgbd_small", 1), ("rgbd", 2), ("lidar", 3), ("lidar128", 4), ("rgbd", 5)]
    for j, (kind, seed) in enumerate(frames):
        k = KINDS[kind]
        s = dict(pts=to_dev(make_frame(kind, seed)), kernel_lap=k.kernel_lap, lam=k.lam,
                 iters_lap=k.iters_lap, kernel_bil=k.kernel_bil, sigma_length=k.sigma_length,
                 sigma_angle=k.sigma_angle, iters_bil=k.iters_bil)
        if with_groups and j != 3:
            s.update(dominant=to_dev(scene_planes(kind, seed)), l_max=k.l_max, ang_min=k.ang_min)
        specs.append(s)
    for j, (M, N, l) in enumerate([(2, 2, 1), (37, 150, 0), (50, 70, 254), (9, 600, 5)]):
        s = dict(pts=to_dev(random_grid(M, N, 40 + j, nan_frac=0.1)), kernel_lap=3, lam=1.0,
                 iters_lap=2, kernel_bil=5, sigma_length=0.1, sigma_angle=0.1, iters_bil=2)
        if with_groups:
            d = rng.normal(size=(l, 3))
            if l:
                d[0] = (0.0, 0.0, -1.0)
            d = (d / np.maximum(np.linalg.norm(d, axis=1, keepdims=True), 1e-30)).astype(np.float32)
            s.update(dominant=to_dev(d.reshape(l, 3)), l_max=0.1, ang_min=0.9)
        specs.append(s)
    return specs


def _single_call_groups(pl, o, s):
    return pl.pl_group_assign(o["points"], o["triangles"], o["normals_T"], o["n_tri"],
                              s["dominant"], s["l_max"], s["ang_min"])


@pytest.mark.parametrize("dtype_name", ["float32", "float16"])
def test_batch_groups_equal_single_call(pl, dtype_name):
    """The batch's group stage gives every frame the labels pl_group_assign
    gives on that frame's (bitwise identical) outputs; frames without groups
    are unaffected, and the plan runs repeatedly and from a bounded graph."""
    import torch
    dtype = getattr(torch, dtype_name)
    specs = _batch_specs(True)
    say("batch groups", len(specs), "frames", dtype_name)
    b = pl.Batch(specs, dtype)
    b.run()
    torch.cuda.synchronize()
    plain = pl.Batch(_batch_specs(False), dtype)
    plain.run()
    torch.cuda.synchronize()
    for i, (o, s) in enumerate(zip(b.outputs, specs)):
        n = int(o["n_tri"].item())
        assert torch.equal(o["normals_T"][:n], plain.outputs[i]["normals_T"][:n]), i
        if "dominant" not in s:
            assert "groups" not in o
            continue
        want = _single_call_groups(pl, o, s)
        torch.cuda.synchronize()
        assert torch.equal(o["groups"][:n], want[:n]), i
    # active subset from a bounded graph: inactive frames keep their labels
    say("batch groups bounded graph")
    for o in b.outputs:
        if "groups" in o:
            o["groups"].fill_(UNTOUCHED)
    act = torch.zeros(len(specs), dtype=torch.uint8, device="cuda:0")
    act[[0, 2, 6]] = 1
    b.capture(act, max_active=3)
    for _ in range(2):
        b.replay(3)
        torch.cuda.synchronize()
    for i, (o, s) in enumerate(zip(b.outputs, specs)):
        if "groups" not in o:
            continue
        n = int(o["n_tri"].item())
        if i in (0, 2, 6):
            assert torch.equal(o["groups"][:n], _single_call_groups(pl, o, s)[:n]), i
        else:
            assert bool((o["groups"] == UNTOUCHED).all()), i


def test_one_shot_batch_groups(pl):
    import torch
    specs = _batch_specs(True)[:3]
    say("one-shot batch groups")
    outs = pl.pl_smooth_batch(specs)
    torch.cuda.synchronize()
    for o, s in zip(outs, specs):
        n = int(o["n_tri"].item())
        assert torch.equal(o["groups"][:n], _single_call_groups(pl, o, s)[:n])
