"""The fused single-frame entry point (pl_smooth_frame) through the C ABI:
every output equals the four single-frame calls (pl_mesh_opc, pl_laplacian,
pl_tri_normals, pl_bilateral with the gather) bit for bit, on the full
workload frames and on random grids, in float32 and float16, for every
placement of the mesh work among the launches (the emit riding a Laplacian
pass, the first bilateral pass, or a launch of its own; frames meshed by
whole rows), and with group labels equal to pl_group_assign's."""
import numpy as np
import pytest

from synth import KINDS, make_frame, random_grid, scene_planes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2007_12065_amd as pl
    return pl


def dev_t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def spec(pts, kl, lam, il, kb, sl, sa, ib):
    return dict(pts=dev_t(pts), kernel_lap=kl, lam=lam, iters_lap=il, kernel_bil=kb,
                sigma_length=sl, sigma_angle=sa, iters_bil=ib)


def kind_spec(kind, seed):
    k = KINDS[kind]
    return spec(make_frame(kind, seed), k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil,
                k.sigma_length, k.sigma_angle, k.iters_bil)


def single(pl, s, dtype):
    m = pl.pl_mesh_opc(s["pts"])
    pts = pl.pl_laplacian(s["pts"], s["kernel_lap"], s["lam"], s["iters_lap"])
    n, c = pl.pl_tri_normals(pts, dtype)
    f, nT = pl.pl_bilateral(n, c, s["kernel_bil"], s["sigma_length"], s["sigma_angle"],
                            s["iters_bil"], tri_map=m["tri_map"])
    return dict(m, points=pts, normals=f, centroids=c, normals_T=nT)


def assert_frame_equal(got, want, tag):
    n = int(host(want["n_tri"])[0])
    assert int(host(got["n_tri"])[0]) == n, tag
    rows = {"triangles": n, "halfedges": 3 * n, "normals_T": n}
    for key in ("tri_valid", "tri_map", "triangles", "halfedges", "points", "normals",
                "centroids", "normals_T"):
        a, b = host(got[key]), host(want[key])
        if key in rows:
            a, b = a[:rows[key]], b[:rows[key]]
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (tag, key)


class tuned:
    """Temporarily install single-frame tile shapes / fusion factors."""

    def __init__(self, pl, entries):
        self.pl, self.entries, self.saved = pl, entries, []

    def __enter__(self):
        # a single-frame entry is set for both frame size classes (stage + 4:
        # the small-frame entry; the random grids here are small frames)
        for stage, kernel, cfg in self.entries:
            for st in (stage, stage + 4) if stage in (0, 1) else (stage,):
                self.saved.append((st, kernel, self.pl.pl_tune_get(st, kernel)))
                self.pl.pl_tune_set(st, kernel, *cfg)

    def __exit__(self, *a):
        for stage, kernel, cfg in self.saved:
            self.pl.pl_tune_set(stage, kernel, *cfg)


@pytest.mark.parametrize("dtype_name", ["float32", "float16"])
@pytest.mark.parametrize("kind", ["rgbd_small", "rgbd", "lidar", "lidar128"])
def test_workload_frames(pl, kind, dtype_name):
    import torch
    dtype = getattr(torch, dtype_name)
    s = kind_spec(kind, 11)
    print(f"[case] pl_smooth_frame {kind} {dtype_name}", flush=True)
    assert_frame_equal(pl.pl_smooth_frame(s, dtype), single(pl, s, dtype), kind)


def random_specs():
    return [
        ("2x2", spec(random_grid(2, 2, 7), 3, 1.0, 2, 3, 0.1, 0.1, 2)),
        ("3x300 k7", spec(random_grid(3, 300, 8, nan_frac=0.2), 7, 0.5, 3, 7, 0.05, 0.3, 1)),
        ("37x150 k9", spec(random_grid(37, 150, 9, nan_frac=0.1), 9, 0.8, 5, 9, 0.2, 0.2, 3)),
        ("50x70 zero sweeps", spec(random_grid(50, 70, 10, nan_frac=0.3), 5, 1.0, 0, 3, 0.1, 0.1, 0)),
        ("9x600", spec(random_grid(9, 600, 11, nan_frac=0.05), 3, 1.0, 9, 5, 0.1, 0.1, 4)),
        ("70x515 all-NaN rows", spec(_nan_rows(random_grid(70, 515, 12)), 3, 1.0, 4, 3, 0.1, 0.1, 2)),
    ]


def _nan_rows(p):
    p = p.copy()
    p[10:14] = np.nan
    p[:, 256:258] = np.nan
    return p


# (stage, kernel, (rows, cols, fuse)) sets that move the emit around: the
# default (emit in the first bilateral pass at 3x3), a fused bilateral (one
# bilateral launch: the emit alone, or in the second Laplacian launch), and
# single-sweep Laplacian launches (the emit in the second Laplacian pass).
TUNINGS = {
    "default": [],
    "bilateral fused": [(1, 3, (8, 32, 2)), (1, 5, (8, 16, 3)), (1, 7, (4, 16, 2)), (1, 9, (4, 16, 2))],
    "one sweep per launch": [(0, 3, (16, 32, 1)), (0, 5, (8, 32, 1)), (1, 3, (8, 32, 1)), (1, 5, (8, 32, 1))],
    "laplacian fused, bilateral fused": [(0, 3, (16, 16, 8)), (0, 5, (8, 16, 5)), (0, 7, (8, 16, 5)),
                                         (0, 9, (4, 16, 5)), (1, 3, (16, 16, 4)), (1, 5, (8, 16, 4)),
                                         (1, 7, (4, 16, 3)), (1, 9, (4, 16, 3))],
    # tile widths that do not divide the mesh's 256-quad row segments: tiles
    # across a segment boundary when the gather ranks triangles from the codes
    "bilateral fused, odd widths": [(0, 3, (16, 24, 8)), (0, 5, (8, 40, 5)), (0, 7, (8, 16, 5)),
                                    (0, 9, (4, 16, 5)), (1, 3, (8, 24, 4)), (1, 5, (4, 20, 4)),
                                    (1, 7, (4, 12, 3)), (1, 9, (2, 12, 3))],
}


@pytest.mark.parametrize("dtype_name", ["float32", "float16"])
@pytest.mark.parametrize("tuning", list(TUNINGS))
def test_random_grids_every_launch_layout(pl, tuning, dtype_name):
    import torch
    dtype = getattr(torch, dtype_name)
    with tuned(pl, TUNINGS[tuning]):
        for tag, s in random_specs():
            print(f"[case] pl_smooth_frame {tag} {tuning} {dtype_name}", flush=True)
            assert_frame_equal(pl.pl_smooth_frame(s, dtype), single(pl, s, dtype),
                               (tag, tuning))


def test_row_meshed_frame(pl):
    """More than 8,192 row segments: the mesh runs as pl_mesh_opc's own two
    launches, the filters carry none of it."""
    import torch
    s = spec(random_grid(300, 7000, 13, nan_frac=0.05), 3, 1.0, 2, 3, 0.1, 0.1, 2)
    print("[case] pl_smooth_frame 300x7000", flush=True)
    assert_frame_equal(pl.pl_smooth_frame(s, torch.float32), single(pl, s, torch.float32),
                       "300x7000")


@pytest.mark.parametrize("dtype_name", ["float32", "float16"])
def test_groups(pl, dtype_name):
    import torch
    dtype = getattr(torch, dtype_name)
    k = KINDS["rgbd"]
    s = kind_spec("rgbd", 12)
    s.update(dominant=dev_t(scene_planes("rgbd", 12)), l_max=k.l_max, ang_min=k.ang_min)
    print(f"[case] pl_smooth_frame groups {dtype_name}", flush=True)
    got = pl.pl_smooth_frame(s, dtype)
    want = single(pl, s, dtype)
    assert_frame_equal(got, want, "groups")
    n = int(host(want["n_tri"])[0])
    labels = pl.pl_group_assign(want["points"], want["triangles"], want["normals_T"],
                                want["n_tri"], s["dominant"], k.l_max, k.ang_min)
    assert np.array_equal(host(got["groups"])[:n], host(labels)[:n])


def test_frame_plan_fused_equals_four_calls(pl):
    """FramePlan.run_fused (preallocated buffers, what the benchmark times)
    against FramePlan.run on the same frames, reusing the plans."""
    import torch
    k = KINDS["rgbd"]
    args = (k.M, k.N, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil, k.sigma_length,
            k.sigma_angle, k.iters_bil, torch.float32, torch.device("cuda:0"))
    a, b = pl.FramePlan(*args), pl.FramePlan(*args)
    for seed in (21, 22):
        x = dev_t(make_frame("rgbd", seed))
        a.run(x)
        b.run_fused(x)
        torch.cuda.synchronize()
        n = int(a.n_tri.item())
        assert int(b.n_tri.item()) == n
        for name in ("points", "tri_valid", "tri_map", "centroids", "filtered"):
            assert torch.equal(getattr(a, name).view(torch.uint8), getattr(b, name).view(torch.uint8)), name
        assert torch.equal(a.triangles[:n], b.triangles[:n])
        assert torch.equal(a.halfedges[:3 * n], b.halfedges[:3 * n])
        assert torch.equal(a.normals_T[:n].view(torch.uint8), b.normals_T[:n].view(torch.uint8))


@pytest.mark.parametrize("kind", ["rgbd_small", "rgbd", "lidar", "lidar128"])
def test_launch_layout(pl, kind):
    """The launches pl_smooth_frame issues under the committed tuning
    (profiles/tune.json): ceil(iters / fuse) filter launches per filter and
    nothing else, the mesh count in the first, the emit in exactly one (the
    second), the normals in the first bilateral pass and the gather in the
    last; at most 3 launches for the RGB-D frames."""
    import math
    import os

    import torch

    from paper_2007_12065_amd import tune
    k = KINDS[kind]
    saved = [(st, kk, pl.pl_tune_get(st, kk)) for st in range(6) for kk in (3, 5)]
    try:
        assert tune.load_cache(os.path.join(os.path.dirname(__file__), "..", "profiles", "tune.json")) > 0
        sl, sb = tune.frame_stages(k.M, k.N)
        fl, fb = pl.pl_tune_get(sl, k.kernel_lap)[2], pl.pl_tune_get(sb, k.kernel_bil)[2]
        plan = pl.FramePlan(k.M, k.N, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil, k.sigma_length,
                            k.sigma_angle, k.iters_bil, torch.float32, torch.device("cuda:0"))
        events = [torch.cuda.Event(enable_timing=True) for _ in range(16)]
        kinds = plan.run_fused_events(dev_t(make_frame(kind, 3)), events)
        torch.cuda.synchronize()
    finally:
        for st, kk, cfg in saved:
            pl.pl_tune_set(st, kk, *cfg)
    nl, nb = math.ceil(k.iters_lap / fl), math.ceil(k.iters_bil / fb)
    print(f"[case] {kind}: launches {[hex(x) for x in kinds]}", flush=True)
    assert len(kinds) == nl + nb
    assert kinds[1] & pl.PL_LAUNCH_MESH_EMIT
    lap = [x for x in kinds if x & pl.PL_LAUNCH_LAPLACIAN]
    bil = [x for x in kinds if x & pl.PL_LAUNCH_BILATERAL]
    assert len(lap) == nl and len(bil) == nb
    assert kinds[0] & pl.PL_LAUNCH_MESH_COUNT
    assert sum(bool(x & pl.PL_LAUNCH_MESH_EMIT) for x in kinds) == 1
    assert bil[0] & pl.PL_LAUNCH_NORMALS and bil[-1] & pl.PL_LAUNCH_GATHER
    assert sum((x >> 8) & 0xff for x in lap) == k.iters_lap
    assert sum((x >> 8) & 0xff for x in bil) == k.iters_bil
    if kind.startswith("rgbd"):
        assert len(kinds) <= 3
