"""The batched path (one launch per stage over mixed frames) gives
every frame exactly its single-frame result, replays correctly from a HIP
graph, and float32 outputs do not depend on tile shapes or sweep fusion."""
import numpy as np
import pytest

from synth import KINDS, make_frame, random_grid

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


def mixed_specs():
    out = []
    for kind, seed in [("rgbd_small", 1), ("rgbd", 2), ("lidar", 3), ("lidar128", 4), ("rgbd", 5)]:
        k = KINDS[kind]
        out.append(spec(make_frame(kind, seed), k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil,
                        k.sigma_length, k.sigma_angle, k.iters_bil))
    out.append(spec(random_grid(2, 2, 7), 3, 1.0, 2, 3, 0.1, 0.1, 2))
    out.append(spec(random_grid(3, 300, 8, nan_frac=0.2), 7, 0.5, 3, 7, 0.05, 0.3, 1))
    out.append(spec(random_grid(37, 150, 9, nan_frac=0.1), 9, 0.8, 5, 9, 0.2, 0.2, 3))
    out.append(spec(random_grid(50, 70, 10, nan_frac=0.3), 5, 1.0, 0, 3, 0.1, 0.1, 0))
    out.append(spec(random_grid(9, 600, 11, nan_frac=0.05), 3, 1.0, 9, 5, 0.1, 0.1, 4))
    return out


def single(pl, s, dtype):
    """The four single-frame ABI calls with the same parameters."""
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


@pytest.mark.parametrize("dtype_name", ["float32", "float16"])
def test_batch_equals_single_frames(pl, dtype_name):
    import torch
    dtype = getattr(torch, dtype_name)
    specs = mixed_specs()
    print("[case] batch of", len(specs), "frames,", dtype_name, flush=True)
    b = pl.Batch(specs, dtype)
    b.run()
    torch.cuda.synchronize()
    for i, s in enumerate(specs):
        assert_frame_equal(b.outputs[i], single(pl, s, dtype), f"frame {i}")
    b.close()


def test_batch_more_frames_than_the_lds_table(pl):
    # past 256 frames the tile lookup searches the prefix sums in global
    # memory; frames on both sides of that bound, with a sparse active mask
    import torch
    rng = np.random.default_rng(12)
    specs = []
    for i in range(300):
        M, N = int(rng.integers(2, 14)), int(rng.integers(2, 70))
        k = int(rng.choice([3, 5]))
        specs.append(spec(random_grid(M, N, 500 + i, nan_frac=0.1), k, 1.0, int(rng.integers(0, 4)),
                          k, 0.1, 0.1, int(rng.integers(0, 3))))
    print("[case] batch of 300 small frames", flush=True)
    b = pl.Batch(specs, torch.float32)
    mask = torch.tensor([1 if i % 3 == 0 else 0 for i in range(300)], dtype=torch.uint8,
                        device="cuda:0")
    b.run(mask)
    torch.cuda.synchronize()
    for i in list(range(0, 30, 3)) + list(range(249, 300, 3)):
        assert_frame_equal(b.outputs[i], single(pl, specs[i], torch.float32), f"frame {i}")
    b.close()


@pytest.mark.parametrize("dtype_name", ["float32", "float16"])
def test_batch_of_full_size_frames_equals_single_frames(pl, dtype_name):
    # four 480x640 (3x3) and four 128x2048 (5x5) frames: thousands of tiles
    # per radius in each batched launch
    import torch
    dtype = getattr(torch, dtype_name)
    specs = []
    for kind, seed in [("rgbd", 41), ("rgbd", 42), ("rgbd", 43), ("rgbd", 44),
                       ("lidar128", 45), ("lidar128", 46), ("lidar128", 47), ("lidar128", 48)]:
        k = KINDS[kind]
        specs.append(spec(make_frame(kind, seed), k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil,
                          k.sigma_length, k.sigma_angle, k.iters_bil))
    print("[case] full-size batch,", dtype_name, flush=True)
    b = pl.Batch(specs, dtype)
    b.run()
    torch.cuda.synchronize()
    for i, sp in enumerate(specs):
        assert_frame_equal(b.outputs[i], single(pl, sp, dtype), f"frame {i}")
    b.close()


@pytest.mark.parametrize("dtype_name", ["float32", "float16"])
def test_smooth_batch_one_shot(pl, dtype_name):
    # pl_smooth_batch (create, run, release) gives the single-frame results
    import torch
    dtype = getattr(torch, dtype_name)
    specs = mixed_specs()[:7]
    print("[case] one-shot batch,", dtype_name, flush=True)
    outs = pl.pl_smooth_batch(specs, dtype)
    torch.cuda.synchronize()
    for i, sp in enumerate(specs):
        assert_frame_equal(outs[i], single(pl, sp, dtype), f"one-shot frame {i}")


def test_batch_graph_replay(pl):
    import torch
    specs = mixed_specs()[:6]
    b = pl.Batch(specs, torch.float32)
    b.run()
    torch.cuda.synchronize()
    want = [{k: (v.clone() if v is not None else None) for k, v in o.items()} for o in b.outputs]
    b.capture()
    other = dev_t(make_frame("rgbd", 77))
    for rep in range(3):
        print("[case] graph replay", rep, flush=True)
        for o in b.outputs:                      # poison every output first
            for v in o.values():
                if v is not None:
                    v.fill_(-7) if v.dtype != torch.uint8 else v.fill_(9)
        pl.pl_laplacian(other, 3, 1.0, 2)        # unrelated eager work between replays
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        for i in range(len(specs)):
            assert_frame_equal(b.outputs[i], want[i], f"replay {rep} frame {i}")
    b.close()


def test_batch_active_subset(pl):
    # frames left out of a run keep their previous outputs; the others are
    # recomputed exactly
    import torch
    specs = mixed_specs()
    b = pl.Batch(specs, torch.float32)
    b.run()
    torch.cuda.synchronize()
    want = [{k: (v.clone() if v is not None else None) for k, v in o.items()} for o in b.outputs]
    mask = torch.tensor([i % 2 for i in range(len(specs))], dtype=torch.uint8, device="cuda:0")
    for o in b.outputs:
        o["normals_T"].fill_(-3)
        o["points"].fill_(-3)
    b.run(mask)
    torch.cuda.synchronize()
    for i, o in enumerate(b.outputs):
        if i % 2:
            assert_frame_equal(o, want[i], f"active frame {i}")
        else:
            assert bool((o["normals_T"] == -3).all()) and bool((o["points"] == -3).all())
    # a graph captured with the mask follows the mask's contents at replay
    b.capture(mask)
    mask.fill_(1)
    torch.cuda.synchronize()
    b.replay()
    torch.cuda.synchronize()
    for i, o in enumerate(b.outputs):
        assert_frame_equal(o, want[i], f"replayed frame {i}")
    b.close()


def test_batch_bounded_graphs(pl):
    # graphs sized for at most k active frames give the full run's bits for
    # every subset of at most k frames; a replay needs a covering bound
    import torch
    specs = mixed_specs()
    b = pl.Batch(specs, torch.float32)
    b.run()
    torch.cuda.synchronize()
    want = [{k: (v.clone() if v is not None else None) for k, v in o.items()} for o in b.outputs]
    mask = torch.zeros(len(specs), dtype=torch.uint8, device="cuda:0")
    for k in (1, 3):
        b.capture(mask, max_active=k)
    with pytest.raises(pl.PLError):
        b.replay(n_active=4)                      # no bound >= 4 captured
    for subset in ([1], [4], [0, 2, 3], [1, 3, 8], [2, 7]):
        print("[case] bounded replay, active", subset, flush=True)
        for o in b.outputs:
            o["normals_T"].fill_(-5)
            o["points"].fill_(-5)
        mask.zero_()
        mask[subset] = 1
        torch.cuda.synchronize()
        b.replay(n_active=len(subset))
        torch.cuda.synchronize()
        for i in subset:
            assert_frame_equal(b.outputs[i], want[i], f"bounded frame {i}")
        for i in set(range(len(specs))) - set(subset):
            assert bool((b.outputs[i]["points"] == -5).all())
    b.close()


def test_batch_runs_repeatedly(pl):
    import torch
    specs = mixed_specs()[5:]
    b = pl.Batch(specs, torch.float32)
    b.run()
    torch.cuda.synchronize()
    first = [host(o["normals_T"]).copy() for o in b.outputs]
    for _ in range(3):
        b.run()
    torch.cuda.synchronize()
    for f, o in zip(first, b.outputs):
        assert np.array_equal(f.view(np.uint8), host(o["normals_T"]).view(np.uint8))
    b.close()


def test_tiling_invariance(pl):
    import torch
    pts = dev_t(make_frame("lidar", 31))
    ref_lap = host(pl.pl_laplacian(pts, 5, 1.0, 4)).copy()
    n, c = pl.pl_tri_normals(dev_t(make_frame("rgbd", 32)))
    ref_bil = host(pl.pl_bilateral(n, c, 3, 0.1, 0.1, 3)[0]).copy()
    # the 64 x 1024 frame reads the small-frame entry
    saved = [pl.pl_tune_get(4, 5), pl.pl_tune_get(1, 3), pl.pl_tune_get(1, 5)]
    try:
        for th, tw, fu in [(4, 64, 1), (16, 16, 2), (8, 128, 4), (32, 8, 3)]:
            print("[case] laplacian tile", th, tw, fu, flush=True)
            pl.pl_tune_set(4, 5, th, tw, fu)
            assert np.array_equal(host(pl.pl_laplacian(pts, 5, 1.0, 4)).view(np.uint8),
                                  ref_lap.view(np.uint8))
        for th, tw, fu in [(4, 64, 1), (16, 16, 2), (8, 32, 3), (2, 128, 1), (16, 32, 1), (16, 32, 2)]:
            print("[case] bilateral tile", th, tw, fu, flush=True)
            pl.pl_tune_set(1, 3, th, tw, fu)
            assert np.array_equal(host(pl.pl_bilateral(n, c, 3, 0.1, 0.1, 3)[0]).view(np.uint8),
                                  ref_bil.view(np.uint8))
        # a 1100 x 1100 frame (thousands of tiles), 3x3 and 5x5
        big = dev_t(random_grid(1100, 1100, 33, nan_frac=0.05, noise=0.01))
        nb, cb = pl.pl_tri_normals(big)
        for k in (3, 5):
            pl.pl_tune_set(1, k, 8, 32, 1)
            refb = host(pl.pl_bilateral(nb, cb, k, 0.1, 0.1, 2)[0]).copy()
            for th, tw, fu in [(16, 32, 1), (16, 32, 2), (4, 64, 1), (16, 16, 2)]:
                print(f"[case] bilateral {k}x{k} 1100x1100 tile", th, tw, fu, flush=True)
                pl.pl_tune_set(1, k, th, tw, fu)
                assert np.array_equal(host(pl.pl_bilateral(nb, cb, k, 0.1, 0.1, 2)[0]).view(np.uint8),
                                      refb.view(np.uint8))
            pl.pl_tune_set(1, k, *saved[1 if k == 3 else 2])
    finally:
        pl.pl_tune_set(4, 5, *saved[0])
        pl.pl_tune_set(1, 3, *saved[1])
        pl.pl_tune_set(1, 5, *saved[2])


def test_batch_overlap_rejected(pl):
    import torch
    s = mixed_specs()[5]
    b = pl.Batch([s], torch.float32)
    arr = (pl.PLFrame * 2)()
    arr[0] = b._frames[0]
    arr[1] = b._frames[0]                       # same outputs twice
    assert pl._lib.pl_batch_workspace(arr, 2, 0) == 0
    assert "overlap" in pl._lib.pl_last_error().decode()
    b.close()


def test_autotune_installs_a_candidate_and_keeps_results(pl, tmp_path):
    import torch
    from paper_2007_12065_amd import tune
    pts = dev_t(make_frame("rgbd_small", 3))
    ref = host(pl.pl_laplacian(pts, 3, 1.0, 3)).copy()
    ls, bs = tune.frame_stages(120, 160)          # a small frame: the *_SMALL entries
    assert (ls, bs) == (pl.PL_STAGE_LAPLACIAN_SMALL, pl.PL_STAGE_BILATERAL_SMALL)
    saved = [pl.pl_tune_get(ls, 3), pl.pl_tune_get(bs, 3)]
    try:
        cache = str(tmp_path / "tune.json")
        rep = tune.autotune([(pts, 3, 3, 3, 2)], cache_path=cache, reps=3)
        assert tuple(rep["laplacian_small_k3"]["best"]) in tune.LAP_CANDIDATES[3]
        assert tuple(rep["bilateral_small_k3"]["best"]) in tune.BIL_CANDIDATES[3]
        assert pl.pl_tune_get(ls, 3) == tuple(rep["laplacian_small_k3"]["best"])
        assert np.array_equal(host(pl.pl_laplacian(pts, 3, 1.0, 3)).view(np.uint8), ref.view(np.uint8))
        pl.pl_tune_set(ls, 3, *saved[0])
        assert tune.load_cache(cache) == 2
        assert pl.pl_tune_get(ls, 3) == tuple(rep["laplacian_small_k3"]["best"])
    finally:
        pl.pl_tune_set(ls, 3, *saved[0])
        pl.pl_tune_set(bs, 3, *saved[1])


def test_autotune_batch_stages(pl, tmp_path):
    import torch
    from paper_2007_12065_amd import tune
    specs = [mixed_specs()[0], mixed_specs()[2]]          # 3x3 and 5x5 frames
    saved = {(s, k): pl.pl_tune_get(s, k) for s in (2, 3) for k in (3, 5)}
    try:
        cache = str(tmp_path / "tune.json")
        rep = tune.autotune_batch(specs, cache_path=cache, reps=2)
        assert set(rep) == {"batch_laplacian_k3", "batch_laplacian_k5", "batch_bilateral_k3",
                            "batch_bilateral_k5"}
        for name, r in rep.items():
            k = int(name[-1])
            cands = tune.LAP_CANDIDATES if "laplacian" in name else tune.BIL_CANDIDATES
            assert tuple(r["best"]) in cands[k]
        assert pl.pl_tune_get(pl.PL_STAGE_BATCH_BILATERAL, 5) == tuple(rep["batch_bilateral_k5"]["best"])
        b = pl.Batch(specs, torch.float32)
        b.run()
        torch.cuda.synchronize()
        for i, sp in enumerate(specs):
            assert_frame_equal(b.outputs[i], single(pl, sp, torch.float32), f"tuned frame {i}")
        b.close()
        for (s, k), v in saved.items():
            pl.pl_tune_set(s, k, *v)
        assert tune.load_cache(cache) == 4
        assert pl.pl_tune_get(pl.PL_STAGE_BATCH_BILATERAL, 5) == tuple(rep["batch_bilateral_k5"]["best"])
    finally:
        for (s, k), v in saved.items():
            pl.pl_tune_set(s, k, *v)
