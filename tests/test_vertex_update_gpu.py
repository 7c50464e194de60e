"""GPU parity of the vertex update (the second stage of the bilateral
denoising the paper cites; restated, pinned in the oracle tests) through the
C ABI: identical float32 inputs, points within 1e-5 relative of the FP64
oracle (Euclidean, per vertex), invalid points copied bitwise, on grids
spanning several 256-point blocks with ragged tails, NaN holes, 0-5 sweeps,
float32 and float16 normals, and the full-size synthetic frames."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
VERTEX_RTOL = 1e-5


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


def check(pl, pts, normals, iters):
    import torch
    got = pl.pl_vertex_update(to_dev(pts), to_dev(normals), iters)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    want = oracle.vertex_update(pts.astype(np.float64), normals.astype(np.float64), iters, threads=8)
    bad = np.isnan(pts).any(-1)
    assert np.array_equal(np.isnan(got).any(-1), bad)
    assert np.array_equal(got[bad].view(np.uint32), pts[bad].view(np.uint32))
    ok = ~bad
    rel = np.linalg.norm(got[ok].astype(np.float64) - want[ok], axis=-1) / np.linalg.norm(want[ok], axis=-1)
    assert rel.max() <= VERTEX_RTOL, rel.max()
    return got


@pytest.mark.parametrize("M,N,seed", [(2, 2, 1), (3, 300, 2), (37, 520, 3), (64, 257, 4), (9, 1000, 5),
                                      (70000, 3, 6)])
def test_random_grids(pl, orc, M, N, seed):
    g = synth.random_grid(M, N, seed, nan_frac=0.1, noise=0.02)
    n, _ = orc.tri_normals(g)
    nf = orc.bilateral(n.astype(np.float32), _.astype(np.float32), 3, 0.1, 0.1, 1).astype(np.float32)
    for iters in (0, 1, 2, 5):
        say("vertex update", M, N, "iters", iters)
        check(pl, g, nf, iters)
    say("vertex update f16", M, N)
    check(pl, g, nf.astype(np.float16), 2)


@pytest.mark.parametrize("kind", ["rgbd", "lidar"])
def test_full_frames(pl, orc, kind):
    k = synth.KINDS[kind]
    p = synth.make_frame(kind, 41)
    r = orc.pipeline(p, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil, k.sigma_length,
                     k.sigma_angle, k.iters_bil, threads=8)
    pts = r["points"].astype(np.float32)
    nf = r["filtered"].astype(np.float32)
    say("vertex update full", kind)
    check(pl, pts, nf, 3)
