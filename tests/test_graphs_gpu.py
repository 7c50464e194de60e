"""The group assignment, Gaussian accumulator, user-mesh half-edge and
vertex update entry points captured into a HIP graph: every replay (with
eager work and synchronisation between replays) gives the eager result.
The accumulator's replays add up (its scratch histograms return to zero
after each integration)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


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


def test_graph_replays(pl, orc):
    import torch
    k = synth.KINDS["rgbd_small"]
    p = synth.make_frame("rgbd_small", 5)
    r = orc.pipeline(p, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil, k.sigma_length,
                     k.sigma_angle, k.iters_bil, threads=4)
    pts = to_dev(r["points"].astype(np.float32))
    T = to_dev(r["triangles"])
    nT = to_dev(r["normals_T"].astype(np.float32))
    nf = to_dev(r["filtered"].astype(np.float32))
    n_tri = torch.tensor([len(r["triangles"])], dtype=torch.int32, device="cuda:0")
    dom = to_dev(synth.scene_planes("rgbd_small", 5))
    _, _, C = oracle.ga_icosahedron(3)
    ga = pl.GaussianAccumulator(cells=C)
    cap = len(r["triangles"])
    groups = torch.empty(cap, dtype=torch.uint8, device="cuda:0")
    counts = torch.zeros(ga.n_cells, dtype=torch.uint32, device="cuda:0")
    he = torch.empty(3 * cap, dtype=torch.int32, device="cuda:0")
    moved = torch.empty_like(pts)

    def work():
        pl.pl_group_assign(pts, T, nT, n_tri, dom, k.l_max, k.ang_min, out=groups)
        ga.integrate(nT, n=n_tri, counts=counts)
        pl.pl_user_halfedges(T, n_tri, out=he)
        pl.pl_vertex_update(pts, nf, 2, out=moved)

    say("graph eager reference")
    work()
    torch.cuda.synchronize()
    want = (groups.clone(), counts.clone(), he.clone(), moved.clone())
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    counts.zero_()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        work()
    for rep in range(3):
        say("graph replay", rep)
        groups.fill_(77)
        he.fill_(-77)
        moved.fill_(0.0)
        counts.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(groups, want[0]), rep
        assert torch.equal(counts, want[1]), rep
        assert torch.equal(he, want[2]), rep
        assert torch.equal(moved.view(torch.int32), want[3].view(torch.int32)), rep  # NaN-aware: bits
        _ = (pts * 2).sum().item()          # eager work between replays
    # replays without clearing: the accumulator's counts add up
    counts.zero_()
    torch.cuda.synchronize()
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    assert torch.equal(counts.to(torch.int64), 3 * want[1].to(torch.int64))
    ga.close()
