"""The README's usage example runs as written (one frame: the whole path,
also through the fused entry, group labels and a Gaussian accumulator
histogram), and its outputs are consistent: the fused entry's N_T equals
the single calls', labels for every triangle of T, counts summing to the
sampled normals."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_readme_example():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2007_12065_amd as pl
    from synth import make_frame, scene_planes

    pts = torch.from_numpy(make_frame("rgbd", 1000)).cuda()
    r = pl.smooth_frame(pts, kernel_lap=3, lam=1.0, iters_lap=4,
                        kernel_bil=3, sigma_length=0.1, sigma_angle=0.1, iters_bil=2)
    f = pl.pl_smooth_frame(dict(pts=pts, kernel_lap=3, lam=1.0, iters_lap=4, kernel_bil=3,
                                sigma_length=0.1, sigma_angle=0.1, iters_bil=2), torch.float32)
    labels = pl.pl_group_assign(r["points"], r["triangles"], r["normals_T"], r["n_tri"],
                                torch.from_numpy(scene_planes("rgbd", 1000)).cuda(), 0.05, 0.96)
    ga = pl.GaussianAccumulator(4)
    counts, _ = ga.integrate(r["normals_T"], n=r["n_tri"], stride=8)
    torch.cuda.synchronize()
    n = int(r["n_tri"].item())
    assert int(f["n_tri"].item()) == n
    assert torch.equal(f["normals_T"][:n].view(torch.uint8), r["normals_T"][:n].view(torch.uint8))
    lab = labels[:n].cpu().numpy()
    assert set(np.unique(lab)) <= {0, 1, 2, 255} and np.mean(lab != 255) > 0.5
    valid = ~np.isnan(r["normals_T"][:n].cpu().numpy()).any(1)
    assert int(counts.sum().item()) == int(valid[::8].sum())
    ga.close()
