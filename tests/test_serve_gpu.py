"""The continuous-batching server on the GPU: every request's result equals
that frame's result through the single-frame calls (served alone), however
the requests were grouped into steps, with slots reused and steps
overlapping."""
import numpy as np
import pytest

from synth import KINDS, make_frame, poisson_arrivals

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pl():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2007_12065_amd as pl
    return pl


def classes_and_frames():
    from paper_2007_12065_amd.serve import FrameClass
    kinds = ("rgbd_small", "lidar", "rgbd")
    classes = {k: FrameClass(k, KINDS[k].M, KINDS[k].N, KINDS[k].kernel_lap, KINDS[k].lam,
                             KINDS[k].iters_lap, KINDS[k].kernel_bil, KINDS[k].sigma_length,
                             KINDS[k].sigma_angle, KINDS[k].iters_bil) for k in kinds}
    frames = {k: [make_frame(k, 700 + 10 * j + i) for i in range(3)] for j, k in enumerate(kinds)}
    return classes, frames


@pytest.mark.parametrize("device_inputs", [False, True])
def test_served_results_equal_single_frame_results(pl, device_inputs):
    import torch
    from paper_2007_12065_amd.serve import ADMITTED, Server
    classes, frames = classes_and_frames()
    # alone: each frame through the four single-frame calls, float16 normals
    alone = {}
    for k, fs in frames.items():
        c = classes[k]
        for i, f in enumerate(fs):
            x = torch.from_numpy(f).to("cuda:0")
            m = pl.pl_mesh_opc(x)
            p = pl.pl_laplacian(x, c.kernel_lap, c.lam, c.iters_lap)
            n, cen = pl.pl_tri_normals(p, torch.float16)
            nf, nT = pl.pl_bilateral(n, cen, c.kernel_bil, c.sigma_length, c.sigma_angle,
                                     c.iters_bil, tri_map=m["tri_map"])
            nt = int(m["n_tri"].item())
            alone[(k, i)] = (nt, m["triangles"][:nt].cpu().numpy(), p.cpu().numpy(),
                             nT[:nt].cpu().numpy(), nf.cpu().numpy())
    src = frames if not device_inputs else {k: [torch.from_numpy(f).to("cuda:0") for f in v]
                                            for k, v in frames.items()}
    # a budget for only a few slots of each class, arrivals fast enough for
    # multi-frame steps, waiting requests and slot reuse
    srv = Server(classes, src, 600 << 20, torch.float16, max_inflight=2)
    srv.presize({"rgbd_small": 2, "lidar": 2, "rgbd": 2})
    times, kinds = poisson_arrivals(4000.0, 0.03, seed=77,
                                    mix=(("rgbd", 0.4), ("lidar", 0.3), ("rgbd_small", 0.3)))
    seen = []

    def on_done(r, out):
        nt = int(out["n_tri"].item())
        got = (nt, out["triangles"][:nt].cpu().numpy(), out["points"].cpu().numpy(),
               out["normals_T"][:nt].cpu().numpy(), out["normals"].cpu().numpy())
        want = alone[(r.cls, r.frame)]
        assert got[0] == want[0], (r.rid, r.cls)
        for a, b, name in zip(got[1:], want[1:], ("triangles", "points", "normals_T", "normals")):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (r.rid, r.cls, name)
        seen.append(r.rid)

    print("[case] served stream of", len(times), "requests, device inputs", device_inputs, flush=True)
    res = srv.serve(times, kinds, warmup_s=0.0, on_done=on_done)
    assert len(seen) == len(times) and res["rejected"] == 0
    assert res["max_step"] >= 2                  # requests really shared steps
