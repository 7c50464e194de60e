"""Whole-path oracle checks on the 120x160 synthetic RGBD frame."""
import numpy as np

from synth import config_frame
from test_oracle_mesh import hashmap_twins


def test_pipeline_rgbd_small(orc):
    pts, k = config_frame(0)
    r = orc.pipeline(pts, k.kernel_lap, k.lam, k.iters_lap, k.kernel_bil,
                     k.sigma_length, k.sigma_angle, k.iters_bil, threads=4)
    M, N = pts.shape[:2]
    # validity is unchanged by smoothing, so meshing before or after agrees
    assert np.array_equal(np.isnan(r["points"]), np.isnan(pts))
    tm2, tris2 = orc.mesh(r["points"])
    assert np.array_equal(tm2, r["tri_map"]) and np.array_equal(tris2, r["triangles"])
    assert np.array_equal(r["halfedges"], hashmap_twins(r["triangles"]))
    nt = r["normals_T"]
    assert nt.shape == (len(r["triangles"]), 3)
    assert np.allclose(np.linalg.norm(nt, axis=-1), 1.0, atol=1e-12)
    # smoothing pulls normals together: mean angle to the floor normal drops
    floor = np.array([0.0, -np.sin(np.radians(10)), -np.cos(np.radians(10))])
    raw = orc.gather(r["normals"], r["tri_map"], len(r["triangles"]))
    err_raw = np.degrees(np.arccos(np.clip(raw @ floor, -1, 1)))
    err_f = np.degrees(np.arccos(np.clip(nt @ floor, -1, 1)))
    assert np.median(err_f) < np.median(err_raw)


def test_thread_count_invariant(orc):
    pts, k = config_frame(0)
    a = orc.pipeline(pts, 3, 1.0, 2, 3, 0.1, 0.1, 2, threads=1)
    b = orc.pipeline(pts, 3, 1.0, 2, 3, 0.1, 0.1, 2, threads=4)
    for key in a:
        assert np.array_equal(a[key], b[key], equal_nan=True)
