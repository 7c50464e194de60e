"""The allocation-free mesh entry point (pl_mesh_opc_static) through the C
ABI: its outputs equal pl_mesh_opc's bit for bit on two calls in a row, the
second on a smaller frame (the static scratch keeps the first call's codes),
and on a frame meshed by whole quad rows."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _frame(M, N, seed, nan_frac=0.08):
    rng = np.random.default_rng(seed)
    u, v = np.meshgrid(np.arange(M, dtype=np.float64), np.arange(N, dtype=np.float64),
                       indexing="ij")
    p = np.stack([v * 0.01, u * 0.01, 2.0 + 0.01 * rng.standard_normal((M, N))], -1)
    p[rng.random((M, N)) < nan_frac] = np.nan
    return torch.from_numpy(p.astype(np.float32))


def _check_equal(pl, pts, cap=None):
    dev = torch.device("cuda:0")
    x = pts.to(dev)
    print(f"[no_alloc] frame {tuple(pts.shape[:2])} cap {cap}", flush=True)
    ref = pl.pl_mesh_opc(x, cap=cap)
    got = pl.pl_mesh_opc_static(x, cap=cap)
    torch.cuda.synchronize(dev)
    n = int(ref["n_tri"].item())
    assert int(got["n_tri"].item()) == n
    w = n if cap is None else min(n, cap)
    assert torch.equal(got["tri_valid"], ref["tri_valid"])
    assert torch.equal(got["tri_map"], ref["tri_map"])
    assert torch.equal(got["triangles"][:w], ref["triangles"][:w])
    assert torch.equal(got["halfedges"][:3 * w], ref["halfedges"][:3 * w])
    return n


def test_static_mesh_equals_workspace_mesh():
    import paper_2007_12065_amd as pl
    # the 480x640 frame, then a smaller one: the second call must not see
    # the first call's codes and counts in the shared scratch
    n1 = _check_equal(pl, _frame(480, 640, 1))
    n2 = _check_equal(pl, _frame(37, 301, 2, nan_frac=0.3))
    assert n1 > n2 > 0
    # all-NaN, a capacity below |T|, and a frame of more than 8,192 row
    # segments (meshed by whole rows)
    assert _check_equal(pl, _frame(5, 7, 3, nan_frac=1.0)) == 0
    _check_equal(pl, _frame(64, 1024, 4), cap=1000)
    _check_equal(pl, _frame(300, 7000, 5))
    # too large for the scratch: rejected, nothing enqueued
    big = torch.empty((3000, 3000, 3), dtype=torch.float32, device="cuda:0")
    with pytest.raises(pl.PLError, match="static scratch"):
        pl.pl_mesh_opc_static(big, cap=1)
