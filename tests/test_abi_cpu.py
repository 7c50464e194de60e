"""The C ABI without a GPU: the library loads, exports every entry point its
header declares, and rejects bad arguments before launching anything."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pl.h")


@pytest.fixture(scope="module")
def pl():
    import paper_2007_12065_amd as pl
    return pl


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pl_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported(pl):
    names = header_functions()
    assert "pl_mesh_opc" in names and "pl_bilateral" in names
    lib = ctypes.CDLL(pl.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(pl.EXPORTS)


def test_version(pl):
    assert pl.pl_version() == 105


def test_workspace_sizes(pl):
    lib = pl._lib
    M, N = 480, 640
    assert lib.pl_mesh_opc_workspace(M, N) >= (M - 1) * (N - 1) + 4 * (M - 1)
    assert lib.pl_laplacian_workspace(M, N, 1) == 0
    assert lib.pl_laplacian_workspace(M, N, 4) == 12 * M * N
    assert lib.pl_bilateral_workspace(M, N, 0, 1) == 0
    assert lib.pl_bilateral_workspace(M, N, 0, 2) == 2 * (M - 1) * (N - 1) * 12
    assert lib.pl_bilateral_workspace(M, N, 1, 2) == 2 * (M - 1) * (N - 1) * 6
    assert lib.pl_mesh_opc_workspace(1, 5) == 0


A, B, C = 0x100000, 0x200000, 0x300000     # fake aligned addresses, never dereferenced


def err(pl):
    return pl._lib.pl_last_error().decode()


def test_mesh_static_argument_errors(pl):
    """The allocation-free mesh entry validates like pl_mesh_opc and rejects
    frames whose codes and counts exceed its static scratch, all before it
    looks up the scratch or launches anything."""
    lib = pl._lib
    f = lib.pl_mesh_opc_static
    assert f(A, 10, 1, None, B, C, None, 10, C + 4096, None) == -2
    assert f(A, 10, 10, None, B, C, None, -1, C + 4096, None) == -1
    assert f(A, 10, 10, None, None, C, None, 10, C + 4096, None) == -1
    assert "tri_map" in err(pl)
    assert f(A, 10, 10, None, B + 4, C, None, 10, C + 4096, None) == -1
    # 3000 x 3000: 9 M quads of codes, above the 8 MiB scratch
    assert lib.pl_mesh_opc_workspace(3000, 3000) > 8 << 20
    assert f(A, 3000, 3000, None, B, C, None, 10, C + 4096, None) == -2
    assert "static scratch" in err(pl)
    # 2000 x 4096 fits
    assert lib.pl_mesh_opc_workspace(2000, 4096) <= 8 << 20
    # an output overlapping the points
    assert f(A, 10, 10, None, A + 16, C, None, 10, C + 4096, None) == -4


def test_laplacian_argument_errors(pl):
    lib = pl._lib
    assert lib.pl_laplacian(A, B, 1, 5, 3, 1.0, 1, None, 0, None) == -2
    assert lib.pl_laplacian(A, B, 10, 10, 4, 1.0, 1, None, 0, None) == -3
    assert lib.pl_laplacian(A, B, 10, 10, 11, 1.0, 1, None, 0, None) == -3
    assert lib.pl_laplacian(A, B, 10, 10, 3, 1.5, 1, None, 0, None) == -1
    assert lib.pl_laplacian(A, B, 10, 10, 3, float("nan"), 1, None, 0, None) == -1
    assert lib.pl_laplacian(A, B, 10, 10, 3, 1.0, -1, None, 0, None) == -1
    assert lib.pl_laplacian(None, B, 10, 10, 3, 1.0, 1, None, 0, None) == -1
    assert "pts_in" in err(pl)
    assert lib.pl_laplacian(A + 4, B, 10, 10, 3, 1.0, 1, None, 0, None) == -1
    assert "aligned" in err(pl)
    assert lib.pl_laplacian(A, A + 16, 10, 10, 3, 1.0, 1, None, 0, None) == -4
    assert lib.pl_laplacian(A, B, 10, 10, 3, 1.0, 3, None, 0, None) == -5
    assert lib.pl_laplacian(A, B, 10, 10, 3, 1.0, 3, C, 100, None) == -5


def test_mesh_argument_errors(pl):
    lib = pl._lib
    ws = lib.pl_mesh_opc_workspace(10, 10)
    assert lib.pl_mesh_opc(A, 10, 1, None, B, C, None, 10, C + 4096, C + 8192, ws, None) == -2
    assert lib.pl_mesh_opc(A, 40000, 40000, None, B, C, None, 10, C + 4096, C + 8192, ws, None) == -2
    assert lib.pl_mesh_opc(A, 10, 10, None, B, C, None, -1, C + 4096, C + 8192, ws, None) == -1
    assert lib.pl_mesh_opc(A, 10, 10, None, None, C, None, 10, C + 4096, C + 8192, ws, None) == -1
    assert lib.pl_mesh_opc(A, 10, 10, None, B, C, None, 10, C + 4096, None, 0, None) == -5
    # tri_map overlapping the points
    assert lib.pl_mesh_opc(A, 10, 10, None, A + 256, C, None, 10, C + 4096, C + 8192, ws, None) == -4


def test_normals_and_bilateral_argument_errors(pl):
    lib = pl._lib
    assert lib.pl_tri_normals(A, 10, 10, B, 7, C, None) == -1
    assert lib.pl_tri_normals(A, 10, 10, A, 0, C, None) == -4
    def bil(nin=A, cen=B, ndt=0, M=10, N=10, K=3, sl=0.1, sa=0.1, it=1, nout=C,
            tm=None, nT=None, ws=None, wsb=0):
        return lib.pl_bilateral(nin, cen, ndt, M, N, K, sl, sa, it, nout, tm, nT, ws, wsb, None)
    assert bil(K=2) == -3
    assert bil(sl=0.0) == -1
    assert bil(sa=float("inf")) == -1
    assert bil(ndt=3) == -1
    assert bil(tm=C + 65536) == -1            # gather without a destination
    assert bil(nout=A) == -4
    assert bil(it=2) == -5


def test_group_assign_argument_errors(pl):
    lib = pl._lib
    D = 0x400000

    def ga(pts=A, n_pts=100, tris=B, nT=C, ndt=0, n_tri=D, cap=50, dom=D + 256, l=3,
           l_max=0.05, ang_min=0.96, groups=D + 4096):
        return lib.pl_group_assign(pts, n_pts, tris, nT, ndt, n_tri, cap, dom, l, l_max,
                                   ang_min, groups, None)
    assert ga(ndt=2) == -1
    assert ga(l=255) == -1 and "254" in err(pl)
    assert ga(l=-1) == -1
    assert ga(l_max=-0.5) == -1
    assert ga(l_max=float("nan")) == -1
    assert ga(ang_min=float("nan")) == -1
    assert ga(cap=-1) == -1
    assert ga(n_pts=-1) == -1
    assert ga(cap=1 << 30) == -2
    assert ga(n_tri=None) == -1 and "n_tri" in err(pl)
    assert ga(dom=None) == -1 and "dominant" in err(pl)
    assert ga(groups=B + 8) == -1 and "aligned" in err(pl)
    assert ga(groups=B + 16) == -4          # labels written over the triangle list
    assert ga(groups=A + 32) == -4          # ... or over the points
    assert ga(groups=D) == -4               # ... or over the triangle count


def test_batch_group_fields_checked(pl):
    """The optional group-assignment fields of pl_frame are validated with
    the rest of the frame (host-only: no device memory is touched)."""
    lib = pl._lib
    M, N = 8, 9
    T = 2 * (M - 1) * (N - 1)
    base = 0x10000000
    f = pl.PLFrame()
    f.M, f.N, f.kernel_lap, f.iters_lap, f.lambda_ = M, N, 3, 1, 1.0
    f.kernel_bil, f.iters_bil, f.sigma_length, f.sigma_angle = 3, 1, 0.1, 0.1
    for j, name in enumerate(["pts", "pts_out", "normals", "centroids", "tri_map", "triangles",
                              "n_tri", "normals_T"]):
        setattr(f, name, base + j * 0x100000)
    arr = (pl.PLFrame * 1)(f)
    plain = lib.pl_batch_workspace(arr, 1, 0)
    assert plain > 0
    arr[0].groups = base + 0x1000000
    arr[0].dominant, arr[0].n_dominant, arr[0].l_max, arr[0].ang_min = base + 0x1100000, 3, 0.05, 0.96
    assert lib.pl_batch_workspace(arr, 1, 0) > plain        # one more queue
    for field, bad in (("n_dominant", 255), ("l_max", -1.0), ("ang_min", float("nan")),
                       ("dominant", None), ("groups", base + 0x1000008)):
        g = pl.PLFrame.from_buffer_copy(arr[0])
        setattr(g, field, bad)
        assert lib.pl_batch_workspace((pl.PLFrame * 1)(g), 1, 0) == 0, field
        assert "group" in err(pl), field
    g = pl.PLFrame.from_buffer_copy(arr[0])
    g.groups = g.triangles + 16 * 12                      # labels over the triangle list
    assert lib.pl_batch_workspace((pl.PLFrame * 1)(g), 1, 0) == 0
    assert "overlap" in err(pl)
    # l = 0 needs no dominant array
    g = pl.PLFrame.from_buffer_copy(arr[0])
    g.n_dominant, g.dominant = 0, None
    assert lib.pl_batch_workspace((pl.PLFrame * 1)(g), 1, 0) > plain
    assert T > 0


def test_ga_host_side(pl):
    """Accumulator sizes and argument checks (host only)."""
    import numpy as np
    lib = pl._lib
    sizes = [lib.pl_ga_workspace(L) for L in range(6)]
    assert all(s > 0 for s in sizes) and sizes == sorted(sizes)
    # cells, bin table and candidate lists: the cells alone take 12 B each
    assert sizes[4] > 12 * 5120
    assert lib.pl_ga_workspace(-1) == 0 and lib.pl_ga_workspace(6) == 0
    cells = np.array([[0, 0, 1], [0, 1, 0], [1, 0, 0]], dtype=np.float32)
    cp = cells.ctypes.data_as(ctypes.c_void_p)
    assert lib.pl_ga_workspace_cells(cp, 3) > 0
    bad = cells * 1.01
    assert lib.pl_ga_workspace_cells(bad.ctypes.data_as(ctypes.c_void_p), 3) == 0
    assert lib.pl_ga_workspace_cells(None, 3) == 0
    h = ctypes.c_void_p()
    assert lib.pl_ga_create(9, A, 1 << 20, None, ctypes.byref(h)) == -1 and not h.value
    assert lib.pl_ga_create(2, A, 16, None, ctypes.byref(h)) == -5
    assert lib.pl_ga_integrate(None, A, 0, B, 10, 1, C, None, None) == -1
    assert lib.pl_ga_cell_count(None) == 0


def test_user_halfedges_host_side(pl):
    lib = pl._lib
    assert lib.pl_user_halfedges_workspace(0) == 0
    assert lib.pl_user_halfedges_workspace(-1) == 0
    assert lib.pl_user_halfedges_workspace(1000) >= 4 * 1000 * 16 + 12 * 1000
    assert lib.pl_user_halfedges_workspace(1 << 30) == 0
    ws = lib.pl_user_halfedges_workspace(100)
    D = 0x400000
    assert lib.pl_user_halfedges(A, B, -1, C, D, ws, None) == -1
    assert lib.pl_user_halfedges(A, None, 100, C, D, ws, None) == -1
    assert lib.pl_user_halfedges(A, B, 100, C, D, ws - 16, None) == -5
    assert lib.pl_user_halfedges(A, B, 100, A + 256, D, ws, None) == -4   # output over T
    assert lib.pl_user_halfedges(A, B, 100, C, C + 256, ws, None) == -4   # workspace over output


def test_vertex_update_argument_errors(pl):
    lib = pl._lib
    assert lib.pl_vertex_update_workspace(10, 10, 1) == 0
    assert lib.pl_vertex_update_workspace(10, 10, 2) >= 12 * 100
    assert lib.pl_vertex_update_workspace(1, 10, 2) == 0
    ws = lib.pl_vertex_update_workspace(10, 10, 3)
    assert lib.pl_vertex_update(A, B, 1, 10, C, 0, 1, None, 0, None) == -2
    assert lib.pl_vertex_update(A, B, 10, 10, C, 5, 1, None, 0, None) == -1
    assert lib.pl_vertex_update(A, B, 10, 10, C, 0, -1, None, 0, None) == -1
    assert lib.pl_vertex_update(None, B, 10, 10, C, 0, 1, None, 0, None) == -1
    assert lib.pl_vertex_update(A, A + 64, 10, 10, C, 0, 1, None, 0, None) == -4
    assert lib.pl_vertex_update(A, B, 10, 10, C, 0, 3, None, 0, None) == -5
    assert lib.pl_vertex_update(A, B, 10, 10, C, 0, 3, B + 16, ws, None) == -4


def test_tuning_table_stages(pl):
    # six independent tables: single large frames, single small frames and
    # batches, each for the Laplacian and the bilateral
    saved = {(s, k): pl.pl_tune_get(s, k) for s in range(6) for k in (3, 5)}
    try:
        for s in range(6):
            pl.pl_tune_set(s, 3, 4 + s, 32, 1)
        for s in range(6):
            assert pl.pl_tune_get(s, 3) == (4 + s, 32, 1)
        assert pl.pl_tune_get(pl.PL_STAGE_BATCH_BILATERAL, 5) == saved[(3, 5)]
        assert pl.pl_tune_get(pl.PL_STAGE_BILATERAL_SMALL, 5) == saved[(5, 5)]
        with pytest.raises(pl.PLError):
            pl.pl_tune_set(6, 3, 8, 32, 1)                   # no such stage
        with pytest.raises(pl.PLError):
            pl.pl_tune_set(-1, 3, 8, 32, 1)
        with pytest.raises(pl.PLError):
            pl.pl_tune_set(pl.PL_STAGE_BATCH_LAPLACIAN, 3, 8, 32, 0)   # fuse < 1
        with pytest.raises(pl.PLError):
            pl.pl_tune_set(pl.PL_STAGE_BATCH_BILATERAL, 9, 128, 128, 4)  # LDS too large
        with pytest.raises(pl.PLError):
            pl.pl_tune_get(0, 4)                              # even window
        assert pl.pl_tune_get(pl.PL_STAGE_BATCH_LAPLACIAN, 3) == (6, 32, 1)
    finally:
        for (s, k), v in saved.items():
            pl.pl_tune_set(s, k, *v)
