"""Python binding of libpl.so, the gfx950 HIP library for organized-point-cloud
meshing and smoothing (Polylidar3D, arXiv 2007.12065, Sec. 4.2 and Sec. 5).

The functions carry the C ABI's names (include/pl.h) and only marshal
arguments: they check tensor placement, allocate outputs and workspaces with
PyTorch on the tensors' device, and pass raw device pointers and the current
HIP stream.  Every step runs in the library's kernels; there is no CPU path.
Importing this module fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# PL_LIBRARY names another build of the same library (the host-sanitizer
# build of sanitize.py); by default the in-tree libpl.so
LIB_PATH = os.environ.get("PL_LIBRARY") or os.path.join(_HERE, "libpl.so")

PL_F32, PL_F16 = 0, 1
_STATUS = {0: "PL_OK", -1: "PL_ERR_ARG", -2: "PL_ERR_SHAPE", -3: "PL_ERR_KERNEL",
           -4: "PL_ERR_ALIAS", -5: "PL_ERR_WORKSPACE", -6: "PL_ERR_HIP"}

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: the HIP library must be built first "
        "(python -c 'import __graft_entry__ as g; g.build()')")

_lib = ctypes.CDLL(LIB_PATH)
_vp, _i32, _f32, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_size_t
_lib.pl_version.restype = _i32
_lib.pl_last_error.restype = ctypes.c_char_p
_lib.pl_mesh_opc_workspace.argtypes = [_i32, _i32]
_lib.pl_mesh_opc_workspace.restype = _sz
_lib.pl_mesh_opc.argtypes = [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _sz, _vp]
_lib.pl_mesh_opc.restype = _i32
_lib.pl_mesh_opc_static.argtypes = [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp]
_lib.pl_mesh_opc_static.restype = _i32
_lib.pl_laplacian_workspace.argtypes = [_i32, _i32, _i32]
_lib.pl_laplacian_workspace.restype = _sz
_lib.pl_laplacian_fused_sweeps.argtypes = [_i32]
_lib.pl_laplacian_fused_sweeps.restype = _i32
_lib.pl_laplacian.argtypes = [_vp, _vp, _i32, _i32, _i32, _f32, _i32, _vp, _sz, _vp]
_lib.pl_laplacian.restype = _i32
_lib.pl_tri_normals.argtypes = [_vp, _i32, _i32, _vp, _i32, _vp, _vp]
_lib.pl_tri_normals.restype = _i32
_lib.pl_bilateral_workspace.argtypes = [_i32, _i32, _i32, _i32]
_lib.pl_bilateral_workspace.restype = _sz
_lib.pl_bilateral.argtypes = [_vp, _vp, _i32, _i32, _i32, _i32, _f32, _f32, _i32,
                              _vp, _vp, _vp, _vp, _sz, _vp]
_lib.pl_bilateral.restype = _i32

class PLFrame(ctypes.Structure):
    """Mirror of the C struct pl_frame (include/pl.h)."""
    _fields_ = [("pts", _vp), ("M", _i32), ("N", _i32), ("kernel_lap", _i32),
                ("iters_lap", _i32), ("lambda_", _f32), ("kernel_bil", _i32),
                ("iters_bil", _i32), ("sigma_length", _f32), ("sigma_angle", _f32),
                ("pts_out", _vp), ("normals", _vp), ("centroids", _vp), ("tri_valid", _vp),
                ("tri_map", _vp), ("triangles", _vp), ("halfedges", _vp), ("n_tri", _vp),
                ("normals_T", _vp), ("dominant", _vp), ("n_dominant", _i32), ("l_max", _f32),
                ("ang_min", _f32), ("groups", _vp)]


_lib.pl_tune_get.argtypes = [_i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                             ctypes.POINTER(_i32)]
_lib.pl_tune_get.restype = _i32
_lib.pl_tune_set.argtypes = [_i32, _i32, _i32, _i32, _i32]
_lib.pl_tune_set.restype = _i32
_lib.pl_batch_workspace.argtypes = [ctypes.POINTER(PLFrame), _i32, _i32]
_lib.pl_batch_workspace.restype = _sz
_lib.pl_batch_create.argtypes = [ctypes.POINTER(PLFrame), _i32, _i32, _vp, _sz, _vp,
                                 ctypes.POINTER(_vp)]
_lib.pl_batch_create.restype = _i32
_lib.pl_batch_run.argtypes = [_vp, _vp, _vp]
_lib.pl_batch_run.restype = _i32
_lib.pl_batch_capture.argtypes = [_vp, _vp, _vp]
_lib.pl_batch_capture.restype = _i32
_lib.pl_batch_replay.argtypes = [_vp, _vp]
_lib.pl_batch_replay.restype = _i32
_lib.pl_batch_capture_bounded.argtypes = [_vp, _vp, _i32, _vp]
_lib.pl_batch_capture_bounded.restype = _i32
_lib.pl_batch_replay_bounded.argtypes = [_vp, _i32, _vp]
_lib.pl_batch_replay_bounded.restype = _i32
_lib.pl_smooth_frame_workspace.argtypes = [ctypes.POINTER(PLFrame), _i32]
_lib.pl_smooth_frame_workspace.restype = _sz
_lib.pl_smooth_frame.argtypes = [ctypes.POINTER(PLFrame), _i32, _vp, _sz, _vp]
_lib.pl_smooth_frame.restype = _i32
_lib.pl_smooth_frame_events.argtypes = [ctypes.POINTER(PLFrame), _i32, _vp, _sz, _vp, _i32, _vp,
                                        _i32, ctypes.POINTER(_i32), _vp]
_lib.pl_smooth_frame_events.restype = _i32
_lib.pl_smooth_batch.argtypes = [_vp, _i32, _i32, _vp, _sz, _vp]
_lib.pl_smooth_batch.restype = _i32
_lib.pl_batch_destroy.argtypes = [_vp]
_lib.pl_batch_destroy.restype = None
_lib.pl_group_assign.argtypes = [_vp, _i32, _vp, _vp, _i32, _vp, _i32, _vp, _i32, _f32, _f32,
                                 _vp, _vp]
_lib.pl_group_assign.restype = _i32
_lib.pl_ga_workspace.argtypes = [_i32]
_lib.pl_ga_workspace.restype = _sz
_lib.pl_ga_workspace_cells.argtypes = [_vp, _i32]
_lib.pl_ga_workspace_cells.restype = _sz
_lib.pl_ga_create.argtypes = [_i32, _vp, _sz, _vp, ctypes.POINTER(_vp)]
_lib.pl_ga_create.restype = _i32
_lib.pl_ga_create_cells.argtypes = [_vp, _i32, _vp, _sz, _vp, ctypes.POINTER(_vp)]
_lib.pl_ga_create_cells.restype = _i32
_lib.pl_ga_cell_count.argtypes = [_vp]
_lib.pl_ga_cell_count.restype = _i32
_lib.pl_ga_cells.argtypes = [_vp]
_lib.pl_ga_cells.restype = _vp
_lib.pl_ga_integrate.argtypes = [_vp, _vp, _i32, _vp, _i32, _i32, _vp, _vp, _vp]
_lib.pl_ga_integrate.restype = _i32
_lib.pl_ga_destroy.argtypes = [_vp]
_lib.pl_ga_destroy.restype = None
_lib.pl_user_halfedges_workspace.argtypes = [_i32]
_lib.pl_user_halfedges_workspace.restype = _sz
_lib.pl_user_halfedges.argtypes = [_vp, _vp, _i32, _vp, _vp, _sz, _vp]
_lib.pl_user_halfedges.restype = _i32
_lib.pl_vertex_update_workspace.argtypes = [_i32, _i32, _i32]
_lib.pl_vertex_update_workspace.restype = _sz
_lib.pl_vertex_update.argtypes = [_vp, _vp, _i32, _i32, _vp, _i32, _i32, _vp, _sz, _vp]
_lib.pl_vertex_update.restype = _i32

PL_STAGE_LAPLACIAN, PL_STAGE_BILATERAL, PL_STAGE_BATCH_LAPLACIAN, PL_STAGE_BATCH_BILATERAL = 0, 1, 2, 3
PL_STAGE_LAPLACIAN_SMALL, PL_STAGE_BILATERAL_SMALL = 4, 5
SMALL_FRAME_POINTS = 1 << 17      # frames of at most this many points read the *_SMALL entries

EXPORTS = ["pl_version", "pl_last_error", "pl_mesh_opc_workspace", "pl_mesh_opc",
           "pl_mesh_opc_static",
           "pl_laplacian_workspace", "pl_laplacian_fused_sweeps", "pl_laplacian", "pl_tri_normals",
           "pl_bilateral_workspace", "pl_bilateral", "pl_tune_get", "pl_tune_set",
           "pl_batch_workspace", "pl_batch_create", "pl_batch_run", "pl_batch_capture",
           "pl_batch_replay", "pl_batch_capture_bounded", "pl_batch_replay_bounded",
           "pl_batch_destroy", "pl_smooth_batch", "pl_smooth_frame_workspace", "pl_smooth_frame", "pl_smooth_frame_events",
           "pl_group_assign", "pl_ga_workspace",
           "pl_ga_workspace_cells", "pl_ga_create", "pl_ga_create_cells", "pl_ga_cell_count",
           "pl_ga_cells", "pl_ga_integrate", "pl_ga_destroy", "pl_user_halfedges_workspace",
           "pl_user_halfedges", "pl_vertex_update_workspace", "pl_vertex_update"]


class PLError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.pl_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(status: int, where: str) -> None:
    if status != 0:
        raise PLError(status, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_tensor(t: torch.Tensor, dtype, name: str) -> None:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _ws(nbytes: int, device) -> torch.Tensor | None:
    return torch.empty(nbytes, dtype=torch.uint8, device=device) if nbytes else None


def _ndt(dtype) -> int:
    if dtype in (torch.float32, "f32", PL_F32):
        return PL_F32
    if dtype in (torch.float16, "f16", PL_F16):
        return PL_F16
    raise ValueError(f"normal storage must be float32 or float16, got {dtype}")


def _tdtype(ndt: int):
    return torch.float32 if ndt == PL_F32 else torch.float16


def pl_version() -> int:
    return int(_lib.pl_version())


def lap_fused_sweeps(kernel: int) -> int:
    """Laplacian sweeps fused per kernel launch for this window size."""
    return int(_lib.pl_laplacian_fused_sweeps(kernel))


def pl_mesh_opc(pts: torch.Tensor, *, tri_valid: bool = True, halfedges: bool = True,
                cap: int | None = None) -> dict:
    """Alg. 1 and Alg. 2 on a [M, N, 3] float32 device tensor.  Returns a dict
    of device tensors: tri_valid (uint8 [2Q] or None), tri_map (int32 [2Q]),
    triangles (int32 [cap, 3]), halfedges (int32 [3 cap] or None) and n_tri
    (int32 [1]); only the first n_tri rows of triangles/halfedges are set."""
    _dev_tensor(pts, torch.float32, "pts")
    if pts.dim() != 3 or pts.shape[2] != 3:
        raise ValueError("pts must be [M, N, 3]")
    M, N = int(pts.shape[0]), int(pts.shape[1])
    dev = pts.device
    T = 2 * max(M - 1, 0) * max(N - 1, 0)
    cap = T if cap is None else int(cap)
    out = dict(
        tri_valid=torch.empty(T, dtype=torch.uint8, device=dev) if tri_valid else None,
        tri_map=torch.empty(T, dtype=torch.int32, device=dev),
        triangles=torch.empty((max(cap, 1), 3), dtype=torch.int32, device=dev),
        halfedges=torch.empty(3 * max(cap, 1), dtype=torch.int32, device=dev) if halfedges else None,
        n_tri=torch.empty(1, dtype=torch.int32, device=dev),
    )
    ws_n = _lib.pl_mesh_opc_workspace(M, N)
    ws = _ws(ws_n, dev)
    _check(_lib.pl_mesh_opc(_ptr(pts), M, N, _ptr(out["tri_valid"]), _ptr(out["tri_map"]),
                            _ptr(out["triangles"]), _ptr(out["halfedges"]), cap,
                            _ptr(out["n_tri"]), _ptr(ws), ws_n, _stream(dev)), "pl_mesh_opc")
    return out


def pl_mesh_opc_static(pts: torch.Tensor, *, tri_valid: bool = True, halfedges: bool = True,
                       cap: int | None = None, out: dict | None = None) -> dict:
    """pl_mesh_opc without a workspace (the library's static scratch).  With
    `out` (a dict of preallocated tensors with pl_mesh_opc's keys) nothing is
    allocated, so the call can sit in a graph capture or a serving loop."""
    _dev_tensor(pts, torch.float32, "pts")
    if pts.dim() != 3 or pts.shape[2] != 3:
        raise ValueError("pts must be [M, N, 3]")
    M, N = int(pts.shape[0]), int(pts.shape[1])
    dev = pts.device
    T = 2 * max(M - 1, 0) * max(N - 1, 0)
    cap = T if cap is None else int(cap)
    if out is None:
        out = dict(
            tri_valid=torch.empty(T, dtype=torch.uint8, device=dev) if tri_valid else None,
            tri_map=torch.empty(T, dtype=torch.int32, device=dev),
            triangles=torch.empty((max(cap, 1), 3), dtype=torch.int32, device=dev),
            halfedges=torch.empty(3 * max(cap, 1), dtype=torch.int32, device=dev) if halfedges else None,
            n_tri=torch.empty(1, dtype=torch.int32, device=dev),
        )
    _check(_lib.pl_mesh_opc_static(_ptr(pts), M, N, _ptr(out.get("tri_valid")),
                                   _ptr(out["tri_map"]), _ptr(out["triangles"]),
                                   _ptr(out.get("halfedges")), cap, _ptr(out["n_tri"]),
                                   _stream(dev)), "pl_mesh_opc_static")
    return out


def pl_laplacian(pts: torch.Tensor, kernel: int, lam: float, iterations: int,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """Eqs. (1)-(2), Sec. 5.1: `iterations` Jacobi sweeps; returns [M, N, 3]."""
    _dev_tensor(pts, torch.float32, "pts")
    M, N = int(pts.shape[0]), int(pts.shape[1])
    out = torch.empty_like(pts) if out is None else out
    _dev_tensor(out, torch.float32, "out")
    ws_n = _lib.pl_laplacian_workspace(M, N, iterations)
    ws = _ws(ws_n, pts.device)
    _check(_lib.pl_laplacian(_ptr(pts), _ptr(out), M, N, kernel, lam, iterations,
                             _ptr(ws), ws_n, _stream(pts.device)), "pl_laplacian")
    return out


def pl_tri_normals(pts: torch.Tensor, dtype=torch.float32):
    """Sec. 5.2: (normals, centroids) in T_FC layout [M-1, N-1, 2, 3]; normals
    stored as `dtype` (float32 or float16), centroids float32."""
    _dev_tensor(pts, torch.float32, "pts")
    M, N = int(pts.shape[0]), int(pts.shape[1])
    ndt = _ndt(dtype)
    shape = (max(M - 1, 1), max(N - 1, 1), 2, 3)
    normals = torch.empty(shape, dtype=_tdtype(ndt), device=pts.device)
    centroids = torch.empty(shape, dtype=torch.float32, device=pts.device)
    _check(_lib.pl_tri_normals(_ptr(pts), M, N, _ptr(normals), ndt, _ptr(centroids),
                               _stream(pts.device)), "pl_tri_normals")
    return normals, centroids


def pl_bilateral(normals: torch.Tensor, centroids: torch.Tensor, kernel: int,
                 sigma_length: float, sigma_angle: float, iterations: int,
                 tri_map: torch.Tensor | None = None, out: torch.Tensor | None = None,
                 normals_T: torch.Tensor | None = None):
    """Eqs. (3)-(6), Sec. 5.2.  Returns (filtered normals in T_FC layout,
    normals gathered onto T [2Q, 3] or None); the storage type follows
    `normals` (float32 or float16)."""
    ndt = _ndt(normals.dtype)
    _dev_tensor(normals, _tdtype(ndt), "normals")
    _dev_tensor(centroids, torch.float32, "centroids")
    if normals.dim() != 4 or tuple(normals.shape[2:]) != (2, 3):
        raise ValueError("normals must be [M-1, N-1, 2, 3]")
    M, N = int(normals.shape[0]) + 1, int(normals.shape[1]) + 1
    dev = normals.device
    out = torch.empty_like(normals) if out is None else out
    if tri_map is not None:
        _dev_tensor(tri_map, torch.int32, "tri_map")
        if normals_T is None:
            normals_T = torch.empty((2 * (M - 1) * (N - 1), 3), dtype=normals.dtype, device=dev)
    ws_n = _lib.pl_bilateral_workspace(M, N, ndt, iterations)
    ws = _ws(ws_n, dev)
    _check(_lib.pl_bilateral(_ptr(normals), _ptr(centroids), ndt, M, N, kernel,
                             sigma_length, sigma_angle, iterations, _ptr(out), _ptr(tri_map),
                             _ptr(normals_T) if tri_map is not None else None,
                             _ptr(ws), ws_n, _stream(dev)), "pl_bilateral")
    return out, (normals_T if tri_map is not None else None)


def smooth_frame(pts: torch.Tensor, kernel_lap: int, lam: float, iters_lap: int,
                 kernel_bil: int, sigma_length: float, sigma_angle: float, iters_bil: int,
                 normal_dtype=torch.float32) -> dict:
    """The whole path on one frame in the paper's order: mesh (Alg. 1-2),
    Laplacian, centroids and normals, bilateral, gather onto T.  All outputs
    stay on the device; nothing synchronises."""
    mesh = pl_mesh_opc(pts)
    smooth = pl_laplacian(pts, kernel_lap, lam, iters_lap)
    normals, centroids = pl_tri_normals(smooth, normal_dtype)
    filtered, normals_T = pl_bilateral(normals, centroids, kernel_bil, sigma_length,
                                       sigma_angle, iters_bil, tri_map=mesh["tri_map"])
    return dict(mesh, points=smooth, normals=normals, centroids=centroids,
                filtered=filtered, normals_T=normals_T)


def pl_group_assign(points: torch.Tensor, triangles: torch.Tensor, normals_T: torch.Tensor,
                    n_tri: torch.Tensor, dominant: torch.Tensor | None, l_max: float,
                    ang_min: float, out: torch.Tensor | None = None) -> torch.Tensor:
    """Alg. 4, Sec. 7.1: uint8 group label [cap] of each triangle of T.

    points     float32 [M, N, 3] or [n, 3] device tensor (the smoothed vertices)
    triangles  int32 [cap, 3] (T), normals_T [cap, 3] float32 or float16
    n_tri      int32 [1] device tensor (|T|; rows at or past it are left as
               they were, uninitialised when `out` is allocated here)
    dominant   float32 [l, 3] device tensor of dominant normals, l <= 254
               (None or empty: every label is 255)."""
    _dev_tensor(points, torch.float32, "points")
    _dev_tensor(triangles, torch.int32, "triangles")
    ndt = _ndt(normals_T.dtype)
    _dev_tensor(normals_T, _tdtype(ndt), "normals_T")
    _dev_tensor(n_tri, torch.int32, "n_tri")
    if points.shape[-1] != 3 or triangles.dim() != 2 or triangles.shape[1] != 3:
        raise ValueError("points must be [..., 3] and triangles [cap, 3]")
    cap = int(triangles.shape[0])
    if tuple(normals_T.shape) != (cap, 3):
        raise ValueError("normals_T must be [cap, 3] like triangles")
    l = 0
    if dominant is not None and dominant.numel():
        _dev_tensor(dominant, torch.float32, "dominant")
        if dominant.dim() != 2 or dominant.shape[1] != 3:
            raise ValueError("dominant must be [l, 3]")
        l = int(dominant.shape[0])
    else:
        dominant = None
    dev = points.device
    out = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev) if out is None else out
    _dev_tensor(out, torch.uint8, "out")
    _check(_lib.pl_group_assign(_ptr(points), points.numel() // 3, _ptr(triangles),
                                _ptr(normals_T), ndt, _ptr(n_tri), cap, _ptr(dominant), l,
                                l_max, ang_min, _ptr(out), _stream(dev)), "pl_group_assign")
    return out[:cap]


def pl_vertex_update(pts: torch.Tensor, normals: torch.Tensor, iterations: int,
                     out: torch.Tensor | None = None) -> torch.Tensor:
    """Vertex update from filtered normals (the cited second stage of
    bilateral denoising): [M, N, 3] float32 points moved toward the planes of
    their triangles; normals in T_FC layout [M-1, N-1, 2, 3] (float32 or
    float16)."""
    _dev_tensor(pts, torch.float32, "pts")
    ndt = _ndt(normals.dtype)
    _dev_tensor(normals, _tdtype(ndt), "normals")
    M, N = int(pts.shape[0]), int(pts.shape[1])
    if tuple(normals.shape) != (M - 1, N - 1, 2, 3):
        raise ValueError("normals must be [M-1, N-1, 2, 3]")
    out = torch.empty_like(pts) if out is None else out
    _dev_tensor(out, torch.float32, "out")
    ws_n = _lib.pl_vertex_update_workspace(M, N, iterations)
    ws = _ws(ws_n, pts.device)
    _check(_lib.pl_vertex_update(_ptr(pts), _ptr(out), M, N, _ptr(normals), ndt, int(iterations),
                                 _ptr(ws), ws_n, _stream(pts.device)), "pl_vertex_update")
    return out


def pl_user_halfedges(triangles: torch.Tensor, n_tri: torch.Tensor | None = None,
                      out: torch.Tensor | None = None) -> torch.Tensor:
    """Sec. 4.3: twin of every half-edge of a user mesh, int32 [3 cap]
    (option 1 for edges shared by more than two triangles).  `triangles` is
    int32 [cap, 3] on the device; n_tri an int32 [1] device tensor (None =
    cap).  Entries past 3 n_tri are left as they were (uninitialised when
    `out` is allocated here)."""
    _dev_tensor(triangles, torch.int32, "triangles")
    if triangles.dim() != 2 or triangles.shape[1] != 3:
        raise ValueError("triangles must be [cap, 3]")
    cap = int(triangles.shape[0])
    dev = triangles.device
    if n_tri is None:
        n_tri = torch.full((1,), cap, dtype=torch.int32, device=dev)
    _dev_tensor(n_tri, torch.int32, "n_tri")
    out = torch.empty(max(3 * cap, 1), dtype=torch.int32, device=dev) if out is None else out
    _dev_tensor(out, torch.int32, "out")
    ws_n = _lib.pl_user_halfedges_workspace(cap)
    ws = _ws(ws_n, dev)
    _check(_lib.pl_user_halfedges(_ptr(triangles), _ptr(n_tri), cap, _ptr(out), _ptr(ws), ws_n,
                                  _stream(dev)), "pl_user_halfedges")
    return out[:3 * cap]


class GaussianAccumulator:
    """Sec. 6.1: a refined icosahedron's cells (pl_ga_* in include/pl.h).

    GaussianAccumulator(level) builds the library's level-`level` cells;
    GaussianAccumulator(cells=host float32 [n, 3]) uses the given unit cell
    normals.  The workspace is allocated here and kept with the handle."""

    def __init__(self, level: int | None = None, cells=None, device=None):
        import numpy as np
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        h = _vp()
        if cells is None:
            n = _lib.pl_ga_workspace(int(level))
            if n == 0:
                raise PLError(-1, "pl_ga_workspace")
            self.ws = torch.empty(n, dtype=torch.uint8, device=self.device)
            _check(_lib.pl_ga_create(int(level), _ptr(self.ws), n, _stream(self.device),
                                     ctypes.byref(h)), "pl_ga_create")
        else:
            c = np.ascontiguousarray(np.asarray(cells, dtype=np.float32).reshape(-1, 3))
            cp = c.ctypes.data_as(ctypes.c_void_p)
            n = _lib.pl_ga_workspace_cells(cp, len(c))
            if n == 0:
                raise PLError(-1, "pl_ga_workspace_cells")
            self.ws = torch.empty(n, dtype=torch.uint8, device=self.device)
            _check(_lib.pl_ga_create_cells(cp, len(c), _ptr(self.ws), n, _stream(self.device),
                                           ctypes.byref(h)), "pl_ga_create_cells")
        self._h = h
        self.n_cells = int(_lib.pl_ga_cell_count(h))

    def cells(self) -> torch.Tensor:
        """The cell normals, float32 [n_cells, 3] (a copy)."""
        out = torch.empty((self.n_cells, 3), dtype=torch.float32, device=self.device)
        base = _lib.pl_ga_cells(self._h)
        off = base - self.ws.data_ptr()
        out.copy_(self.ws[off:off + 12 * self.n_cells].view(torch.float32).view(self.n_cells, 3))
        return out

    def integrate(self, normals: torch.Tensor, n: torch.Tensor | None = None, stride: int = 1,
                  counts: torch.Tensor | None = None, cell_out: bool | torch.Tensor = False):
        """Alg. 3 over rows 0, stride, ... below n (int32 [1] device tensor;
        None = all rows) of normals [cap, 3] (float32 or float16).  Returns
        (counts uint32 [n_cells], added to when given; cell per integrated row
        int32 or None)."""
        ndt = _ndt(normals.dtype)
        _dev_tensor(normals, _tdtype(ndt), "normals")
        if normals.dim() != 2 or normals.shape[1] != 3:
            raise ValueError("normals must be [cap, 3]")
        cap = int(normals.shape[0])
        if n is None:
            n = torch.full((1,), cap, dtype=torch.int32, device=normals.device)
        _dev_tensor(n, torch.int32, "n")
        if counts is None:
            counts = torch.zeros(self.n_cells, dtype=torch.uint32, device=normals.device)
        _dev_tensor(counts, torch.uint32, "counts")
        rows = 0 if cap == 0 else (cap - 1) // stride + 1
        if cell_out is True:
            cell_out = torch.empty(max(rows, 1), dtype=torch.int32, device=normals.device)
        elif cell_out is False:
            cell_out = None
        _check(_lib.pl_ga_integrate(self._h, _ptr(normals), ndt, _ptr(n), cap, int(stride),
                                    _ptr(counts), _ptr(cell_out), _stream(normals.device)),
               "pl_ga_integrate")
        return counts, (cell_out[:rows] if cell_out is not None else None)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.pl_ga_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FramePlan:
    """Device buffers for one frame shape, allocated once, and the four ABI
    calls of the whole path on them.  run() only enqueues work on the current
    stream (mesh, Laplacian, normals, bilateral with the gather onto T) and
    allocates nothing."""

    def __init__(self, M: int, N: int, kernel_lap: int, lam: float, iters_lap: int,
                 kernel_bil: int, sigma_length: float, sigma_angle: float, iters_bil: int,
                 normal_dtype=torch.float32, device=None):
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.M, self.N, self.device = M, N, dev
        self.kernel_lap, self.lam, self.iters_lap = kernel_lap, lam, iters_lap
        self.kernel_bil, self.sigma_length, self.sigma_angle = kernel_bil, sigma_length, sigma_angle
        self.iters_bil = iters_bil
        self.ndt = _ndt(normal_dtype)
        T = 2 * (M - 1) * (N - 1)
        nd = _tdtype(self.ndt)
        e = lambda shape, dt: torch.empty(shape, dtype=dt, device=dev)
        self.points = e((M, N, 3), torch.float32)
        self.tri_valid = e(T, torch.uint8)
        self.tri_map = e(T, torch.int32)
        self.triangles = e((T, 3), torch.int32)
        self.halfedges = e(3 * T, torch.int32)
        self.n_tri = e(1, torch.int32)
        self.normals = e((M - 1, N - 1, 2, 3), nd)
        self.centroids = e((M - 1, N - 1, 2, 3), torch.float32)
        self.filtered = e((M - 1, N - 1, 2, 3), nd)
        self.normals_T = e((T, 3), nd)
        self.groups = e(T, torch.uint8)
        self._ws_mesh_n = _lib.pl_mesh_opc_workspace(M, N)
        self._ws_lap_n = _lib.pl_laplacian_workspace(M, N, iters_lap)
        self._ws_bil_n = _lib.pl_bilateral_workspace(M, N, self.ndt, iters_bil)
        self.ws_mesh = _ws(self._ws_mesh_n, dev)
        self.ws_lap = _ws(self._ws_lap_n, dev)
        self.ws_bil = _ws(self._ws_bil_n, dev)
        self.T = T

    def run_mesh(self, pts, s):
        _check(_lib.pl_mesh_opc(_ptr(pts), self.M, self.N, _ptr(self.tri_valid), _ptr(self.tri_map),
                                _ptr(self.triangles), _ptr(self.halfedges), self.T, _ptr(self.n_tri),
                                _ptr(self.ws_mesh), self._ws_mesh_n, s), "pl_mesh_opc")

    def run_laplacian(self, pts, s):
        _check(_lib.pl_laplacian(_ptr(pts), _ptr(self.points), self.M, self.N, self.kernel_lap,
                                 self.lam, self.iters_lap, _ptr(self.ws_lap), self._ws_lap_n, s),
               "pl_laplacian")

    def run_normals(self, s):
        _check(_lib.pl_tri_normals(_ptr(self.points), self.M, self.N, _ptr(self.normals), self.ndt,
                                   _ptr(self.centroids), s), "pl_tri_normals")

    def run_bilateral(self, s):
        _check(_lib.pl_bilateral(_ptr(self.normals), _ptr(self.centroids), self.ndt, self.M, self.N,
                                 self.kernel_bil, self.sigma_length, self.sigma_angle, self.iters_bil,
                                 _ptr(self.filtered), _ptr(self.tri_map), _ptr(self.normals_T),
                                 _ptr(self.ws_bil), self._ws_bil_n, s), "pl_bilateral")

    def run_groups(self, dominant: torch.Tensor, l_max: float, ang_min: float, s=None):
        """Alg. 4 on this frame's T, smoothed points and filtered normals_T
        (after run()); labels land in self.groups[:n_tri]."""
        s = _stream(self.device) if s is None else s
        _dev_tensor(dominant, torch.float32, "dominant")
        _check(_lib.pl_group_assign(_ptr(self.points), self.M * self.N, _ptr(self.triangles),
                                    _ptr(self.normals_T), self.ndt, _ptr(self.n_tri), self.T,
                                    _ptr(dominant), int(dominant.shape[0]), l_max, ang_min,
                                    _ptr(self.groups), s), "pl_group_assign")

    def run(self, pts: torch.Tensor) -> None:
        s = _stream(self.device)
        self.run_mesh(pts, s)
        self.run_laplacian(pts, s)
        self.run_normals(s)
        self.run_bilateral(s)

    def _fused_frame(self, pts):
        if getattr(self, "_frame", None) is None:
            f = PLFrame()
            f.M, f.N = self.M, self.N
            f.kernel_lap, f.iters_lap, f.lambda_ = self.kernel_lap, self.iters_lap, self.lam
            f.kernel_bil, f.iters_bil = self.kernel_bil, self.iters_bil
            f.sigma_length, f.sigma_angle = self.sigma_length, self.sigma_angle
            for buf, field in ((self.points, "pts_out"), (self.filtered, "normals"),
                               (self.centroids, "centroids"), (self.tri_valid, "tri_valid"),
                               (self.tri_map, "tri_map"), (self.triangles, "triangles"),
                               (self.halfedges, "halfedges"), (self.n_tri, "n_tri"),
                               (self.normals_T, "normals_T")):
                setattr(f, field, buf.data_ptr())
            f.pts = pts.data_ptr()
            self._ws_frame_n = _lib.pl_smooth_frame_workspace(ctypes.byref(f), self.ndt)
            if self._ws_frame_n == 0:
                raise PLError(-1, "pl_smooth_frame_workspace")
            self.ws_frame = _ws(self._ws_frame_n, self.device)
            self._frame = f
        return self._frame

    def run_fused_events(self, pts: torch.Tensor, events: list, s=None) -> list:
        """run_fused with the torch.cuda.Event list `events` (enable_timing)
        recorded before the first launch and after each launch; returns the
        launches' kinds (PL_LAUNCH_* bits, fused sweeps in bits 8..15)."""
        f = self._fused_frame(pts)
        f.pts = pts.data_ptr()
        s = _stream(self.device) if s is None else s
        for e in events:          # torch creates an event at its first record
            if not e.cuda_event:
                e.record()
        ev = (_vp * len(events))(*[e.cuda_event for e in events])
        kinds = (_i32 * 16)()
        n = _i32()
        _check(_lib.pl_smooth_frame_events(ctypes.byref(f), self.ndt, _ptr(self.ws_frame),
                                           self._ws_frame_n, ev, len(events), kinds, 16,
                                           ctypes.byref(n), s), "pl_smooth_frame_events")
        return [int(kinds[i]) for i in range(min(n.value, 16))]

    def run_fused(self, pts: torch.Tensor, s=None) -> None:
        """The same outputs as run() (except the unfiltered normals, which
        stay internal) through pl_smooth_frame: three to a few launches
        instead of six."""
        f = self._fused_frame(pts)
        f.pts = pts.data_ptr()
        s = _stream(self.device) if s is None else s
        _check(_lib.pl_smooth_frame(ctypes.byref(f), self.ndt, _ptr(self.ws_frame),
                                    self._ws_frame_n, s), "pl_smooth_frame")


PL_LAUNCH_LAPLACIAN, PL_LAUNCH_BILATERAL, PL_LAUNCH_NORMALS, PL_LAUNCH_GATHER = 1, 2, 4, 8
PL_LAUNCH_MESH_COUNT, PL_LAUNCH_MESH_EMIT, PL_LAUNCH_GROUPS = 16, 32, 64


def pl_tune_get(stage: int, kernel: int) -> tuple[int, int, int]:
    """(tile_rows, tile_cols, fuse) used for a stage and window size."""
    r, c, f = _i32(), _i32(), _i32()
    _check(_lib.pl_tune_get(stage, kernel, ctypes.byref(r), ctypes.byref(c), ctypes.byref(f)),
           "pl_tune_get")
    return r.value, c.value, f.value


def pl_tune_set(stage: int, kernel: int, tile_rows: int, tile_cols: int, fuse: int) -> None:
    _check(_lib.pl_tune_set(stage, kernel, tile_rows, tile_cols, fuse), "pl_tune_set")


def _marshal_frames(frames: list, ndt: int, halfedges: bool = True, tri_valid: bool = True):
    """PLFrame array over `frames` (dicts: pts [M, N, 3] float32 device tensor,
    kernel_lap, lam, iters_lap, kernel_bil, sigma_length, sigma_angle,
    iters_bil; optionally dominant [l, 3] float32 device tensor, l_max and
    ang_min for group assignment, Alg. 4) with freshly allocated outputs
    (plus groups uint8 [2Q] for frames that give dominant normals); returns
    (array, outputs)."""
    if not frames:
        raise ValueError("a batch needs at least one frame")
    nd = _tdtype(ndt)
    device = frames[0]["pts"].device
    outputs = []
    arr = (PLFrame * len(frames))()
    for i, f in enumerate(frames):
        pts = f["pts"]
        _dev_tensor(pts, torch.float32, f"frames[{i}].pts")
        M, N = int(pts.shape[0]), int(pts.shape[1])
        T = 2 * max(M - 1, 1) * max(N - 1, 1)
        e = lambda shape, dt: torch.empty(shape, dtype=dt, device=device)
        o = dict(points=e((M, N, 3), torch.float32),
                 normals=e((M - 1, N - 1, 2, 3), nd),
                 centroids=e((M - 1, N - 1, 2, 3), torch.float32),
                 tri_valid=e(T, torch.uint8) if tri_valid else None,
                 tri_map=e(T, torch.int32), triangles=e((T, 3), torch.int32),
                 halfedges=e(3 * T, torch.int32) if halfedges else None,
                 n_tri=e(1, torch.int32), normals_T=e((T, 3), nd))
        dom = f.get("dominant")
        if dom is not None:
            _dev_tensor(dom, torch.float32, f"frames[{i}].dominant")
            if dom.dim() != 2 or dom.shape[1] != 3:
                raise ValueError(f"frames[{i}].dominant must be [l, 3]")
            o["groups"] = e(T, torch.uint8)
        outputs.append(o)
        a = arr[i]
        a.pts = pts.data_ptr()
        a.M, a.N = M, N
        a.kernel_lap, a.iters_lap, a.lambda_ = f["kernel_lap"], f["iters_lap"], f["lam"]
        a.kernel_bil, a.iters_bil = f["kernel_bil"], f["iters_bil"]
        a.sigma_length, a.sigma_angle = f["sigma_length"], f["sigma_angle"]
        for key, field in (("points", "pts_out"), ("normals", "normals"),
                           ("centroids", "centroids"), ("tri_valid", "tri_valid"),
                           ("tri_map", "tri_map"), ("triangles", "triangles"),
                           ("halfedges", "halfedges"), ("n_tri", "n_tri"),
                           ("normals_T", "normals_T")):
            setattr(a, field, o[key].data_ptr() if o[key] is not None else None)
        if dom is not None:
            a.dominant = dom.data_ptr() if dom.numel() else None
            a.n_dominant = int(dom.shape[0])
            a.l_max, a.ang_min = float(f["l_max"]), float(f["ang_min"])
            a.groups = o["groups"].data_ptr()
    return arr, outputs


def pl_smooth_batch(frames: list, normal_dtype=torch.float32) -> list:
    """One pass of the whole path over `frames` (as for Batch) through the
    one-shot entry point; returns each frame's output dict."""
    ndt = _ndt(normal_dtype)
    device = frames[0]["pts"].device if frames else None
    arr, outputs = _marshal_frames(frames, ndt)
    ws_n = _lib.pl_batch_workspace(arr, len(frames), ndt)
    if ws_n == 0:
        raise PLError(-1, "pl_batch_workspace")
    ws = torch.empty(ws_n, dtype=torch.uint8, device=device)
    _check(_lib.pl_smooth_batch(arr, len(frames), ndt, _ptr(ws), ws_n, _stream(device)),
           "pl_smooth_batch")
    for o, f in zip(outputs, frames):  # the caching allocator keeps ws until the stream is past
        o["_ws"] = ws
        o["_dominant"] = f.get("dominant")
    return outputs


def pl_smooth_frame(frame: dict, normal_dtype=torch.float32) -> dict:
    """The whole path on one frame (keys as for Batch) through the fused
    single-frame entry point; returns the output dict (points, normals =
    filtered T_FC normals, centroids, tri_valid, tri_map, triangles,
    halfedges, n_tri, normals_T, and groups if dominant normals are given)."""
    ndt = _ndt(normal_dtype)
    device = frame["pts"].device
    arr, outputs = _marshal_frames([frame], ndt)
    ws_n = _lib.pl_smooth_frame_workspace(arr, ndt)
    if ws_n == 0:
        raise PLError(-1, "pl_smooth_frame_workspace")
    ws = torch.empty(ws_n, dtype=torch.uint8, device=device)
    _check(_lib.pl_smooth_frame(arr, ndt, _ptr(ws), ws_n, _stream(device)), "pl_smooth_frame")
    out = outputs[0]
    out["_ws"] = ws                 # the caching allocator keeps it until the stream is past
    out["_dominant"] = frame.get("dominant")
    return out


class Batch:
    """A batch of frames through the whole path with one launch per stage (pl_batch_* in include/pl.h).

    `frames` is a list of dicts with keys pts ([M, N, 3] float32 device
    tensor), kernel_lap, lam, iters_lap, kernel_bil, sigma_length,
    sigma_angle, iters_bil, and optionally dominant ([l, 3] float32 device
    tensor), l_max and ang_min for group assignment (Alg. 4).  Outputs are
    allocated here, once, and stay bound to the plan: outputs[i] holds
    points, normals (filtered, T_FC layout), centroids, tri_valid, tri_map,
    triangles, halfedges, n_tri, normals_T (and groups)."""

    def __init__(self, frames: list, normal_dtype=torch.float32, halfedges: bool = True,
                 tri_valid: bool = True):
        self.ndt = _ndt(normal_dtype)
        arr, self.outputs = _marshal_frames(frames, self.ndt, halfedges, tri_valid)
        self.device = frames[0]["pts"].device
        self.inputs = [f["pts"] for f in frames]
        self._dominant = [f.get("dominant") for f in frames]   # read by every run
        self._frames = arr
        n = len(frames)
        ws_n = _lib.pl_batch_workspace(arr, n, self.ndt)
        if ws_n == 0:
            raise PLError(-1, "pl_batch_workspace")
        self.ws = torch.empty(ws_n, dtype=torch.uint8, device=self.device)
        h = _vp()
        _check(_lib.pl_batch_create(arr, n, self.ndt, _ptr(self.ws), ws_n, _stream(self.device),
                                    ctypes.byref(h)), "pl_batch_create")
        self._h = h
        self.n = n
        self.triangles_total = sum(2 * (int(x.shape[0]) - 1) * (int(x.shape[1]) - 1)
                                   for x in self.inputs)

    def run(self, active: torch.Tensor | None = None) -> None:
        """One pass over the frames with active[i] != 0 (uint8 device tensor
        of length n; None = all frames)."""
        if active is not None:
            _dev_tensor(active, torch.uint8, "active")
        _check(_lib.pl_batch_run(self._h, _ptr(active), _stream(self.device)), "pl_batch_run")

    def capture(self, active: torch.Tensor | None = None, max_active: int | None = None) -> None:
        """Record run(active) into a HIP graph owned by the plan; the graph
        reads the mask's contents at each replay.  With `max_active`, the
        graph is sized for replays with at most that many active frames
        (pl_batch_capture_bounded); the plan keeps one graph per bound.
        Capture happens on a private stream (the legacy default stream
        cannot be captured); nothing executes while recording."""
        if active is not None:
            _dev_tensor(active, torch.uint8, "active")
        self._cap_active = active
        self._cap_stream = torch.cuda.Stream(self.device)
        h = ctypes.c_void_p(self._cap_stream.cuda_stream)
        if max_active is None:
            _check(_lib.pl_batch_capture(self._h, _ptr(active), h), "pl_batch_capture")
        else:
            _check(_lib.pl_batch_capture_bounded(self._h, _ptr(active), int(max_active), h),
                   "pl_batch_capture_bounded")

    def replay(self, n_active: int | None = None) -> None:
        """Launch the captured graph on the current stream; with `n_active`,
        the graph of the smallest captured bound >= n_active (the caller
        guarantees that at most n_active frames are active)."""
        if n_active is None:
            _check(_lib.pl_batch_replay(self._h, _stream(self.device)), "pl_batch_replay")
        else:
            _check(_lib.pl_batch_replay_bounded(self._h, int(n_active), _stream(self.device)),
                   "pl_batch_replay_bounded")

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.pl_batch_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
