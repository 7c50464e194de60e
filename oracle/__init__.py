"""FP64 CPU oracle for organized-point-cloud meshing and smoothing.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the GPU library never does, and the
two share no code.

Every function promotes its float32 input to float64 and calls the C routines
in ``pl_oracle.c`` (each cites the passage of the paper it follows).  Array
layouts match the GPU library: points ``[M, N, 3]``; per-triangle arrays in GID
order ``[M-1, N-1, 2, 3]`` with GID = 2 (u (N-1) + v) + k (Sec. 4.2).

Parity unpinned: ``vertex_update`` (the paper gives no formula for the vertex
update; its pins check a restatement of the cited method's update).  Every
other function is pinned by the tests to what the paper and the mathematics
fix.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pl_oracle.c")
# PL_ORACLE_LIBRARY names another build of the same C file (the sanitizer
# build of paper_2007_12065_amd/sanitize.py); by default the in-tree one
_LIB = os.environ.get("PL_ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
_lib = None

__all__ = ["build", "mesh", "halfedges", "laplacian", "tri_normals",
           "bilateral", "gather", "pipeline", "group_assign", "ga_icosahedron", "ga_integrate",
           "user_halfedges", "vertex_update"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FP contraction).
    A library named by PL_ORACLE_LIBRARY is used as it is."""
    if os.environ.get("PL_ORACLE_LIBRARY"):
        return _LIB
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
            "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i32, i64, dbl = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        vp = ctypes.c_void_p
        lib.oracle_mesh_triangles.argtypes = [vp, i32, i32, vp, vp]
        lib.oracle_mesh_triangles.restype = i64
        lib.oracle_mesh_halfedges.argtypes = [vp, i32, i32, i64, vp]
        lib.oracle_mesh_halfedges.restype = None
        lib.oracle_laplacian.argtypes = [vp, vp, i32, i32, i32, dbl, i32, i32]
        lib.oracle_laplacian.restype = None
        lib.oracle_tri_normals.argtypes = [vp, i32, i32, vp, vp, i32]
        lib.oracle_tri_normals.restype = None
        lib.oracle_bilateral.argtypes = [vp, vp, i32, i32, i32, dbl, dbl, i32, vp, i32]
        lib.oracle_bilateral.restype = None
        lib.oracle_gather.argtypes = [vp, vp, i32, i32, vp]
        lib.oracle_gather.restype = None
        lib.oracle_group_assign.argtypes = [vp, i64, vp, i64, vp, vp, i32,
                                            ctypes.c_float, ctypes.c_float, vp]
        lib.oracle_group_assign.restype = None
        lib.oracle_ga_sizes.argtypes = [i32, vp, vp]
        lib.oracle_ga_sizes.restype = i32
        lib.oracle_ga_icosahedron.argtypes = [i32, vp, vp, vp]
        lib.oracle_ga_icosahedron.restype = i32
        lib.oracle_ga_integrate.argtypes = [vp, i32, vp, i64, i32, vp, vp]
        lib.oracle_ga_integrate.restype = None
        lib.oracle_user_halfedges.argtypes = [vp, i64, vp]
        lib.oracle_user_halfedges.restype = None
        lib.oracle_vertex_update.argtypes = [vp, i32, i32, vp, i32, vp, i32]
        lib.oracle_vertex_update.restype = None
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def mesh(pts):
    """Alg. 1: returns (tri_map int32 [2(M-1)(N-1)], triangles int32 [n, 3])."""
    p = _f64(pts)
    M, N = p.shape[:2]
    Q2 = 2 * (M - 1) * (N - 1)
    tri_map = np.empty(Q2, dtype=np.int32)
    tris = np.empty((max(Q2, 1), 3), dtype=np.int32)
    n = _load().oracle_mesh_triangles(_ptr(p), M, N, _ptr(tri_map), _ptr(tris))
    return tri_map, tris[:n].copy()


def halfedges(tri_map, M: int, N: int, n_tri: int):
    """Alg. 2: twin half-edge array int32 [3 n_tri], -1 = border."""
    tm = np.ascontiguousarray(tri_map, dtype=np.int32)
    he = np.empty(max(3 * n_tri, 1), dtype=np.int32)
    _load().oracle_mesh_halfedges(_ptr(tm), M, N, n_tri, _ptr(he))
    return he[:3 * n_tri].copy()


def laplacian(pts, kernel: int, lam: float, iterations: int, threads: int = 1):
    """Eqs. (1)-(2), Sec. 5.1: smoothed points float64 [M, N, 3]."""
    p = _f64(pts)
    M, N = p.shape[:2]
    out = np.empty_like(p)
    _load().oracle_laplacian(_ptr(p), _ptr(out), M, N, kernel, lam, iterations, threads)
    return out


def tri_normals(pts, threads: int = 1):
    """Sec. 5.2: (normals, centroids), each float64 [M-1, N-1, 2, 3]."""
    p = _f64(pts)
    M, N = p.shape[:2]
    n = np.empty((M - 1, N - 1, 2, 3), dtype=np.float64)
    c = np.empty_like(n)
    _load().oracle_tri_normals(_ptr(p), M, N, _ptr(n), _ptr(c), threads)
    return n, c


def bilateral(normals, centroids, kernel: int, sigma_length: float,
              sigma_angle: float, iterations: int, threads: int = 1):
    """Eqs. (3)-(6), Sec. 5.2: filtered normals float64 [M-1, N-1, 2, 3]."""
    n = _f64(normals)
    c = _f64(centroids)
    Mq, Nq = n.shape[:2]
    out = np.empty_like(n)
    _load().oracle_bilateral(_ptr(n), _ptr(c), Mq + 1, Nq + 1, kernel,
                             sigma_length, sigma_angle, iterations, _ptr(out), threads)
    return out


def gather(normals, tri_map, n_tri: int):
    """Sec. 5.2: normals of the final mesh T, float64 [n_tri, 3]."""
    n = _f64(normals)
    Mq, Nq = n.shape[:2]
    tm = np.ascontiguousarray(tri_map, dtype=np.int32)
    out = np.full((max(n_tri, 1), 3), np.nan, dtype=np.float64)
    _load().oracle_gather(_ptr(n), _ptr(tm), Mq + 1, Nq + 1, _ptr(out))
    return out[:n_tri].copy()


def pipeline(pts, kernel_lap: int, lam: float, iters_lap: int, kernel_bil: int,
             sigma_length: float, sigma_angle: float, iters_bil: int,
             threads: int = 1) -> dict:
    """The whole path on one frame, in the paper's order: mesh (Alg. 1-2),
    Laplacian, centroids and normals, bilateral, gather to T."""
    M, N = pts.shape[:2]
    tri_map, tris = mesh(pts)
    he = halfedges(tri_map, M, N, len(tris))
    smooth = laplacian(pts, kernel_lap, lam, iters_lap, threads)
    normals, centroids = tri_normals(smooth, threads)
    filtered = bilateral(normals, centroids, kernel_bil, sigma_length,
                         sigma_angle, iters_bil, threads)
    normals_T = gather(filtered, tri_map, len(tris))
    return dict(tri_map=tri_map, triangles=tris, halfedges=he, points=smooth,
                normals=normals, centroids=centroids, filtered=filtered,
                normals_T=normals_T)


def group_assign(points, triangles, normals, dominant, l_max: float, ang_min: float):
    """Alg. 4 (Sec. 7.1): group label uint8 [n] of every triangle of T.

    `points` float32 [..., 3] (the smoothed vertices; flattened), `triangles`
    int32 [n, 3] vertex indices, `normals` [n, 3] (the filtered normals of T,
    converted to float32), `dominant` [l, 3] dominant plane normals.  The
    decisions are taken in float32 (see oracle_group_assign)."""
    p = np.ascontiguousarray(np.asarray(points, dtype=np.float32).reshape(-1, 3))
    t = np.ascontiguousarray(np.asarray(triangles, dtype=np.int32).reshape(-1, 3))
    n = np.ascontiguousarray(np.asarray(normals, dtype=np.float32).reshape(-1, 3))
    d = np.ascontiguousarray(np.asarray(dominant, dtype=np.float32).reshape(-1, 3))
    if len(n) != len(t):
        raise ValueError("one normal per triangle")
    out = np.empty(max(len(t), 1), dtype=np.uint8)
    _load().oracle_group_assign(_ptr(p), len(p), _ptr(t), len(t), _ptr(n), _ptr(d), len(d),
                                float(l_max), float(ang_min), _ptr(out))
    return out[:len(t)].copy()


def ga_icosahedron(level: int):
    """Sec. 6.1.1: the refined icosahedron of `level` as (vertices float64
    [V, 3], faces int32 [F, 3], cell normals float32 [F, 3])."""
    lib = _load()
    nv, nf = ctypes.c_int64(), ctypes.c_int64()
    if lib.oracle_ga_sizes(int(level), ctypes.byref(nv), ctypes.byref(nf)) != 0:
        raise ValueError("level must be in [0, 7]")
    V = np.empty((nv.value, 3), dtype=np.float64)
    F = np.empty((nf.value, 3), dtype=np.int32)
    C = np.empty((nf.value, 3), dtype=np.float32)
    if lib.oracle_ga_icosahedron(int(level), _ptr(V), _ptr(F), _ptr(C)) != 0:
        raise RuntimeError("icosahedron refinement produced the wrong vertex count")
    return V, F, C


def ga_integrate(cells, normals, stride: int = 1):
    """Alg. 3 by definition (Sec. 6.1.3): (cell index int32 per integrated
    row, counts uint32 [n_cells]) for rows 0, stride, 2 stride, ... of the
    float32 normals (decisions in float32, see oracle_ga_integrate)."""
    c = np.ascontiguousarray(np.asarray(cells, dtype=np.float32).reshape(-1, 3))
    n = np.ascontiguousarray(np.asarray(normals, dtype=np.float32).reshape(-1, 3))
    if stride < 1:
        raise ValueError("stride must be >= 1")
    rows = (len(n) + stride - 1) // stride
    idx = np.empty(max(rows, 1), dtype=np.int32)
    counts = np.zeros(len(c), dtype=np.uint32)
    _load().oracle_ga_integrate(_ptr(c), len(c), _ptr(n), len(n), int(stride), _ptr(idx),
                                _ptr(counts))
    return idx[:rows].copy(), counts


def user_halfedges(triangles):
    """Sec. 4.3: twin of every half-edge of a user mesh (int32 [3 n]); edges
    shared by more than two triangles keep the first pair (option 1, see
    oracle_user_halfedges)."""
    t = np.ascontiguousarray(np.asarray(triangles, dtype=np.int32).reshape(-1, 3))
    out = np.empty(max(3 * len(t), 1), dtype=np.int32)
    _load().oracle_user_halfedges(_ptr(t), len(t), _ptr(out))
    return out[:3 * len(t)].copy()


def vertex_update(pts, normals, iterations: int, threads: int = 1):
    """Vertex update from filtered normals (the second stage of bilateral
    mesh denoising, Sun et al. 2007, restated; see oracle_vertex_update):
    float64 [M, N, 3]."""
    p = _f64(pts)
    M, N = p.shape[:2]
    n = _f64(normals)
    if n.shape != (M - 1, N - 1, 2, 3):
        raise ValueError("normals must be [M-1, N-1, 2, 3]")
    out = np.empty_like(p)
    _load().oracle_vertex_update(_ptr(p), M, N, _ptr(n), int(iterations), _ptr(out), threads)
    return out
