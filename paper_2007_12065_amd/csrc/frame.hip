// The whole path on one frame in as few launches as its dependencies allow
// (pl_smooth_frame): mesh (Sec. 4.2, Alg. 1 and Alg. 2), Laplacian (Sec. 2.3
// Eqs. 1-2, Sec. 5.1), centroids and normals, bilateral filter with the
// gather onto T (Eqs. 3-6, Sec. 5.2), and optionally the group labels
// (Sec. 7.1, Alg. 4).  Every launch runs the tile bodies of tiles.h, so the
// outputs equal those of pl_mesh_opc, pl_laplacian, pl_tri_normals and
// pl_bilateral called in turn, bit for bit.
//
// Launch sequence:
//   1. the Laplacian's first pass over its point tiles and, in the same
//      launch, the mesh's validity codes and counts (both read only the
//      input points);
//   2. the Laplacian's further passes, then the bilateral passes.  The first
//      bilateral pass computes the centroids and raw normals of every quad it
//      stages from the smoothed points and writes the centroids, so there is
//      no normals launch and the raw normals never travel through HBM; the
//      last pass gathers onto T.
// The mesh emit (T_map, T, HE) needs every count, so it rides in the second
// launch.  When that one is the gathering bilateral pass, the gather cannot
// read T_map (written by the same launch): it ranks each triangle in T
// from the mesh's codes and segment counts instead (the same numbers), so a
// 480 x 640 frame whose two bilateral sweeps fuse into one pass takes two
// launches.
//
// A launch that carries mesh work has two kinds of workgroups: the filter's
// tiles first, then one workgroup per 256-quad row segment of the mesh.
// (Frames of more than kMeshSegMax segments are meshed by whole quad rows,
// whose emit body needs more registers than the filters may use; they get
// pl_mesh_opc's own two launches before the filters, which at that size
// cost little.)  Each kind is dealt over the eight XCDs on its own (each
// part padded to a multiple of eight workgroups, and xcd_remap_active gives
// each XCD a contiguous run), and mesh workgroups stage their data in the
// same dynamic LDS the filter tiles use.
#include "groups.h"
#include "tiles.h"
#include "tuning.h"

namespace pl {

namespace {

enum MeshKind { kMeshNone = 0, kMeshCount = 1, kMeshEmit = 2 };

struct MeshJob {
    const float *pts;
    uint8_t *codes, *tri_valid;
    int *counts;
    int32_t *tri_map, *tris, *he, *n_tri;
    int cap, Mq, N, S;
    int units;       // row segments, Mq S
    int per_group;   // consecutive segments per workgroup (1)
    int groups;      // mesh workgroups: ceil(units / per_group)
};

// Mesh workgroups of a launch, padded to whole rounds of the eight XCDs.
__host__ __device__ inline int mesh_blocks(const MeshJob &mj) {
    return (mj.groups + kNumXcd - 1) / kNumXcd * kNumXcd;
}

template <int Kind>
__device__ __forceinline__ void mesh_job(const MeshJob &j, int g, float4 *lds) {
    const int k0 = g * j.per_group;
    const int k1 = min(k0 + j.per_group, j.units);
    for (int k = k0; k < k1; ++k) {
        if constexpr (Kind == kMeshCount)
            mesh_count_seg(j.pts, j.N, k / j.S, k % j.S, j.S, j.codes, j.tri_valid, j.counts,
                           *reinterpret_cast<MeshCountSegLds *>(lds));
        else
            mesh_emit_seg(j.codes, j.counts, j.Mq, j.N, k / j.S, k % j.S, j.S, j.tri_map, j.tris,
                          j.he, j.cap, j.n_tri, *reinterpret_cast<MeshEmitSegLds *>(lds));
    }
}

template <int R, int Kind>
__global__ __launch_bounds__(kTileBlock) void k_frame_laplacian(
    const float *__restrict__ src, float *__restrict__ dst, int M, int N, float lam, int F,
    int TH, int TW, int tiles_x, int ntiles, int filter_blocks, MeshJob mj) {
    extern __shared__ float4 lds[];
    const int b = (int)blockIdx.x;
    if (Kind != kMeshNone && b >= filter_blocks) {      // the mesh's workgroups follow the tiles
        const int g = xcd_remap_active(b - filter_blocks, mj.groups);
        if (g >= 0) mesh_job<Kind>(mj, g, lds);
        return;
    }
    const int tile = xcd_remap_active(b, ntiles);
    if (tile < 0) return;
    lap_tile<R>(src, dst, M, N, lam, F, TH, TW, (tile / tiles_x) * TH, (tile % tiles_x) * TW, lds);
}

// FromPts: the first pass (raw normals and centroids from the smoothed points).
// ByCodes: the gathering pass beside the emit, ranking triangles from the
// mesh codes (GatherCodes) instead of reading T_map.
template <int R, typename NT, bool FromPts, int Kind, bool ByCodes = false>
__global__ __launch_bounds__(kTileBlock, kBilWavesPerSimd) void k_frame_bilateral(
    const NT *__restrict__ nin, const float *__restrict__ cen, NT *__restrict__ nout, int Mq,
    int Nq, float ka, float kb, int F, int TQH, int TQW, int tiles_x, int ntiles,
    int filter_blocks, const int32_t *__restrict__ tri_map, NT *__restrict__ nT,
    const float *__restrict__ pts, float *__restrict__ cen_out, MeshJob mj) {
    extern __shared__ float4 lds[];
    const int b = (int)blockIdx.x;
    if (Kind != kMeshNone && b >= filter_blocks) {      // the mesh's workgroups follow the tiles
        const int g = xcd_remap_active(b - filter_blocks, mj.groups);
        if (g >= 0) mesh_job<Kind>(mj, g, lds);
        return;
    }
    const int tile = xcd_remap_active(b, ntiles);
    if (tile < 0) return;
    bil_tile<R, NT, FromPts, ByCodes, bil_frame_lanes<R>()>(
        nin, cen, nout, Mq, Nq, ka, kb, F, TQH, TQW, (tile / tiles_x) * TQH, (tile % tiles_x) * TQW,
        tri_map, nT, lds, pts, cen_out, GatherCodes{mj.codes, mj.counts, mj.S});
}

// Optional record of the launches (pl_smooth_frame_events): an event before
// the first launch and after each one, and what each launch carried.
struct LaunchLog {
    hipEvent_t *ev;
    int n_ev;
    int32_t *kinds;
    int n_kinds;
    int n;
};

pl_status log_start(LaunchLog *log, hipStream_t s) {
    if (!log || log->n_ev < 1) return PL_OK;
    return hip_check(hipEventRecord(log->ev[0], s), "hipEventRecord");
}

pl_status log_launch(LaunchLog *log, int32_t kind, hipStream_t s) {
    if (!log) return PL_OK;
    if (log->n < log->n_kinds && log->kinds) log->kinds[log->n] = kind;
    ++log->n;
    if (log->n < log->n_ev) return hip_check(hipEventRecord(log->ev[log->n], s), "hipEventRecord");
    return PL_OK;
}

int mesh_bits(int kind) {
    return kind == kMeshCount ? PL_LAUNCH_MESH_COUNT : kind == kMeshEmit ? PL_LAUNCH_MESH_EMIT : 0;
}

size_t mesh_lds(int kind) {
    if (kind == kMeshCount) return sizeof(MeshCountSegLds);
    if (kind == kMeshEmit) return sizeof(MeshEmitSegLds);
    return 0;
}

int round8(int x) { return (x + kNumXcd - 1) / kNumXcd * kNumXcd; }

template <int R, int Kind>
pl_status lap_launch(const float *src, float *dst, int M, int N, float lam, int F, TileCfg c,
                     const MeshJob &mj, hipStream_t s) {
    const int tiles_x = (N + c.tw - 1) / c.tw;
    const int ntiles = tiles_x * ((M + c.th - 1) / c.th);
    const int fb = Kind == kMeshNone ? ntiles : round8(ntiles);
    const int grid = fb + (Kind == kMeshNone ? 0 : mesh_blocks(mj));
    size_t lds = lap_lds_bytes(R, F, c.th, c.tw);
    lds = lds > mesh_lds(Kind) ? lds : mesh_lds(Kind);
    if (pl_status st = allow_lds((const void *)k_frame_laplacian<R, Kind>, lds)) return st;
    k_frame_laplacian<R, Kind><<<grid, kTileBlock, lds, s>>>(src, dst, M, N, lam, F, c.th, c.tw,
                                                             tiles_x, ntiles, fb, mj);
    return hip_check(hipGetLastError(), "k_frame_laplacian");
}

template <int R>
pl_status lap_dispatch(int kind, const float *src, float *dst, int M, int N, float lam, int F,
                       TileCfg c, const MeshJob &mj, hipStream_t s) {
    switch (kind) {
    case kMeshCount: return lap_launch<R, kMeshCount>(src, dst, M, N, lam, F, c, mj, s);
    case kMeshEmit: return lap_launch<R, kMeshEmit>(src, dst, M, N, lam, F, c, mj, s);
    default: return lap_launch<R, kMeshNone>(src, dst, M, N, lam, F, c, mj, s);
    }
}

template <int R, typename NT, bool FromPts, int Kind, bool ByCodes = false>
pl_status bil_launch(const NT *nin, const float *cen, NT *nout, int Mq, int Nq, float ka,
                     float kb, int F, TileCfg c, const int32_t *tri_map, NT *nT,
                     const float *pts, float *cen_out, const MeshJob &mj, hipStream_t s) {
    const int tiles_x = (Nq + c.tw - 1) / c.tw;
    const int ntiles = tiles_x * ((Mq + c.th - 1) / c.th);
    const int fb = Kind == kMeshNone ? ntiles : round8(ntiles);
    const int grid = fb + (Kind == kMeshNone ? 0 : mesh_blocks(mj));
    size_t lds = bil_lds_bytes(R, F, c.th, c.tw, bil_waves(R, false));
    lds = lds > mesh_lds(Kind) ? lds : mesh_lds(Kind);
    if (pl_status st = allow_lds((const void *)k_frame_bilateral<R, NT, FromPts, Kind, ByCodes>, lds))
        return st;
    k_frame_bilateral<R, NT, FromPts, Kind, ByCodes><<<grid, kTileBlock, lds, s>>>(
        nin, cen, nout, Mq, Nq, ka, kb, F, c.th, c.tw, tiles_x, ntiles, fb, tri_map, nT, pts,
        cen_out, mj);
    return hip_check(hipGetLastError(), "k_frame_bilateral");
}

template <int R, typename NT>
pl_status bil_dispatch(bool from_pts, int kind, const NT *nin, const float *cen, NT *nout,
                       int Mq, int Nq, float ka, float kb, int F, TileCfg c,
                       const int32_t *tri_map, NT *nT, const float *pts, float *cen_out,
                       const MeshJob &mj, bool gather_codes, hipStream_t s) {
    if (!from_pts)
        return bil_launch<R, NT, false, kMeshNone>(nin, cen, nout, Mq, Nq, ka, kb, F, c, tri_map,
                                                   nT, pts, cen_out, mj, s);
    if (kind == kMeshEmit && gather_codes)
        return bil_launch<R, NT, true, kMeshEmit, true>(nin, cen, nout, Mq, Nq, ka, kb, F, c,
                                                        nullptr, nT, pts, cen_out, mj, s);
    if (kind == kMeshEmit)
        return bil_launch<R, NT, true, kMeshEmit>(nin, cen, nout, Mq, Nq, ka, kb, F, c, tri_map,
                                                  nT, pts, cen_out, mj, s);
    return bil_launch<R, NT, true, kMeshNone>(nin, cen, nout, Mq, Nq, ka, kb, F, c, tri_map, nT,
                                              pts, cen_out, mj, s);
}

template <typename NT>
pl_status run(const pl_frame &f, void *ws, hipStream_t s, LaunchLog *log) {
    const int M = f.M, N = f.N, Mq = M - 1, Nq = N - 1;
    const size_t P = (size_t)M * N, Q = (size_t)Mq * Nq, T = 2 * Q;
    char *w = static_cast<char *>(ws);
    MeshJob mj{};
    mj.pts = f.pts;
    mj.codes = reinterpret_cast<uint8_t *>(w);
    mj.counts = reinterpret_cast<int *>(w + align_up(Q, 256));
    mj.tri_valid = f.tri_valid;
    mj.tri_map = f.tri_map;
    mj.tris = f.triangles;
    mj.he = f.halfedges;
    mj.n_tri = f.n_tri;
    mj.cap = (int)T;
    mj.Mq = Mq;
    mj.N = N;
    mj.S = mesh_segments(Nq);
    mj.units = Mq * mj.S;
    // one row segment per workgroup: several per workgroup (fewer, longer
    // mesh workgroups) left the emit finishing after the filter's tiles
    mj.per_group = 1;
    mj.groups = mj.units;
    // frames meshed by whole rows: pl_mesh_opc's launches first, and no
    // mesh work in the filter launches
    const bool rows = (long)Mq * mj.S > kMeshSegMax;
    if (pl_status st = log_start(log, s)) return st;
    if (rows) {
        if (pl_status st = launch_mesh(f.pts, M, N, f.tri_valid, f.tri_map, f.triangles,
                                       f.halfedges, (int)T, f.n_tri, ws, s))
            return st;
        if (pl_status st = log_launch(log, PL_LAUNCH_MESH_COUNT, s)) return st;
        if (pl_status st = log_launch(log, PL_LAUNCH_MESH_EMIT, s)) return st;
    }
    w += mesh_workspace(M, N);
    float *lap_tmp = f.iters_lap > 1 ? reinterpret_cast<float *>(w) : nullptr;
    w += f.iters_lap > 1 ? align_up(12 * P, 256) : 0;
    NT *bil_tmp = f.iters_bil > 1 ? reinterpret_cast<NT *>(w) : nullptr;

    const int Rl = f.kernel_lap / 2, Rb = f.kernel_bil / 2;
    const TileCfg cl = tile_cfg(frame_stage(true, M, N), Rl), cb = tile_cfg(frame_stage(false, M, N), Rb);
    const int Ll = f.iters_lap == 0 ? 1 : (f.iters_lap + cl.fuse - 1) / cl.fuse;
    const int Lb = f.iters_bil == 0 ? 1 : (f.iters_bil + cb.fuse - 1) / cb.fuse;

    const float *cur = f.pts;
    int left = f.iters_lap;
    for (int l = 0; l < Ll; ++l) {
        const int F = left < cl.fuse ? left : cl.fuse;
        left -= F;
        float *dst = ((Ll - 1 - l) % 2 == 0) ? f.pts_out : lap_tmp;    // last lands in pts_out
        const int kind = rows ? kMeshNone : l == 0 ? kMeshCount : (l == 1 ? kMeshEmit : kMeshNone);
        pl_status st;
        switch (Rl) {
        case 1: st = lap_dispatch<1>(kind, cur, dst, M, N, f.lambda, F, cl, mj, s); break;
        case 2: st = lap_dispatch<2>(kind, cur, dst, M, N, f.lambda, F, cl, mj, s); break;
        case 3: st = lap_dispatch<3>(kind, cur, dst, M, N, f.lambda, F, cl, mj, s); break;
        default: st = lap_dispatch<4>(kind, cur, dst, M, N, f.lambda, F, cl, mj, s); break;
        }
        if (st) return st;
        if (pl_status e = log_launch(log, PL_LAUNCH_LAPLACIAN | mesh_bits(kind) | (F << 8), s))
            return e;
        cur = dst;
    }

    const float log2e = 1.4426950408889634f;
    const float ka = log2e / (2.0f * f.sigma_length * f.sigma_length);
    const float kb = log2e / (2.0f * f.sigma_angle * f.sigma_angle);
    NT *nout = static_cast<NT *>(f.normals);
    NT *nT = static_cast<NT *>(f.normals_T);
    const NT *ncur = nullptr;
    left = f.iters_bil;
    for (int l = 0; l < Lb; ++l) {
        const int F = left < cb.fuse ? left : cb.fuse;
        left -= F;
        const bool last = l == Lb - 1;
        NT *dst = ((Lb - 1 - l) % 2 == 0) ? nout : bil_tmp;             // last lands in normals
        // the emit rides in the second launch; when that is the gathering
        // pass, the gather ranks the triangles from the mesh codes itself
        const int kind = (!rows && Ll + l == 1) ? kMeshEmit : kMeshNone;
        const bool by_codes = last && kind == kMeshEmit;
        const int32_t *tm = last && !by_codes ? f.tri_map : nullptr;
        pl_status st;
        switch (Rb) {
        case 1: st = bil_dispatch<1, NT>(l == 0, kind, ncur, f.centroids, dst, Mq, Nq, ka, kb, F, cb, tm, nT, f.pts_out, f.centroids, mj, by_codes, s); break;
        case 2: st = bil_dispatch<2, NT>(l == 0, kind, ncur, f.centroids, dst, Mq, Nq, ka, kb, F, cb, tm, nT, f.pts_out, f.centroids, mj, by_codes, s); break;
        case 3: st = bil_dispatch<3, NT>(l == 0, kind, ncur, f.centroids, dst, Mq, Nq, ka, kb, F, cb, tm, nT, f.pts_out, f.centroids, mj, by_codes, s); break;
        default: st = bil_dispatch<4, NT>(l == 0, kind, ncur, f.centroids, dst, Mq, Nq, ka, kb, F, cb, tm, nT, f.pts_out, f.centroids, mj, by_codes, s); break;
        }
        if (st) return st;
        const int32_t what = PL_LAUNCH_BILATERAL | (l == 0 ? PL_LAUNCH_NORMALS : 0) |
                             (last ? PL_LAUNCH_GATHER : 0) | mesh_bits(kind) | (F << 8);
        if (pl_status e = log_launch(log, what, s)) return e;
        ncur = dst;
    }

    if (f.groups) {
        if (pl_status st = launch_group_assign(f.pts_out, (int)P, f.triangles, f.normals_T,
                                               sizeof(NT) == 4 ? PL_F32 : PL_F16, f.n_tri,
                                               (int)T, f.dominant, f.n_dominant, f.l_max,
                                               f.ang_min, f.groups, s))
            return st;
        return log_launch(log, PL_LAUNCH_GROUPS, s);
    }
    return PL_OK;
}

}  // namespace

size_t smooth_frame_workspace(const pl_frame &f, pl_dtype ndt) {
    const size_t P = (size_t)f.M * f.N, T = 2 * (size_t)(f.M - 1) * (f.N - 1);
    return mesh_workspace(f.M, f.N) + (f.iters_lap > 1 ? align_up(12 * P, 256) : 0) +
           (f.iters_bil > 1 ? align_up(T * 3 * (ndt == PL_F32 ? 4 : 2), 256) : 0);
}

pl_status launch_smooth_frame(const pl_frame &f, pl_dtype ndt, void *ws, hipStream_t s,
                              hipEvent_t *events, int n_events, int32_t *kinds, int n_kinds,
                              int32_t *n_launches) {
    LaunchLog log{events, n_events, kinds, n_kinds, 0};
    LaunchLog *lp = (events && n_events > 0) || (kinds && n_kinds > 0) || n_launches ? &log
                                                                                      : nullptr;
    const pl_status st = ndt == PL_F32 ? run<float>(f, ws, s, lp) : run<__half>(f, ws, s, lp);
    if (n_launches) *n_launches = log.n;
    return st;
}

}  // namespace pl
