// Batched path: many frames of different sizes and filter settings through
// the whole pipeline with one launch per stage (per sweep pass for the
// filters), whatever the number of frames.
//
// Plan (pl_batch_create, host): validates every frame, lays out a workspace
// holding one descriptor per frame, the per-pass source/destination tables
// of the multi-sweep stages, each stage's per-frame tile counts and the
// per-frame scratch (validity codes, row counts, ping-pong buffers), uploads
// the tables once and sizes each launch for all frames active.
//
// Run (pl_batch_run, device only, graph-capturable), over the frames whose
// entry in a device-side activity mask is non-zero:
//   k_batch_prepare    one workgroup per stage: prefix sums of the active
//                      frames' tile counts (the stage's tile queue)
//   k_batch_mesh_count tiles = (frame, quad row)        -> codes, row counts
//   k_batch_mesh_emit  tiles = (frame, quad row)        -> T_map, T, HE, |T|
//   k_batch_laplacian  one launch per sweep pass, tiles = (frame, point tile)
//   k_batch_bilateral  one launch per sweep pass, tiles = (frame, quad tile);
//                      the first pass computes the raw normals and centroids
//                      from the smoothed points while staging its tiles (and
//                      writes the centroids), so there is no normals stage;
//                      the frame's last pass gathers onto T
//   k_batch_groups     tiles = (frame, 1024 rows of T)  -> group labels
//                      (frames that asked for them)
// Every tile runs the same device body as the single-frame kernels
// (tiles.h), so each frame's outputs equal its single-frame results.
//
// Tile queue.  A stage's tiles are numbered frame by frame over the active
// frames only; the launch has one workgroup per tile of the whole batch and
// the hardware dispatcher hands them out as CUs free up.  Workgroup b takes
// a tile number by XCD: the dispatcher deals workgroups round-robin over the
// eight XCDs, and each XCD takes one contiguous eighth of the ACTIVE total
// (not of the grid, which is sized for a bound on the active frames), so
// neighbouring tiles, which share halo lines, meet in the same L2 and all
// eight XCDs share the work however few frames are active.  Workgroups past
// their XCD's share exit at once.  The number is mapped back to (frame,
// tile) by binary search over the prefix sums staged in LDS.  (A
// persistent grid popping tiles from per-XCD atomic counters was measured
// slower: contended device-scope atomics put a floor of several hundred
// microseconds under every stage of a 64-frame batch.)
#include "groups.h"
#include "tiles.h"
#include "tuning.h"

#include <algorithm>
#include <climits>
#include <cstring>
#include <map>
#include <new>
#include <vector>

namespace pl {

namespace {

struct BFrame {
    const float *pts;
    float *pts_out, *lap_tmp;
    void *normals, *bil_tmp;
    float *centroids;
    uint8_t *tri_valid, *codes;
    int32_t *tri_map, *triangles, *halfedges, *n_tri;
    int *row_count;
    void *normals_T;
    int M, N, Mq, Nq;
    int Rl, Rb;
    float lam, ka, kb;
    int lap_th, lap_tw, lap_tiles_x;
    int bil_th, bil_tw, bil_tiles_x;
    const float *dom;              // group assignment (groups != nullptr)
    uint8_t *groups;
    int n_dom;
    float lmax2, ang_min;
};

struct PassFrame {                 // one frame's part of one sweep pass
    const void *src;
    void *dst;
    int F;                         // sweeps in this pass (0: copy)
    int gather;                    // bilateral: last pass, gather onto T
};

struct QueueDev {                  // one stage's tile queue, in the workspace
    const int *count;              // [n] tiles of each frame in this stage
    int *start;                    // [n + 1] prefix over active frames (per run)
};

// Per run, for every queue (one workgroup each): exclusive prefix sums of
// the active frames' tile counts, the total in start[n].
__global__ __launch_bounds__(kTileBlock) void k_batch_prepare(const QueueDev *__restrict__ qs,
                                                             int n,
                                                             const uint8_t *__restrict__ active) {
    __shared__ int wsum[kTileBlock / kWave];
    __shared__ int carry_s;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const QueueDev Q = qs[blockIdx.x];
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < n; base += kTileBlock) {
        const int i = base + threadIdx.x;
        const int x = (i < n && active[i]) ? Q.count[i] : 0;
        const int incl = wave_inclusive_scan(x);
        if (lane == kWave - 1) wsum[wid] = incl;
        __syncthreads();
        int before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < kTileBlock / kWave; ++w) {
            before += w < wid ? wsum[w] : 0;
            all += wsum[w];
        }
        const int carry = carry_s;
        if (i < n) Q.start[i] = carry + before + incl - x;
        __syncthreads();
        if (threadIdx.x == 0) carry_s = carry + all;
        __syncthreads();
    }
    if (threadIdx.x == 0) Q.start[n] = carry_s;
}

constexpr int kLdsFrames = 256;    // prefix sums staged in LDS up to this many frames

// This workgroup's tile: false when its number is past the active total
// (the whole workgroup then exits).
__device__ __forceinline__ bool queue_tile(const QueueDev &Q, int n, int *s_start, int2 &t) {
    // the number depends only on blockIdx and the active total, so a
    // workgroup without a tile leaves before touching LDS or a barrier
    const int g = xcd_remap_active((int)blockIdx.x, Q.start[n]);
    if (g < 0) return false;
    for (int i = threadIdx.x; i <= n && i <= kLdsFrames; i += kTileBlock) s_start[i] = Q.start[i];
    __syncthreads();
    const int *start = n <= kLdsFrames ? s_start : Q.start;
    int lo = 0, hi = n;                       // last frame with start <= g
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (start[mid] <= g) lo = mid; else hi = mid;
    }
    // uniform across the workgroup: frame descriptors then load into SGPRs
    t = make_int2(__builtin_amdgcn_readfirstlane(lo), __builtin_amdgcn_readfirstlane(g - start[lo]));
    return true;
}

#define PL_QUEUE_TILE(Q, n, t)                                              \
    __shared__ int s_start_[kLdsFrames + 1];                                \
    int2 t;                                                                 \
    if (!queue_tile(Q, n, s_start_, t)) return;

__global__ __launch_bounds__(kTileBlock) void k_batch_mesh_count(const BFrame *__restrict__ fr,
                                                                 QueueDev Q, int n) {
    PL_QUEUE_TILE(Q, n, t)
    __shared__ MeshCountRowLds L;
    const BFrame &f = fr[t.x];
    mesh_count_row(f.pts, f.N, t.y, f.codes, f.tri_valid, f.row_count, L);
}

__global__ __launch_bounds__(kTileBlock) void k_batch_mesh_emit(const BFrame *__restrict__ fr,
                                                                QueueDev Q, int n) {
    PL_QUEUE_TILE(Q, n, t)
    const BFrame &f = fr[t.x];
    __shared__ MeshEmitRowLds L;
    mesh_emit_row(f.codes, f.row_count, f.Mq, f.N, t.y, f.tri_map, f.triangles, f.halfedges,
                  2 * f.Mq * f.Nq, f.n_tri, L);
}

template <int R>
__global__ __launch_bounds__(kTileBlock) void k_batch_laplacian(const BFrame *__restrict__ fr,
                                                                const PassFrame *__restrict__ pass,
                                                                QueueDev Q, int n) {
    extern __shared__ float4 lds[];
    PL_QUEUE_TILE(Q, n, t)
    const BFrame &f = fr[t.x];
    const PassFrame &p = pass[t.x];
    const int ty0 = (t.y / f.lap_tiles_x) * f.lap_th, tx0 = (t.y % f.lap_tiles_x) * f.lap_tw;
    lap_tile<R>(static_cast<const float *>(p.src), static_cast<float *>(p.dst), f.M, f.N, f.lam,
                p.F, f.lap_th, f.lap_tw, ty0, tx0, lds);
}

// FromPts: the first pass (raw normals and centroids from the points).
template <int R, typename NT, bool FromPts>
__global__ __launch_bounds__(kTileBlock, kBilWavesPerSimd) void k_batch_bilateral(const BFrame *__restrict__ fr,
                                                                const PassFrame *__restrict__ pass,
                                                                QueueDev Q, int n) {
    extern __shared__ float4 lds[];
    PL_QUEUE_TILE(Q, n, t)
    const BFrame &f = fr[t.x];
    const PassFrame &p = pass[t.x];
    const int qy0 = (t.y / f.bil_tiles_x) * f.bil_th, qx0 = (t.y % f.bil_tiles_x) * f.bil_tw;
    bil_tile<R, NT, FromPts, false, bil_batch_lanes<R>()>(
        FromPts ? nullptr : static_cast<const NT *>(p.src), f.centroids, static_cast<NT *>(p.dst),
        f.Mq, f.Nq, f.ka, f.kb, p.F, f.bil_th, f.bil_tw, qy0, qx0, p.gather ? f.tri_map : nullptr,
        static_cast<NT *>(f.normals_T), lds, f.pts_out, f.centroids);
}

static_assert(kGroupBlock == kTileBlock, "queue tiles are staged by kTileBlock threads");

template <typename NT>
__global__ __launch_bounds__(kGroupBlock) void k_batch_groups(const BFrame *__restrict__ fr,
                                                              QueueDev Q, int n) {
    PL_QUEUE_TILE(Q, n, t)
    const BFrame &f = fr[t.x];
    const int cap = 2 * f.Mq * f.Nq;
    group_rows<NT>(f.pts_out, f.M * f.N, f.triangles, static_cast<const NT *>(f.normals_T),
                   f.n_tri, cap, f.dom, f.n_dom, f.lmax2, f.ang_min, f.groups,
                   (t.y * kGroupBlock + (int)threadIdx.x) * kGroupPer);
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

struct Layout {                    // byte offsets inside the workspace
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += align_up(bytes == 0 ? 1 : bytes, 256);
        return o;
    }
};

struct HostQueue {
    std::vector<int> count;        // [n] tiles per frame
    size_t off_count = 0, off_start = 0;
    long max_tiles = 0;            // all frames active: the launch's workgroups
    std::vector<long> top;         // [k]: tiles of the k frames with the most (k = 0..n)
    int grid = 0;
    size_t lds = 0;
};

struct Pass {                      // one sweep pass: one launch per window radius
    std::vector<PassFrame> tab;    // [n]
    size_t off = 0;
    HostQueue q[kMaxRadius];       // q[R - 1]: the frames with window radius R
};

size_t nt_size(pl_dtype ndt) { return ndt == PL_F32 ? 4 : 2; }

int passes_for(int iters, int fuse) { return iters == 0 ? 1 : (iters + fuse - 1) / fuse; }

}  // namespace

}  // namespace pl

struct pl_batch_s {
    int n = 0;
    pl_dtype ndt = PL_F32;
    uint8_t *ws = nullptr;
    size_t off_frames = 0, off_queues = 0, off_ones = 0;
    int n_queues = 0;              // stage queues with any tile, in table order
    pl::HostQueue mc, me;          // mesh count, mesh emit
    pl::HostQueue grp;             // group assignment (frames with groups)
    std::vector<pl::Pass> lap, bil;
    std::map<int, hipGraphExec_t> graphs;   // bound on active frames -> captured run
};

namespace pl {

namespace {

std::vector<HostQueue *> all_queues(pl_batch_s &b) {
    std::vector<HostQueue *> qs = {&b.mc, &b.me};
    auto any = [](const HostQueue &q) {
        return std::any_of(q.count.begin(), q.count.end(), [](int c) { return c > 0; });
    };
    for (auto *passes : {&b.lap, &b.bil})
        for (auto &p : *passes)
            for (HostQueue &q : p.q)
                if (any(q)) qs.push_back(&q);
    if (any(b.grp)) qs.push_back(&b.grp);
    return qs;
}

}  // namespace

// Workspace layout of a batch; with a plan, also fills and uploads the
// tables (synchronising `stream` once).  Returns the workspace size, or 0
// if the upload failed.
size_t batch_layout(const pl_frame *frames, int n, pl_dtype ndt, pl_batch_s *plan,
                    hipStream_t stream) {
    Layout L;
    pl_batch_s tmp;
    pl_batch_s &b = plan ? *plan : tmp;
    b.n = n;
    b.ndt = ndt;
    b.off_frames = L.take(sizeof(BFrame) * n);
    int maxlap = 0, maxbil = 0;
    for (int i = 0; i < n; ++i) {
        const pl_frame &f = frames[i];
        maxlap = std::max(maxlap, passes_for(f.iters_lap, tile_cfg(kStageBatchLaplacian, f.kernel_lap / 2).fuse));
        maxbil = std::max(maxbil, passes_for(f.iters_bil, tile_cfg(kStageBatchBilateral, f.kernel_bil / 2).fuse));
    }
    b.lap.assign(maxlap, Pass());
    b.bil.assign(maxbil, Pass());
    for (auto &p : b.lap) { p.tab.assign(n, PassFrame{}); p.off = L.take(sizeof(PassFrame) * n); }
    for (auto &p : b.bil) { p.tab.assign(n, PassFrame{}); p.off = L.take(sizeof(PassFrame) * n); }
    for (HostQueue *q : {&b.mc, &b.me, &b.grp}) q->count.assign(n, 0);
    for (auto *passes : {&b.lap, &b.bil})
        for (auto &p : *passes)
            for (HostQueue &q : p.q) q.count.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        const pl_frame &f = frames[i];
        const int Mq = f.M - 1, Nq = f.N - 1;
        b.mc.count[i] = Mq;
        b.me.count[i] = Mq;
        const TileCfg cl = tile_cfg(kStageBatchLaplacian, f.kernel_lap / 2);
        const TileCfg cb = tile_cfg(kStageBatchBilateral, f.kernel_bil / 2);
        const int ltiles = ((f.N + cl.tw - 1) / cl.tw) * ((f.M + cl.th - 1) / cl.th);
        const int btiles = ((Nq + cb.tw - 1) / cb.tw) * ((Mq + cb.th - 1) / cb.th);
        const int lp = passes_for(f.iters_lap, cl.fuse), bp = passes_for(f.iters_bil, cb.fuse);
        for (int p = 0; p < lp; ++p) b.lap[p].q[f.kernel_lap / 2 - 1].count[i] = ltiles;
        for (int p = 0; p < bp; ++p) b.bil[p].q[f.kernel_bil / 2 - 1].count[i] = btiles;
        const long rows_per_tile = (long)kGroupBlock * kGroupPer;
        if (f.groups) b.grp.count[i] = (int)((2L * Mq * Nq + rows_per_tile - 1) / rows_per_tile);
    }
    const std::vector<HostQueue *> qs = all_queues(b);
    for (HostQueue *q : qs) {
        q->off_count = L.take(sizeof(int) * n);
        q->off_start = L.take(sizeof(int) * (n + 1));
        q->max_tiles = 0;
        for (int c : q->count) q->max_tiles += c;
        std::vector<int> sorted(q->count);
        std::sort(sorted.begin(), sorted.end(), [](int a, int c) { return a > c; });
        q->top.assign(n + 1, 0);
        for (int k = 0; k < n; ++k) q->top[k + 1] = q->top[k] + sorted[k];
    }
    b.off_queues = L.take(sizeof(QueueDev) * qs.size());
    b.n_queues = (int)qs.size();
    b.off_ones = L.take(n);
    const size_t table_end = L.off;
    // per-frame scratch
    std::vector<BFrame> bf(n);
    std::vector<size_t> o_codes(n), o_rows(n), o_lap(n, 0), o_bil(n, 0);
    for (int i = 0; i < n; ++i) {
        const pl_frame &f = frames[i];
        const size_t Q = (size_t)(f.M - 1) * (f.N - 1);
        const size_t T = 2 * Q;
        o_codes[i] = L.take(Q);
        o_rows[i] = L.take(sizeof(int) * (f.M - 1));
        const int lp = passes_for(f.iters_lap, tile_cfg(kStageBatchLaplacian, f.kernel_lap / 2).fuse);
        const int bp = passes_for(f.iters_bil, tile_cfg(kStageBatchBilateral, f.kernel_bil / 2).fuse);
        if (lp > 1) o_lap[i] = L.take(12 * (size_t)f.M * f.N);
        if (bp > 1) o_bil[i] = L.take(3 * T * nt_size(ndt));
    }
    if (!plan) return L.off;

    uint8_t *base = b.ws;
    const float log2e = 1.4426950408889634f;
    for (int i = 0; i < n; ++i) {
        const pl_frame &f = frames[i];
        BFrame &d = bf[i];
        d.codes = base + o_codes[i];
        d.row_count = reinterpret_cast<int *>(base + o_rows[i]);
        d.lap_tmp = o_lap[i] ? reinterpret_cast<float *>(base + o_lap[i]) : nullptr;
        d.bil_tmp = o_bil[i] ? static_cast<void *>(base + o_bil[i]) : nullptr;
        d.pts = f.pts;
        d.pts_out = f.pts_out;
        d.normals = f.normals;
        d.centroids = f.centroids;
        d.tri_valid = f.tri_valid;
        d.tri_map = f.tri_map;
        d.triangles = f.triangles;
        d.halfedges = f.halfedges;
        d.n_tri = f.n_tri;
        d.normals_T = f.normals_T;
        d.M = f.M; d.N = f.N; d.Mq = f.M - 1; d.Nq = f.N - 1;
        d.Rl = f.kernel_lap / 2;
        d.Rb = f.kernel_bil / 2;
        d.lam = f.lambda;
        d.ka = log2e / (2.0f * f.sigma_length * f.sigma_length);
        d.kb = log2e / (2.0f * f.sigma_angle * f.sigma_angle);
        const TileCfg cl = tile_cfg(kStageBatchLaplacian, d.Rl), cb = tile_cfg(kStageBatchBilateral, d.Rb);
        d.lap_th = cl.th; d.lap_tw = cl.tw; d.lap_tiles_x = (f.N + cl.tw - 1) / cl.tw;
        d.bil_th = cb.th; d.bil_tw = cb.tw; d.bil_tiles_x = (f.N - 1 + cb.tw - 1) / cb.tw;
        d.dom = f.groups ? f.dominant : nullptr;
        d.groups = f.groups;
        d.n_dom = f.groups ? f.n_dominant : 0;
        d.lmax2 = f.groups ? f.l_max * f.l_max : 0.0f;
        d.ang_min = f.groups ? f.ang_min : 0.0f;
        // sweep passes, the last of each stage landing in the caller's output
        const int lp = passes_for(f.iters_lap, cl.fuse);
        int left = f.iters_lap;
        const void *src = f.pts;
        for (int p = 0; p < lp; ++p) {
            const int F = left < cl.fuse ? left : cl.fuse;
            left -= F;
            void *dst = ((lp - 1 - p) % 2 == 0) ? static_cast<void *>(f.pts_out) : static_cast<void *>(d.lap_tmp);
            b.lap[p].tab[i] = PassFrame{src, dst, F, 0};
            src = dst;
        }
        const int bp = passes_for(f.iters_bil, cb.fuse);
        left = f.iters_bil;
        src = f.pts_out;                 // first pass: from the smoothed points
        for (int p = 0; p < bp; ++p) {
            const int F = left < cb.fuse ? left : cb.fuse;
            left -= F;
            void *dst = ((bp - 1 - p) % 2 == 0) ? f.normals : d.bil_tmp;
            b.bil[p].tab[i] = PassFrame{src, dst, F, p == bp - 1};
            src = dst;
        }
    }
    std::vector<uint8_t> img(table_end, 0);
    std::memcpy(img.data() + b.off_frames, bf.data(), sizeof(BFrame) * n);
    for (auto &p : b.lap) std::memcpy(img.data() + p.off, p.tab.data(), sizeof(PassFrame) * n);
    for (auto &p : b.bil) std::memcpy(img.data() + p.off, p.tab.data(), sizeof(PassFrame) * n);
    std::vector<QueueDev> qd;
    for (HostQueue *q : qs) {
        std::memcpy(img.data() + q->off_count, q->count.data(), sizeof(int) * n);
        qd.push_back(QueueDev{reinterpret_cast<const int *>(base + q->off_count),
                              reinterpret_cast<int *>(base + q->off_start)});
    }
    std::memcpy(img.data() + b.off_queues, qd.data(), sizeof(QueueDev) * qd.size());
    std::memset(img.data() + b.off_ones, 1, n);
    if (hipMemcpyAsync(b.ws, img.data(), table_end, hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return 0;
    return L.off;
}

namespace {

QueueDev dev_queue(const pl_batch_s &b, const HostQueue &q) {
    return QueueDev{reinterpret_cast<const int *>(b.ws + q.off_count),
                    reinterpret_cast<int *>(b.ws + q.off_start)};
}

// One workgroup per tile of the whole batch; kernels above 64 KiB of LDS
// are allowed their size once here.
pl_status size_grid(HostQueue &q, const void *kernel, size_t lds) {
    if (q.max_tiles > INT_MAX) {
        set_error("batch has more than 2^31 - 1 tiles in one stage");
        return PL_ERR_SHAPE;
    }
    if (pl_status st = allow_lds(kernel, lds)) return st;
    q.grid = (int)std::max<long>(1, q.max_tiles);
    q.lds = lds;
    return PL_OK;
}

template <typename NT>
pl_status plan_grids(pl_batch_s &b, const pl_frame *frames) {
    if (pl_status st = size_grid(b.mc, (const void *)k_batch_mesh_count, 0)) return st;
    if (pl_status st = size_grid(b.me, (const void *)k_batch_mesh_emit, 0)) return st;
    if (b.grp.max_tiles > 0)
        if (pl_status st = size_grid(b.grp, (const void *)k_batch_groups<NT>, 0)) return st;
    static const void *const lap_k[kMaxRadius] = {
        (const void *)k_batch_laplacian<1>, (const void *)k_batch_laplacian<2>,
        (const void *)k_batch_laplacian<3>, (const void *)k_batch_laplacian<4>};
    static const void *const bil_k[2][kMaxRadius] = {
        {(const void *)k_batch_bilateral<1, NT, false>, (const void *)k_batch_bilateral<2, NT, false>,
         (const void *)k_batch_bilateral<3, NT, false>, (const void *)k_batch_bilateral<4, NT, false>},
        {(const void *)k_batch_bilateral<1, NT, true>, (const void *)k_batch_bilateral<2, NT, true>,
         (const void *)k_batch_bilateral<3, NT, true>, (const void *)k_batch_bilateral<4, NT, true>}};
    for (Pass &p : b.lap)
        for (int r = 0; r < kMaxRadius; ++r) {
            size_t lds = 0;
            for (int i = 0; i < b.n; ++i) {
                if (!p.q[r].count[i]) continue;
                const TileCfg c = tile_cfg(kStageBatchLaplacian, r + 1);
                lds = std::max(lds, lap_lds_bytes(r + 1, p.tab[i].F, c.th, c.tw));
            }
            if (pl_status st = size_grid(p.q[r], lap_k[r], lds)) return st;
        }
    for (size_t pi = 0; pi < b.bil.size(); ++pi)
        for (int r = 0; r < kMaxRadius; ++r) {
            Pass &p = b.bil[pi];
            size_t lds = 0;
            for (int i = 0; i < b.n; ++i) {
                if (!p.q[r].count[i]) continue;
                const TileCfg c = tile_cfg(kStageBatchBilateral, r + 1);
                lds = std::max(lds, bil_lds_bytes(r + 1, p.tab[i].F, c.th, c.tw, bil_waves(r + 1, true)));
            }
            if (pl_status st = size_grid(p.q[r], bil_k[pi == 0][r], lds)) return st;
        }
    return PL_OK;
}

// Workgroups of a queue's launch when at most `bound` frames are active.
int bounded_grid(const HostQueue &q, int bound) {
    const long t = q.top[std::min<size_t>((size_t)std::max(bound, 0), q.top.size() - 1)];
    return (int)std::max<long>(1, std::min<long>(t, q.grid));
}

template <typename NT>
pl_status run_batch(const pl_batch_s &b, const uint8_t *active, hipStream_t s, int bound) {
    const BFrame *fr = reinterpret_cast<const BFrame *>(b.ws + b.off_frames);
    const QueueDev *qs = reinterpret_cast<const QueueDev *>(b.ws + b.off_queues);
    const int nq = b.n_queues;
    const uint8_t *act = active ? active : b.ws + b.off_ones;
    const int n = b.n;
    k_batch_prepare<<<nq, kTileBlock, 0, s>>>(qs, n, act);
    if (pl_status st = hip_check(hipGetLastError(), "k_batch_prepare")) return st;
    k_batch_mesh_count<<<bounded_grid(b.mc, bound), kTileBlock, 0, s>>>(fr, dev_queue(b, b.mc), n);
    if (pl_status st = hip_check(hipGetLastError(), "k_batch_mesh_count")) return st;
    k_batch_mesh_emit<<<bounded_grid(b.me, bound), kTileBlock, 0, s>>>(fr, dev_queue(b, b.me), n);
    if (pl_status st = hip_check(hipGetLastError(), "k_batch_mesh_emit")) return st;
    for (const Pass &p : b.lap) {
        const PassFrame *pt = reinterpret_cast<const PassFrame *>(b.ws + p.off);
        for (int r = 0; r < kMaxRadius; ++r) {
            const HostQueue &q = p.q[r];
            if (q.max_tiles == 0) continue;
            const dim3 g(bounded_grid(q, bound)), blk(kTileBlock);
            const QueueDev d = dev_queue(b, q);
            switch (r + 1) {
            case 1: k_batch_laplacian<1><<<g, blk, q.lds, s>>>(fr, pt, d, n); break;
            case 2: k_batch_laplacian<2><<<g, blk, q.lds, s>>>(fr, pt, d, n); break;
            case 3: k_batch_laplacian<3><<<g, blk, q.lds, s>>>(fr, pt, d, n); break;
            default: k_batch_laplacian<4><<<g, blk, q.lds, s>>>(fr, pt, d, n); break;
            }
            if (pl_status st = hip_check(hipGetLastError(), "k_batch_laplacian")) return st;
        }
    }
    for (size_t pi = 0; pi < b.bil.size(); ++pi) {
        const Pass &p = b.bil[pi];
        const PassFrame *pt = reinterpret_cast<const PassFrame *>(b.ws + p.off);
        for (int r = 0; r < kMaxRadius; ++r) {
            const HostQueue &q = p.q[r];
            if (q.max_tiles == 0) continue;
            const dim3 g(bounded_grid(q, bound)), blk(kTileBlock);
            const QueueDev d = dev_queue(b, q);
            if (pi == 0) {
                switch (r + 1) {
                case 1: k_batch_bilateral<1, NT, true><<<g, blk, q.lds, s>>>(fr, pt, d, n); break;
                case 2: k_batch_bilateral<2, NT, true><<<g, blk, q.lds, s>>>(fr, pt, d, n); break;
                case 3: k_batch_bilateral<3, NT, true><<<g, blk, q.lds, s>>>(fr, pt, d, n); break;
                default: k_batch_bilateral<4, NT, true><<<g, blk, q.lds, s>>>(fr, pt, d, n); break;
                }
            } else {
                switch (r + 1) {
                case 1: k_batch_bilateral<1, NT, false><<<g, blk, q.lds, s>>>(fr, pt, d, n); break;
                case 2: k_batch_bilateral<2, NT, false><<<g, blk, q.lds, s>>>(fr, pt, d, n); break;
                case 3: k_batch_bilateral<3, NT, false><<<g, blk, q.lds, s>>>(fr, pt, d, n); break;
                default: k_batch_bilateral<4, NT, false><<<g, blk, q.lds, s>>>(fr, pt, d, n); break;
                }
            }
            if (pl_status st = hip_check(hipGetLastError(), "k_batch_bilateral")) return st;
        }
    }
    if (b.grp.max_tiles > 0) {
        k_batch_groups<NT><<<bounded_grid(b.grp, bound), kGroupBlock, 0, s>>>(fr, dev_queue(b, b.grp), n);
        if (pl_status st = hip_check(hipGetLastError(), "k_batch_groups")) return st;
    }
    return PL_OK;
}

}  // namespace

size_t batch_workspace(const pl_frame *frames, int n, pl_dtype ndt) {
    return batch_layout(frames, n, ndt, nullptr, nullptr);
}

pl_status batch_create(const pl_frame *frames, int n, pl_dtype ndt, void *ws, hipStream_t s,
                       pl_batch_s **out) {
    pl_batch_s *b = new (std::nothrow) pl_batch_s();
    if (!b) {
        set_error("out of host memory");
        return PL_ERR_ARG;
    }
    b->ws = static_cast<uint8_t *>(ws);
    if (batch_layout(frames, n, ndt, b, s) == 0) {
        delete b;
        set_error("uploading the batch tables failed");
        return PL_ERR_HIP;
    }
    const pl_status st = ndt == PL_F32 ? plan_grids<float>(*b, frames) : plan_grids<__half>(*b, frames);
    if (st) {
        delete b;
        return st;
    }
    *out = b;
    return PL_OK;
}

int batch_size(const pl_batch_s *b) { return b->n; }

pl_status batch_run(const pl_batch_s *b, const uint8_t *active, hipStream_t s) {
    return b->ndt == PL_F32 ? run_batch<float>(*b, active, s, b->n)
                            : run_batch<__half>(*b, active, s, b->n);
}

pl_status batch_capture(pl_batch_s *b, const uint8_t *active, int bound, hipStream_t s) {
    bound = std::max(1, std::min(bound, b->n));
    auto old = b->graphs.find(bound);
    if (old != b->graphs.end()) {
        (void)hipGraphExecDestroy(old->second);
        b->graphs.erase(old);
    }
    hipGraph_t g = nullptr;
    if (pl_status st = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal),
                                 "hipStreamBeginCapture"))
        return st;
    const pl_status run_st = b->ndt == PL_F32 ? run_batch<float>(*b, active, s, bound)
                                              : run_batch<__half>(*b, active, s, bound);
    const pl_status end_st = hip_check(hipStreamEndCapture(s, &g), "hipStreamEndCapture");
    if (run_st || end_st) {
        if (g) (void)hipGraphDestroy(g);
        return run_st ? run_st : end_st;
    }
    hipGraphExec_t exec = nullptr;
    const pl_status inst = hip_check(hipGraphInstantiate(&exec, g, nullptr, nullptr, 0),
                                     "hipGraphInstantiate");
    (void)hipGraphDestroy(g);
    if (inst == PL_OK) b->graphs[bound] = exec;
    return inst;
}

pl_status batch_replay(const pl_batch_s *b, int n_active, hipStream_t s) {
    auto it = b->graphs.lower_bound(std::max(n_active, 1));
    if (it == b->graphs.end()) {
        set_error("no captured graph of this batch allows %d active frames", n_active);
        return PL_ERR_ARG;
    }
    return hip_check(hipGraphLaunch(it->second, s), "hipGraphLaunch");
}

void batch_destroy(pl_batch_s *b) {
    if (!b) return;
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    delete b;
}

}  // namespace pl
