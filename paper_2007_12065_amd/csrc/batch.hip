// Batched path: many frames of different sizes and filter settings through
// the whole pipeline with one persistent launch per stage.
//
// Plan (pl_batch_create, host): validates every frame, lays out a workspace
// holding one descriptor per frame, the per-pass source/destination tables
// of the multi-sweep stages, a tile list per stage and per-frame scratch
// (validity codes, row counts, ping-pong buffers), uploads the tables once
// and picks a resident grid per kernel from the occupancy API.
//
// Run (pl_batch_run, device only, graph-capturable):
//   k_batch_reset      zero the queue counters
//   k_batch_mesh_count tiles = (frame, quad row)        -> codes, row counts
//   k_batch_mesh_emit  tiles = (frame, quad row)        -> T_map, T, HE, |T|
//   k_batch_laplacian  one launch per sweep pass, tiles = (frame, point tile)
//   k_batch_normals    tiles = (frame, 1024 quads)      -> raw normals, centroids
//   k_batch_bilateral  one launch per sweep pass, tiles = (frame, quad tile);
//                      the frame's last pass gathers onto T
// Every tile runs the same device body as the single-frame kernels
// (tiles.h), so each frame's outputs equal its single-frame results.
//
// Work queue.  A stage's tiles are listed frame by frame and cut into eight
// contiguous segments of about equal cost, one per XCD: workgroup b starts
// on segment b mod 8 (the XCD it was dispatched to), so neighbouring tiles,
// which share halo lines, meet in the same L2.  A workgroup pops tiles with
// an atomic counter and, once its segment is empty, steals from the others
// in turn; each counter is bumped at most grid-size times past its end, so
// every workgroup leaves the loop after at most eight empty pops.
#include "tiles.h"
#include "tuning.h"

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

namespace pl {

namespace {

constexpr int kQueues = kNumXcd;

struct BFrame {
    const float *pts;
    float *pts_out, *lap_tmp;
    void *nraw, *normals, *bil_tmp;
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
};

struct PassFrame {                 // one frame's part of one sweep pass
    const void *src;
    void *dst;
    int F;                         // sweeps in this pass (0: copy)
    int active;
    int gather;                    // bilateral: last pass, gather onto T
};

struct Queue {                     // device view of one stage's tile queue
    const int2 *tiles;             // (frame, tile index in frame)
    const int *seg;                // [kQueues + 1] segment starts
    int *counter;                  // [kQueues]
};

// Pop the next tile for this workgroup, or return false when every segment
// is exhausted.  `q` is the segment being drained (starts at blockIdx mod 8).
__device__ __forceinline__ bool pop_tile(const Queue &Q, int &q, int &tries, int2 &tile) {
    __shared__ int s_idx;
    while (tries < kQueues) {
        if (threadIdx.x == 0) s_idx = atomicAdd(&Q.counter[q], 1);
        __syncthreads();
        const int i = s_idx;
        __syncthreads();
        const int n = Q.seg[q + 1] - Q.seg[q];
        if (i < n) {
            tile = Q.tiles[Q.seg[q] + i];
            return true;
        }
        q = (q + 1) % kQueues;
        ++tries;
    }
    return false;
}

__global__ void k_batch_reset(int *counters, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i] = 0;
}

__global__ __launch_bounds__(kTileBlock) void k_batch_mesh_count(const BFrame *__restrict__ fr,
                                                                 Queue Q) {
    int q = blockIdx.x % kQueues, tries = 0;
    int2 t;
    while (pop_tile(Q, q, tries, t)) {
        const BFrame &f = fr[t.x];
        mesh_count_row(f.pts, f.N, t.y, f.codes, f.tri_valid, f.row_count);
    }
}

__global__ __launch_bounds__(kTileBlock) void k_batch_mesh_emit(const BFrame *__restrict__ fr,
                                                                Queue Q) {
    int q = blockIdx.x % kQueues, tries = 0;
    int2 t;
    while (pop_tile(Q, q, tries, t)) {
        const BFrame &f = fr[t.x];
        mesh_emit_row(f.codes, f.row_count, f.Mq, f.N, t.y, f.tri_map, f.triangles, f.halfedges,
                      2 * f.Mq * f.Nq, f.n_tri);
    }
}

__global__ __launch_bounds__(kTileBlock) void k_batch_laplacian(const BFrame *__restrict__ fr,
                                                                const PassFrame *__restrict__ pass,
                                                                Queue Q) {
    extern __shared__ float4 lds[];
    int q = blockIdx.x % kQueues, tries = 0;
    int2 t;
    while (pop_tile(Q, q, tries, t)) {
        const BFrame &f = fr[t.x];
        const PassFrame &p = pass[t.x];
        const float *src = static_cast<const float *>(p.src);
        float *dst = static_cast<float *>(p.dst);
        const int ty0 = (t.y / f.lap_tiles_x) * f.lap_th, tx0 = (t.y % f.lap_tiles_x) * f.lap_tw;
        switch (f.Rl) {
        case 1: lap_tile<1>(src, dst, f.M, f.N, f.lam, p.F, f.lap_th, f.lap_tw, ty0, tx0, lds); break;
        case 2: lap_tile<2>(src, dst, f.M, f.N, f.lam, p.F, f.lap_th, f.lap_tw, ty0, tx0, lds); break;
        case 3: lap_tile<3>(src, dst, f.M, f.N, f.lam, p.F, f.lap_th, f.lap_tw, ty0, tx0, lds); break;
        default: lap_tile<4>(src, dst, f.M, f.N, f.lam, p.F, f.lap_th, f.lap_tw, ty0, tx0, lds); break;
        }
    }
}

constexpr int kNormalsChunk = 4 * kTileBlock;   // quads per normals tile

template <typename NT>
__global__ __launch_bounds__(kTileBlock) void k_batch_normals(const BFrame *__restrict__ fr,
                                                              Queue Q) {
    int q = blockIdx.x % kQueues, tries = 0;
    int2 t;
    while (pop_tile(Q, q, tries, t)) {
        const BFrame &f = fr[t.x];
        const size_t Qn = (size_t)f.Mq * f.Nq;
        const size_t q0 = (size_t)t.y * kNormalsChunk;
        for (size_t qq = q0 + threadIdx.x; qq < Qn && qq < q0 + kNormalsChunk; qq += kTileBlock)
            normals_quad<NT>(f.pts_out, f.N, f.Nq, qq, static_cast<NT *>(f.nraw), f.centroids);
    }
}

template <typename NT>
__global__ __launch_bounds__(kTileBlock) void k_batch_bilateral(const BFrame *__restrict__ fr,
                                                                const PassFrame *__restrict__ pass,
                                                                Queue Q) {
    extern __shared__ float4 lds[];
    int q = blockIdx.x % kQueues, tries = 0;
    int2 t;
    while (pop_tile(Q, q, tries, t)) {
        const BFrame &f = fr[t.x];
        const PassFrame &p = pass[t.x];
        const NT *src = static_cast<const NT *>(p.src);
        NT *dst = static_cast<NT *>(p.dst);
        const int32_t *tm = p.gather ? f.tri_map : nullptr;
        NT *nT = static_cast<NT *>(f.normals_T);
        const int qy0 = (t.y / f.bil_tiles_x) * f.bil_th, qx0 = (t.y % f.bil_tiles_x) * f.bil_tw;
        switch (f.Rb) {
        case 1: bil_tile<1, NT>(src, f.centroids, dst, f.Mq, f.Nq, f.ka, f.kb, p.F, f.bil_th, f.bil_tw, qy0, qx0, tm, nT, lds); break;
        case 2: bil_tile<2, NT>(src, f.centroids, dst, f.Mq, f.Nq, f.ka, f.kb, p.F, f.bil_th, f.bil_tw, qy0, qx0, tm, nT, lds); break;
        case 3: bil_tile<3, NT>(src, f.centroids, dst, f.Mq, f.Nq, f.ka, f.kb, p.F, f.bil_th, f.bil_tw, qy0, qx0, tm, nT, lds); break;
        default: bil_tile<4, NT>(src, f.centroids, dst, f.Mq, f.Nq, f.ka, f.kb, p.F, f.bil_th, f.bil_tw, qy0, qx0, tm, nT, lds); break;
        }
    }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

struct Layout {                    // byte offsets inside the workspace
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += align_up(bytes, 256);
        return o;
    }
};

struct HostQueue {                 // a stage's tiles before upload
    std::vector<int2> tiles;
    std::vector<double> cost;
    size_t off_tiles = 0, off_seg = 0;
    int counter0 = 0;              // index of its first counter
    int grid = 0;
    size_t lds = 0;
};

struct Pass {
    std::vector<PassFrame> tab;    // [n]
    size_t off = 0;
    HostQueue q;
};

}  // namespace

}  // namespace pl

struct pl_batch_s {
    int n = 0;
    pl_dtype ndt = PL_F32;
    uint8_t *ws = nullptr;
    size_t off_frames = 0, off_counters = 0;
    int ncounters = 0;
    pl::HostQueue mc, me, nq;      // mesh count, mesh emit, normals
    std::vector<pl::Pass> lap, bil;
    hipGraphExec_t graph = nullptr;
};

namespace pl {

namespace {

size_t nt_size(pl_dtype ndt) { return ndt == PL_F32 ? 4 : 2; }

int passes_for(int iters, int fuse) { return iters == 0 ? 1 : (iters + fuse - 1) / fuse; }

// Split a stage's tile list into kQueues contiguous segments of about equal
// total cost (segment starts, kQueues + 1 entries).
std::vector<int> segments(const std::vector<double> &cost) {
    double total = 0;
    for (double c : cost) total += c;
    std::vector<int> seg(kQueues + 1, (int)cost.size());
    seg[0] = 0;
    double acc = 0;
    int s = 1;
    for (size_t i = 0; i < cost.size() && s < kQueues; ++i) {
        acc += cost[i];
        while (s < kQueues && acc >= total * s / kQueues) seg[s++] = (int)i + 1;
    }
    for (int k = 1; k <= kQueues; ++k) seg[k] = std::max(seg[k], seg[k - 1]);
    return seg;
}

struct Range {
    uintptr_t a, b;
    int frame;
    bool out;
};

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
        maxlap = std::max(maxlap, passes_for(f.iters_lap, tile_cfg(kStageLaplacian, f.kernel_lap / 2).fuse));
        maxbil = std::max(maxbil, passes_for(f.iters_bil, tile_cfg(kStageBilateral, f.kernel_bil / 2).fuse));
    }
    b.lap.assign(maxlap, Pass());
    b.bil.assign(maxbil, Pass());
    for (auto &p : b.lap) { p.tab.assign(n, PassFrame{}); p.off = L.take(sizeof(PassFrame) * n); }
    for (auto &p : b.bil) { p.tab.assign(n, PassFrame{}); p.off = L.take(sizeof(PassFrame) * n); }
    // tile lists
    b.mc.tiles.clear(); b.me.tiles.clear(); b.nq.tiles.clear();
    b.mc.cost.clear(); b.me.cost.clear(); b.nq.cost.clear();
    for (int i = 0; i < n; ++i) {
        const pl_frame &f = frames[i];
        const int Mq = f.M - 1, Nq = f.N - 1;
        for (int u = 0; u < Mq; ++u) {
            b.mc.tiles.push_back(make_int2(i, u)); b.mc.cost.push_back(Nq);
            b.me.tiles.push_back(make_int2(i, u)); b.me.cost.push_back(Nq);
        }
        const size_t Q = (size_t)Mq * Nq;
        for (size_t c = 0; c * kNormalsChunk < Q; ++c) {
            b.nq.tiles.push_back(make_int2(i, (int)c)); b.nq.cost.push_back(1.0);
        }
    }
    for (size_t p = 0; p < b.lap.size(); ++p) {
        HostQueue &q = b.lap[p].q;
        for (int i = 0; i < n; ++i) {
            const pl_frame &f = frames[i];
            const TileCfg c = tile_cfg(kStageLaplacian, f.kernel_lap / 2);
            if ((int)p >= passes_for(f.iters_lap, c.fuse)) continue;
            const int tx = (f.N + c.tw - 1) / c.tw, ty = (f.M + c.th - 1) / c.th;
            const double cost = (double)(c.th + 2 * c.fuse * (f.kernel_lap / 2)) * (c.tw + 2 * c.fuse * (f.kernel_lap / 2)) *
                                std::max(1, c.fuse) * f.kernel_lap * f.kernel_lap;
            for (int t = 0; t < tx * ty; ++t) { q.tiles.push_back(make_int2(i, t)); q.cost.push_back(cost); }
        }
    }
    for (size_t p = 0; p < b.bil.size(); ++p) {
        HostQueue &q = b.bil[p].q;
        for (int i = 0; i < n; ++i) {
            const pl_frame &f = frames[i];
            const TileCfg c = tile_cfg(kStageBilateral, f.kernel_bil / 2);
            if ((int)p >= passes_for(f.iters_bil, c.fuse)) continue;
            const int tx = (f.N - 1 + c.tw - 1) / c.tw, ty = (f.M - 1 + c.th - 1) / c.th;
            const double cost = (double)c.th * c.tw * std::max(1, c.fuse) * f.kernel_bil * f.kernel_bil;
            for (int t = 0; t < tx * ty; ++t) { q.tiles.push_back(make_int2(i, t)); q.cost.push_back(cost); }
        }
    }
    std::vector<HostQueue *> qs = {&b.mc, &b.me, &b.nq};
    for (auto &p : b.lap) qs.push_back(&p.q);
    for (auto &p : b.bil) qs.push_back(&p.q);
    int counters = 0;
    for (HostQueue *q : qs) {
        q->off_tiles = L.take(sizeof(int2) * std::max<size_t>(q->tiles.size(), 1));
        q->off_seg = L.take(sizeof(int) * (kQueues + 1));
        q->counter0 = counters;
        counters += kQueues;
    }
    b.ncounters = counters;
    b.off_counters = L.take(sizeof(int) * counters);
    // per-frame scratch
    std::vector<BFrame> bf(n);
    size_t scratch_off = L.off;
    (void)scratch_off;
    for (int i = 0; i < n; ++i) {
        const pl_frame &f = frames[i];
        const size_t Q = (size_t)(f.M - 1) * (f.N - 1);
        const size_t T = 2 * Q;
        bf[i].codes = reinterpret_cast<uint8_t *>(L.take(Q));
        bf[i].row_count = reinterpret_cast<int *>(L.take(sizeof(int) * (f.M - 1)));
        const int lp = passes_for(f.iters_lap, tile_cfg(kStageLaplacian, f.kernel_lap / 2).fuse);
        const int bp = passes_for(f.iters_bil, tile_cfg(kStageBilateral, f.kernel_bil / 2).fuse);
        bf[i].lap_tmp = lp > 1 ? reinterpret_cast<float *>(L.take(12 * (size_t)f.M * f.N)) : nullptr;
        bf[i].nraw = reinterpret_cast<void *>(L.take(3 * T * nt_size(ndt)));
        bf[i].bil_tmp = bp > 1 ? reinterpret_cast<void *>(L.take(3 * T * nt_size(ndt))) : nullptr;
    }
    if (plan) {
        // turn offsets into device addresses and fill the descriptors
        uintptr_t base = reinterpret_cast<uintptr_t>(b.ws);
        auto at = [&](void *off) { return off ? reinterpret_cast<void *>(base + reinterpret_cast<uintptr_t>(off)) : nullptr; };
        const float log2e = 1.4426950408889634f;
        for (int i = 0; i < n; ++i) {
            const pl_frame &f = frames[i];
            BFrame &d = bf[i];
            d.codes = static_cast<uint8_t *>(at(d.codes));
            d.row_count = static_cast<int *>(at(d.row_count));
            d.lap_tmp = static_cast<float *>(at(d.lap_tmp));
            d.nraw = at(d.nraw);
            d.bil_tmp = at(d.bil_tmp);
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
            const TileCfg cl = tile_cfg(kStageLaplacian, d.Rl), cb = tile_cfg(kStageBilateral, d.Rb);
            d.lap_th = cl.th; d.lap_tw = cl.tw; d.lap_tiles_x = (f.N + cl.tw - 1) / cl.tw;
            d.bil_th = cb.th; d.bil_tw = cb.tw; d.bil_tiles_x = (f.N - 1 + cb.tw - 1) / cb.tw;
            // sweep passes: the last one lands in the caller's output
            const int lp = passes_for(f.iters_lap, cl.fuse);
            int left = f.iters_lap;
            const void *src = f.pts;
            for (int p = 0; p < lp; ++p) {
                const int F = left < cl.fuse ? left : cl.fuse;
                left -= F;
                void *dst = ((lp - 1 - p) % 2 == 0) ? static_cast<void *>(f.pts_out) : static_cast<void *>(d.lap_tmp);
                b.lap[p].tab[i] = PassFrame{src, dst, F, 1, 0};
                src = dst;
            }
            const int bp = passes_for(f.iters_bil, cb.fuse);
            left = f.iters_bil;
            src = d.nraw;
            for (int p = 0; p < bp; ++p) {
                const int F = left < cb.fuse ? left : cb.fuse;
                left -= F;
                void *dst = ((bp - 1 - p) % 2 == 0) ? f.normals : d.bil_tmp;
                b.bil[p].tab[i] = PassFrame{src, dst, F, 1, p == bp - 1};
                src = dst;
            }
        }
        // host image of the tables
        std::vector<uint8_t> img(L.off, 0);
        std::memcpy(img.data() + b.off_frames, bf.data(), sizeof(BFrame) * n);
        for (auto &p : b.lap) std::memcpy(img.data() + p.off, p.tab.data(), sizeof(PassFrame) * n);
        for (auto &p : b.bil) std::memcpy(img.data() + p.off, p.tab.data(), sizeof(PassFrame) * n);
        for (HostQueue *q : qs) {
            if (!q->tiles.empty())
                std::memcpy(img.data() + q->off_tiles, q->tiles.data(), sizeof(int2) * q->tiles.size());
            const std::vector<int> seg = segments(q->cost);
            std::memcpy(img.data() + q->off_seg, seg.data(), sizeof(int) * seg.size());
        }
        // only the table part is uploaded; per-frame scratch needs no init
        const size_t table_bytes = b.off_counters + align_up(sizeof(int) * counters, 256);
        if (hipMemcpyAsync(b.ws, img.data(), table_bytes, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            return 0;
    }
    return L.off;
}

namespace {

Queue dev_queue(const pl_batch_s &b, const HostQueue &q) {
    Queue d;
    d.tiles = reinterpret_cast<const int2 *>(b.ws + q.off_tiles);
    d.seg = reinterpret_cast<const int *>(b.ws + q.off_seg);
    d.counter = reinterpret_cast<int *>(b.ws + b.off_counters) + q.counter0;
    return d;
}

// Resident grid: occupancy x CUs, never more workgroups than tiles.
pl_status size_grid(HostQueue &q, const void *kernel, size_t lds) {
    int dev = 0, cus = 0, per_cu = 0;
    if (pl_status st = hip_check(hipGetDevice(&dev), "hipGetDevice")) return st;
    if (pl_status st = hip_check(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev),
                                 "hipDeviceGetAttribute"))
        return st;
    if (pl_status st = allow_lds(kernel, lds)) return st;
    if (pl_status st = hip_check(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel,
                                                                              kTileBlock, lds),
                                 "hipOccupancyMaxActiveBlocksPerMultiprocessor"))
        return st;
    const long want = (long)std::max(per_cu, 1) * std::max(cus, 1);
    q.grid = (int)std::max<long>(1, std::min<long>(want, (long)q.tiles.size()));
    q.lds = lds;
    return PL_OK;
}

template <typename NT>
pl_status plan_grids(pl_batch_s &b, const pl_frame *frames) {
    if (pl_status st = size_grid(b.mc, (const void *)k_batch_mesh_count, 0)) return st;
    if (pl_status st = size_grid(b.me, (const void *)k_batch_mesh_emit, 0)) return st;
    if (pl_status st = size_grid(b.nq, (const void *)k_batch_normals<NT>, 0)) return st;
    for (size_t p = 0; p < b.lap.size(); ++p) {
        size_t lds = 0;
        for (int i = 0; i < b.n; ++i) {
            const PassFrame &pf = b.lap[p].tab[i];
            if (!pf.active) continue;
            const int R = frames[i].kernel_lap / 2;
            const TileCfg c = tile_cfg(kStageLaplacian, R);
            lds = std::max(lds, lap_lds_bytes(R, pf.F, c.th, c.tw));
        }
        if (pl_status st = size_grid(b.lap[p].q, (const void *)k_batch_laplacian, lds)) return st;
    }
    for (size_t p = 0; p < b.bil.size(); ++p) {
        size_t lds = 0;
        for (int i = 0; i < b.n; ++i) {
            const PassFrame &pf = b.bil[p].tab[i];
            if (!pf.active) continue;
            const int R = frames[i].kernel_bil / 2;
            const TileCfg c = tile_cfg(kStageBilateral, R);
            lds = std::max(lds, bil_lds_bytes(R, pf.F, c.th, c.tw));
        }
        if (pl_status st = size_grid(b.bil[p].q, (const void *)k_batch_bilateral<NT>, lds)) return st;
    }
    return PL_OK;
}

template <typename NT>
pl_status run_batch(const pl_batch_s &b, hipStream_t s) {
    const BFrame *fr = reinterpret_cast<const BFrame *>(b.ws + b.off_frames);
    int *counters = reinterpret_cast<int *>(b.ws + b.off_counters);
    k_batch_reset<<<1, 256, 0, s>>>(counters, b.ncounters);
    if (pl_status st = hip_check(hipGetLastError(), "k_batch_reset")) return st;
    if (!b.mc.tiles.empty()) {
        k_batch_mesh_count<<<b.mc.grid, kTileBlock, 0, s>>>(fr, dev_queue(b, b.mc));
        if (pl_status st = hip_check(hipGetLastError(), "k_batch_mesh_count")) return st;
        k_batch_mesh_emit<<<b.me.grid, kTileBlock, 0, s>>>(fr, dev_queue(b, b.me));
        if (pl_status st = hip_check(hipGetLastError(), "k_batch_mesh_emit")) return st;
    }
    for (const Pass &p : b.lap) {
        if (p.q.tiles.empty()) continue;
        const PassFrame *pt = reinterpret_cast<const PassFrame *>(b.ws + p.off);
        k_batch_laplacian<<<p.q.grid, kTileBlock, p.q.lds, s>>>(fr, pt, dev_queue(b, p.q));
        if (pl_status st = hip_check(hipGetLastError(), "k_batch_laplacian")) return st;
    }
    if (!b.nq.tiles.empty()) {
        k_batch_normals<NT><<<b.nq.grid, kTileBlock, 0, s>>>(fr, dev_queue(b, b.nq));
        if (pl_status st = hip_check(hipGetLastError(), "k_batch_normals")) return st;
    }
    for (const Pass &p : b.bil) {
        if (p.q.tiles.empty()) continue;
        const PassFrame *pt = reinterpret_cast<const PassFrame *>(b.ws + p.off);
        k_batch_bilateral<NT><<<p.q.grid, kTileBlock, p.q.lds, s>>>(fr, pt, dev_queue(b, p.q));
        if (pl_status st = hip_check(hipGetLastError(), "k_batch_bilateral")) return st;
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

pl_status batch_run(const pl_batch_s *b, hipStream_t s) {
    return b->ndt == PL_F32 ? run_batch<float>(*b, s) : run_batch<__half>(*b, s);
}

pl_status batch_capture(pl_batch_s *b, hipStream_t s) {
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    if (pl_status st = hip_check(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal),
                                 "hipStreamBeginCapture"))
        return st;
    const pl_status run_st = batch_run(b, s);
    const pl_status end_st = hip_check(hipStreamEndCapture(s, &g), "hipStreamEndCapture");
    if (run_st || end_st) {
        if (g) (void)hipGraphDestroy(g);
        return run_st ? run_st : end_st;
    }
    const pl_status inst = hip_check(hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0),
                                     "hipGraphInstantiate");
    (void)hipGraphDestroy(g);
    return inst;
}

pl_status batch_replay(const pl_batch_s *b, hipStream_t s) {
    if (!b->graph) {
        set_error("the batch has no captured graph (call pl_batch_capture first)");
        return PL_ERR_ARG;
    }
    return hip_check(hipGraphLaunch(b->graph, s), "hipGraphLaunch");
}

void batch_destroy(pl_batch_s *b) {
    if (!b) return;
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    delete b;
}

}  // namespace pl
