// Organized-point-cloud mesh extraction (Sec. 4.2, Alg. 1 and Alg. 2) as an
// ordered compaction over segments of quad rows (256 quads, one per thread),
// one frame per call:
//   k_mesh_count : one workgroup per segment -> 2-bit validity code per quad
//                  and the segment's triangle count (mesh_count_seg, tiles.h).
//   k_mesh_emit  : one workgroup per segment -> T_map, T and HE of the
//                  segment, placed by the counts of the segments before it
//                  in row-major order (mesh_emit_seg).
// Every emit workgroup sums the counts before its segment, so that work grows
// with the square of the segment count: frames of more than kMeshSegMax
// segments take whole quad rows per workgroup instead (k_mesh_*_rows over
// mesh_count_row / mesh_emit_row, the batched path's bodies), with the same
// outputs.
// Indices come from prefix sums in GID order, so T is exactly Alg. 1's
// append order and every output is bit-exact and deterministic.
#include "tiles.h"

#include <mutex>

namespace pl {

namespace {

__global__ __launch_bounds__(kTileBlock) void k_mesh_count(const float *__restrict__ pts, int N,
                                                           int S, uint8_t *__restrict__ codes,
                                                           uint8_t *__restrict__ tri_valid,
                                                           int *__restrict__ seg_count) {
    // each XCD takes a contiguous run of segments (whole rows but for its
    // ends): the point row that two neighbouring quad rows share is then
    // fetched once into one L2
    __shared__ MeshCountSegLds L;
    const int k = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    mesh_count_seg(pts, N, k / S, k % S, S, codes, tri_valid, seg_count, L);
}

__global__ __launch_bounds__(kTileBlock) void k_mesh_emit(const uint8_t *__restrict__ codes,
                                                          const int *__restrict__ seg_count,
                                                          int Mq, int N, int S,
                                                          int32_t *__restrict__ tri_map,
                                                          int32_t *__restrict__ tris,
                                                          int32_t *__restrict__ he, int cap,
                                                          int32_t *__restrict__ n_tri) {
    // contiguous segments per XCD, as for the count (the twins read the
    // neighbouring rows' codes)
    __shared__ MeshEmitSegLds L;
    const int k = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    mesh_emit_seg(codes, seg_count, Mq, N, k / S, k % S, S, tri_map, tris, he, cap, n_tri, L);
}

__global__ __launch_bounds__(kTileBlock) void k_mesh_count_rows(const float *__restrict__ pts,
                                                                int N,
                                                                uint8_t *__restrict__ codes,
                                                                uint8_t *__restrict__ tri_valid,
                                                                int *__restrict__ row_count) {
    __shared__ MeshCountRowLds L;
    mesh_count_row(pts, N, xcd_remap((int)blockIdx.x, (int)gridDim.x), codes, tri_valid,
                   row_count, L);
}

__global__ __launch_bounds__(kTileBlock) void k_mesh_emit_rows(const uint8_t *__restrict__ codes,
                                                               const int *__restrict__ row_count,
                                                               int Mq, int N,
                                                               int32_t *__restrict__ tri_map,
                                                               int32_t *__restrict__ tris,
                                                               int32_t *__restrict__ he, int cap,
                                                               int32_t *__restrict__ n_tri) {
    __shared__ MeshEmitRowLds L;
    mesh_emit_row(codes, row_count, Mq, N, xcd_remap((int)blockIdx.x, (int)gridDim.x), tri_map,
                  tris, he, cap, n_tri, L);
}

// Scratch of the allocation-free entry point (pl_mesh_opc_static): the
// validity codes and per-segment counts that pl_mesh_opc keeps in the
// caller's workspace.  Every device the library runs on holds one copy until
// the process ends.  Host code never passes this name to a kernel (in host
// code it is a host-side stand-in, not a device address): it uses the
// address hipGetSymbolAddress returns for the device in question.
constexpr size_t kMeshScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) uint8_t scratch[kMeshScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices];    // device address of `scratch` per device, once looked up

}  // namespace

size_t mesh_static_scratch_bytes() { return kMeshScratchBytes; }

pl_status mesh_static_scratch(hipStream_t s, void **out) {
    int cur = 0;
    if (pl_status st = hip_check(hipGetDevice(&cur), "hipGetDevice")) return st;
    int dev = cur;
    if (s) {
        hipDevice_t d;
        if (pl_status st = hip_check(hipStreamGetDevice(s, &d), "hipStreamGetDevice")) return st;
        dev = (int)d;
    }
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d: the static mesh scratch serves devices 0..%d", dev, kMaxDevices - 1);
        return PL_ERR_ARG;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        // look the array up with its device current: each device holds its
        // own copy at its own address
        if (dev != cur)
            if (pl_status st = hip_check(hipSetDevice(dev), "hipSetDevice")) return st;
        void *p = nullptr;
        const pl_status st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                                       "hipGetSymbolAddress(scratch)");
        if (dev != cur) (void)hipSetDevice(cur);
        if (st) return st;
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return PL_OK;
}

size_t mesh_workspace(int M, int N) {
    const size_t Q = (size_t)(M - 1) * (N - 1);
    return align_up(Q, 256) + align_up(sizeof(int) * (size_t)(M - 1) * mesh_segments(N - 1), 256);
}

pl_status launch_mesh(const float *pts, int M, int N, uint8_t *tri_valid, int32_t *tri_map,
                      int32_t *triangles, int32_t *halfedges, int32_t cap, int32_t *n_tri,
                      void *ws, hipStream_t s) {
    const int Mq = M - 1;
    const size_t Q = (size_t)Mq * (N - 1);
    uint8_t *codes = static_cast<uint8_t *>(ws);
    int *counts = reinterpret_cast<int *>(codes + align_up(Q, 256));
    const int S = mesh_segments(N - 1);
    if ((long)Mq * S > kMeshSegMax) {
        k_mesh_count_rows<<<Mq, kTileBlock, 0, s>>>(pts, N, codes, tri_valid, counts);
        if (pl_status st = hip_check(hipGetLastError(), "k_mesh_count_rows")) return st;
        k_mesh_emit_rows<<<Mq, kTileBlock, 0, s>>>(codes, counts, Mq, N, tri_map, triangles,
                                                   halfedges, cap, n_tri);
        return hip_check(hipGetLastError(), "k_mesh_emit_rows");
    }
    const int blocks = Mq * S;
    k_mesh_count<<<blocks, kTileBlock, 0, s>>>(pts, N, S, codes, tri_valid, counts);
    if (pl_status st = hip_check(hipGetLastError(), "k_mesh_count")) return st;
    k_mesh_emit<<<blocks, kTileBlock, 0, s>>>(codes, counts, Mq, N, S, tri_map, triangles,
                                              halfedges, cap, n_tri);
    return hip_check(hipGetLastError(), "k_mesh_emit");
}

}  // namespace pl
