// Organized-point-cloud mesh extraction (Sec. 4.2, Alg. 1 and Alg. 2) as an
// ordered compaction over quad rows, one frame per call:
//   k_mesh_count : one workgroup per quad row -> 2-bit validity code per quad
//                  and the row's triangle count (mesh_count_row, tiles.h).
//   k_mesh_emit  : one workgroup per quad row -> T_map, T and HE of the row,
//                  placed by the counts of the rows above (mesh_emit_row).
// Indices come from prefix sums in GID order, so T is exactly Alg. 1's
// append order and every output is bit-exact and deterministic.
#include "tiles.h"

namespace pl {

namespace {

__global__ __launch_bounds__(kTileBlock) void k_mesh_count(const float *__restrict__ pts, int N,
                                                           uint8_t *__restrict__ codes,
                                                           uint8_t *__restrict__ tri_valid,
                                                           int *__restrict__ row_count) {
    // each XCD takes a contiguous run of quad rows: the point row that two
    // neighbouring quad rows share is then fetched once into one L2
    mesh_count_row(pts, N, xcd_remap((int)blockIdx.x, (int)gridDim.x), codes, tri_valid,
                   row_count);
}

__global__ __launch_bounds__(kTileBlock) void k_mesh_emit(const uint8_t *__restrict__ codes,
                                                          const int *__restrict__ row_count,
                                                          int Mq, int N,
                                                          int32_t *__restrict__ tri_map,
                                                          int32_t *__restrict__ tris,
                                                          int32_t *__restrict__ he, int cap,
                                                          int32_t *__restrict__ n_tri) {
    // contiguous rows per XCD, as for the count (the twins read the
    // neighbouring rows' codes)
    mesh_emit_row(codes, row_count, Mq, N, xcd_remap((int)blockIdx.x, (int)gridDim.x), tri_map,
                  tris, he, cap, n_tri);
}

}  // namespace

size_t mesh_workspace(int M, int N) {
    const size_t Q = (size_t)(M - 1) * (N - 1);
    return align_up(Q, 256) + align_up(sizeof(int) * (M - 1), 256);
}

pl_status launch_mesh(const float *pts, int M, int N, uint8_t *tri_valid, int32_t *tri_map,
                      int32_t *triangles, int32_t *halfedges, int32_t cap, int32_t *n_tri,
                      void *ws, hipStream_t s) {
    const int Mq = M - 1;
    const size_t Q = (size_t)Mq * (N - 1);
    uint8_t *codes = static_cast<uint8_t *>(ws);
    int *row_count = reinterpret_cast<int *>(codes + align_up(Q, 256));
    k_mesh_count<<<Mq, kTileBlock, 0, s>>>(pts, N, codes, tri_valid, row_count);
    if (pl_status st = hip_check(hipGetLastError(), "k_mesh_count")) return st;
    k_mesh_emit<<<Mq, kTileBlock, 0, s>>>(codes, row_count, Mq, N, tri_map, triangles, halfedges,
                                          cap, n_tri);
    return hip_check(hipGetLastError(), "k_mesh_emit");
}

}  // namespace pl
