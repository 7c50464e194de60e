// Triangle centroids and normals over the implicit full mesh T_FC (Sec. 5.2),
// one thread per quad, 256 consecutive quads per workgroup (normals_block in
// tiles.h).  Pure streaming work: 12 B/point in, 2 x 12 B/triangle out
// (float32 normals).
#include "tiles.h"

namespace pl {

namespace {

template <typename NT>
__global__ __launch_bounds__(kTileBlock) void k_tri_normals(const float *__restrict__ pts, int N,
                                                            int Nq, size_t Q,
                                                            NT *__restrict__ normals,
                                                            float *__restrict__ centroids) {
    __shared__ NormalsStage st;
    // contiguous quad runs per XCD: the point row shared by two quad rows is
    // fetched once into one L2
    const size_t q0 = (size_t)xcd_remap((int)blockIdx.x, (int)gridDim.x) * kTileBlock;
    const int nq = (int)(Q - q0 < (size_t)kTileBlock ? Q - q0 : (size_t)kTileBlock);
    normals_block<NT>(pts, N, Nq, q0, nq, normals, centroids, st);
}

}  // namespace

pl_status launch_tri_normals(const float *pts, int M, int N, void *normals, pl_dtype ndt,
                             float *centroids, hipStream_t s) {
    const int Nq = N - 1;
    const size_t Q = (size_t)(M - 1) * Nq;
    const int blocks = (int)((Q + kTileBlock - 1) / kTileBlock);
    if (ndt == PL_F32)
        k_tri_normals<float><<<blocks, kTileBlock, 0, s>>>(pts, N, Nq, Q,
                                                           static_cast<float *>(normals), centroids);
    else
        k_tri_normals<__half><<<blocks, kTileBlock, 0, s>>>(pts, N, Nq, Q,
                                                            static_cast<__half *>(normals), centroids);
    return hip_check(hipGetLastError(), "k_tri_normals");
}

}  // namespace pl
