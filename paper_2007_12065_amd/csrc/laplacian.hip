// Laplacian vertex filter on the organized cloud (Sec. 2.3 Eqs. 1-2; image
// neighbourhood of Sec. 5.1), one frame per call.  The tile body (temporal
// blocking in LDS, missing-data encoding) is lap_tile in tiles.h; this file
// launches it over the frame's tiles, ceil(iterations / fuse) times, with
// ping-pong buffers so the last launch lands in the output.
#include "tiles.h"
#include "tuning.h"

namespace pl {

namespace {

template <int R>
__global__ __launch_bounds__(kTileBlock) void k_laplacian(const float *__restrict__ src,
                                                          float *__restrict__ dst, int M, int N,
                                                          float lam, int F, int TH, int TW,
                                                          int tiles_x, int ntiles) {
    extern __shared__ float4 lds[];
    const int tile = xcd_remap(blockIdx.x, ntiles);
    lap_tile<R>(src, dst, M, N, lam, F, TH, TW, (tile / tiles_x) * TH, (tile % tiles_x) * TW, lds);
}

template <int R>
pl_status run(const float *in, float *out, int M, int N, float lam, int iterations, float *tmp,
              hipStream_t s) {
    const TileCfg c = tile_cfg(frame_stage(true, M, N), R);
    const int tiles_x = (N + c.tw - 1) / c.tw;
    const int ntiles = tiles_x * ((M + c.th - 1) / c.th);
    // zero sweeps: one copying launch (F = 0)
    const int launches = iterations == 0 ? 1 : (iterations + c.fuse - 1) / c.fuse;
    const float *cur = in;
    int left = iterations;
    for (int l = 0; l < launches; ++l) {
        const int F = left < c.fuse ? left : c.fuse;
        left -= F;
        float *dst = ((launches - 1 - l) % 2 == 0) ? out : tmp;   // last launch lands in out
        const size_t lds = lap_lds_bytes(R, F, c.th, c.tw);
        if (pl_status st = allow_lds((const void *)k_laplacian<R>, lds)) return st;
        k_laplacian<R><<<ntiles, kTileBlock, lds, s>>>(cur, dst, M, N, lam, F, c.th, c.tw,
                                                       tiles_x, ntiles);
        if (pl_status st = hip_check(hipGetLastError(), "k_laplacian")) return st;
        cur = dst;
    }
    return PL_OK;
}

}  // namespace

int laplacian_fused_sweeps(int kernel) { return tile_cfg(kStageLaplacian, kernel / 2).fuse; }

size_t laplacian_workspace(int M, int N, int iterations) {
    // a second point buffer is needed once a call takes two launches; the
    // size must not depend on the tuning state, so ask for it whenever
    // there is more than one sweep
    return iterations > 1 ? sizeof(float) * 3 * (size_t)M * N : 0;
}

pl_status launch_laplacian(const float *in, float *out, int M, int N, int kernel, float lambda,
                           int iterations, void *ws, hipStream_t s) {
    float *tmp = static_cast<float *>(ws);
    switch (kernel / 2) {
    case 1: return run<1>(in, out, M, N, lambda, iterations, tmp, s);
    case 2: return run<2>(in, out, M, N, lambda, iterations, tmp, s);
    case 3: return run<3>(in, out, M, N, lambda, iterations, tmp, s);
    default: return run<4>(in, out, M, N, lambda, iterations, tmp, s);
    }
}

}  // namespace pl
