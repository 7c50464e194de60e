// Bilateral triangle-normal filter on the organized mesh (Sec. 2.3 Eqs. 3-6;
// neighbourhood of Sec. 5.2) and the gather of the result onto T, one frame
// per call.  The tile body (LDS staging, fused sweeps, weight evaluation,
// underflow fallback, missing-data encoding) is bil_tile in tiles.h; this
// file launches it over the frame's tiles ceil(iterations / fuse) times with
// ping-pong buffers; the last launch gathers onto T.
#include "tiles.h"
#include "tuning.h"

namespace pl {

namespace {

template <int R, typename NT>
__global__ __launch_bounds__(kTileBlock, kBilWavesPerSimd) void k_bilateral(
    const NT *__restrict__ nin, const float *__restrict__ cen, NT *__restrict__ nout, int Mq,
    int Nq, float ka, float kb, int F, int TQH, int TQW, int tiles_x, int ntiles,
    const int32_t *__restrict__ tri_map, NT *__restrict__ nT) {
    extern __shared__ float4 lds[];
    const int tile = xcd_remap(blockIdx.x, ntiles);
    bil_tile<R, NT, false, false, bil_frame_lanes<R>()>(nin, cen, nout, Mq, Nq, ka, kb, F, TQH, TQW,
                                                        (tile / tiles_x) * TQH,
                                                        (tile % tiles_x) * TQW, tri_map, nT, lds);
}

template <int R, typename NT>
pl_status run(const NT *nin, const float *cen, int M, int N, float sl, float sa, int iterations,
              NT *nout, const int32_t *tri_map, NT *nT, NT *tmp, hipStream_t s) {
    const TileCfg c = tile_cfg(frame_stage(false, M, N), R);
    const int Mq = M - 1, Nq = N - 1;
    const int tiles_x = (Nq + c.tw - 1) / c.tw;
    const int ntiles = tiles_x * ((Mq + c.th - 1) / c.th);
    const float log2e = 1.4426950408889634f;
    const float ka = log2e / (2.0f * sl * sl);
    const float kb = log2e / (2.0f * sa * sa);
    // zero sweeps: one copying (and gathering) launch with F = 0
    const int launches = iterations == 0 ? 1 : (iterations + c.fuse - 1) / c.fuse;
    const NT *cur = nin;
    int left = iterations;
    for (int l = 0; l < launches; ++l) {
        const int F = left < c.fuse ? left : c.fuse;
        left -= F;
        const bool last = l == launches - 1;
        NT *dst = ((launches - 1 - l) % 2 == 0) ? nout : tmp;    // last launch lands in nout
        const size_t lds = bil_lds_bytes(R, F, c.th, c.tw, bil_waves(R, false));
        if (pl_status st = allow_lds((const void *)k_bilateral<R, NT>, lds)) return st;
        k_bilateral<R, NT><<<ntiles, kTileBlock, lds, s>>>(cur, cen, dst, Mq, Nq, ka, kb, F,
                                                            c.th, c.tw, tiles_x, ntiles,
                                                            last ? tri_map : nullptr, nT);
        if (pl_status st = hip_check(hipGetLastError(), "k_bilateral")) return st;
        cur = dst;
    }
    return PL_OK;
}

template <typename NT>
pl_status dispatch(const NT *nin, const float *cen, int M, int N, int kernel, float sl, float sa,
                   int iterations, NT *nout, const int32_t *tri_map, NT *nT, NT *tmp,
                   hipStream_t s) {
    switch (kernel / 2) {
    case 1: return run<1, NT>(nin, cen, M, N, sl, sa, iterations, nout, tri_map, nT, tmp, s);
    case 2: return run<2, NT>(nin, cen, M, N, sl, sa, iterations, nout, tri_map, nT, tmp, s);
    case 3: return run<3, NT>(nin, cen, M, N, sl, sa, iterations, nout, tri_map, nT, tmp, s);
    default: return run<4, NT>(nin, cen, M, N, sl, sa, iterations, nout, tri_map, nT, tmp, s);
    }
}

}  // namespace

size_t bilateral_workspace(int M, int N, pl_dtype ndt, int iterations) {
    const size_t T = 2 * (size_t)(M - 1) * (N - 1);
    return iterations > 1 ? T * 3 * (ndt == PL_F32 ? 4 : 2) : 0;
}

pl_status launch_bilateral(const void *nin, const float *cen, pl_dtype ndt, int M, int N,
                           int kernel, float sigma_length, float sigma_angle, int iterations,
                           void *nout, const int32_t *tri_map, void *normals_T, void *ws,
                           hipStream_t s) {
    if (ndt == PL_F32)
        return dispatch<float>(static_cast<const float *>(nin), cen, M, N, kernel, sigma_length,
                               sigma_angle, iterations, static_cast<float *>(nout), tri_map,
                               static_cast<float *>(normals_T), static_cast<float *>(ws), s);
    return dispatch<__half>(static_cast<const __half *>(nin), cen, M, N, kernel, sigma_length,
                            sigma_angle, iterations, static_cast<__half *>(nout), tri_map,
                            static_cast<__half *>(normals_T), static_cast<__half *>(ws), s);
}

}  // namespace pl
