// Laplacian vertex filter on the organized cloud (Sec. 2.3 Eqs. 1-2; image
// neighbourhood of Sec. 5.1) with temporal blocking.
//
// Each workgroup owns a TH x TW tile of output pixels.  It stages the tile
// plus a halo of R*F pixels (R = kernel/2, F = sweeps fused in this launch)
// in LDS as float4 (x, y, z, pad), runs F Jacobi sweeps between two LDS
// buffers -- sweep f updates the region that is still exact after f steps,
// shrinking by R per side -- and writes the TH x TW centre back.  HBM sees
// one read and one write of the points per F sweeps; the rest of the cost
// is the per-neighbour arithmetic (one rsqrt and eight FMAs per neighbour).
//
// Invalid pixels (any NaN coordinate) and pixels outside the image are
// staged as (0, 0, 0, +inf): the pad makes the squared distance +inf, whose
// reciprocal square root is exactly 0, so they drop out of both sums without
// a branch and without NaN reaching the accumulators.  Invalid pixels and the
// image border band are never updated; invalid pixels are written back from
// the input bits.
#include "common.h"

namespace pl {

namespace {

#ifndef PL_LAP_TH
#define PL_LAP_TH 16
#endif
#ifndef PL_LAP_TW
#define PL_LAP_TW 64
#endif
#ifndef PL_LAP_FUSE
#define PL_LAP_FUSE 4          // sweeps fused per launch for the 3x3 window
#endif
constexpr int TH = PL_LAP_TH;
constexpr int TW = PL_LAP_TW;
constexpr int kBlock = 256;

struct LapGeom {
    int M, N;
    int tiles_x, ntiles;
};

template <int R>
__global__ __launch_bounds__(kBlock) void k_laplacian(const float *__restrict__ src,
                                                      float *__restrict__ dst, LapGeom g,
                                                      float lam, int F) {
    extern __shared__ float4 lds[];
    const int halo = R * F;
    const int H = TH + 2 * halo, W = TW + 2 * halo;
    float4 *A = lds;
    float4 *B = lds + H * W;
    const int tile = xcd_remap(blockIdx.x, g.ntiles);
    const int ty0 = (tile / g.tiles_x) * TH, tx0 = (tile % g.tiles_x) * TW;
    const int oy = ty0 - halo, ox = tx0 - halo;
    const float inf = __builtin_inff();

    for (int idx = threadIdx.x; idx < H * W; idx += kBlock) {
        const int ly = idx / W, lx = idx - ly * W;
        const int gy = oy + ly, gx = ox + lx;
        float4 p = make_float4(0.f, 0.f, 0.f, inf);
        if (gy >= 0 && gy < g.M && gx >= 0 && gx < g.N) {
            const float *q = src + 3 * ((size_t)gy * g.N + gx);
            const float x = q[0], y = q[1], z = q[2];
            if (!(is_nan_bits(x) || is_nan_bits(y) || is_nan_bits(z))) p = make_float4(x, y, z, 0.f);
        }
        A[idx] = p;
    }
    __syncthreads();

    for (int f = 1; f <= F; ++f) {
        const int lo = R * f;
        const int Hf = H - 2 * lo, Wf = W - 2 * lo;
        for (int idx = threadIdx.x; idx < Hf * Wf; idx += kBlock) {
            const int ry = idx / Wf;
            const int ly = lo + ry, lx = lo + (idx - ry * Wf);
            const int gy = oy + ly, gx = ox + lx;
            const float4 c = A[ly * W + lx];
            float4 o = c;
            const bool active = c.w == 0.f && gy >= R && gy < g.M - R && gx >= R && gx < g.N - R;
            if (active) {
                float ws = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
                for (int dy = -R; dy <= R; ++dy) {
#pragma unroll
                    for (int dx = -R; dx <= R; ++dx) {
                        if (dy == 0 && dx == 0) continue;
                        const float4 p = A[(ly + dy) * W + lx + dx];
                        const float ex = p.x - c.x, ey = p.y - c.y, ez = p.z - c.z;
                        const float d2 = fmaf(ex, ex, fmaf(ey, ey, fmaf(ez, ez, p.w)));
                        float w = __builtin_amdgcn_rsqf(d2);     // 1/||v_j - v_i||
                        w = d2 > 0.f ? w : 0.f;                   // coincident: skipped
                        ws += w;
                        sx = fmaf(w, ex, sx);
                        sy = fmaf(w, ey, sy);
                        sz = fmaf(w, ez, sz);
                    }
                }
                if (ws > 0.f) {
                    const float k = lam / ws;
                    o.x = fmaf(k, sx, c.x);
                    o.y = fmaf(k, sy, c.y);
                    o.z = fmaf(k, sz, c.z);
                }
            }
            B[ly * W + lx] = o;
        }
        __syncthreads();
        float4 *t = A; A = B; B = t;
    }

    for (int idx = threadIdx.x; idx < TH * TW; idx += kBlock) {
        const int ry = idx / TW, rx = idx - ry * TW;
        const int gy = ty0 + ry, gx = tx0 + rx;
        if (gy >= g.M || gx >= g.N) continue;
        const size_t off = 3 * ((size_t)gy * g.N + gx);
        const float4 c = A[(ry + halo) * W + rx + halo];
        if (c.w == 0.f) {
            dst[off] = c.x; dst[off + 1] = c.y; dst[off + 2] = c.z;
        } else {
            dst[off] = src[off]; dst[off + 1] = src[off + 1]; dst[off + 2] = src[off + 2];
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_copy_f32(const float *__restrict__ a,
                                                     float *__restrict__ b, size_t n) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (size_t)gridDim.x * kBlock)
        b[i] = a[i];
}

// Sweeps fused per launch: more sweeps cut HBM traffic but grow the halo
// (LDS and redundant edge work).
int max_fused(int R) { return R == 1 ? PL_LAP_FUSE : (R == 2 ? (PL_LAP_FUSE + 1) / 2 : 1); }

template <int R>
pl_status run(const float *in, float *out, int M, int N, float lam, int iterations,
              float *tmp, hipStream_t s) {
    LapGeom g;
    g.M = M;
    g.N = N;
    g.tiles_x = (N + TW - 1) / TW;
    g.ntiles = g.tiles_x * ((M + TH - 1) / TH);
    const int Fmax = max_fused(R);
    const int launches = (iterations + Fmax - 1) / Fmax;
    const float *cur = in;
    int left = iterations;
    for (int l = 0; l < launches; ++l) {
        const int F = left < Fmax ? left : Fmax;
        left -= F;
        // alternate so that the last launch lands in `out`
        float *dst = ((launches - 1 - l) % 2 == 0) ? out : tmp;
        const int halo = R * F;
        const size_t lds = 2 * sizeof(float4) * (TH + 2 * halo) * (TW + 2 * halo);
        k_laplacian<R><<<g.ntiles, kBlock, lds, s>>>(cur, dst, g, lam, F);
        if (pl_status st = hip_check(hipGetLastError(), "k_laplacian")) return st;
        cur = dst;
    }
    return PL_OK;
}

}  // namespace

int laplacian_fused_sweeps(int kernel) { return max_fused(kernel / 2); }

size_t laplacian_workspace(int M, int N, int iterations) {
    // an intermediate point buffer is needed once there are two launches
    return iterations > 1 ? sizeof(float) * 3 * (size_t)M * N : 0;
}

pl_status launch_laplacian(const float *in, float *out, int M, int N, int kernel,
                           float lambda, int iterations, void *ws, hipStream_t s) {
    if (iterations == 0) {
        const size_t n = 3 * (size_t)M * N;
        const int blocks = (int)((n + kBlock - 1) / kBlock < 4096 ? (n + kBlock - 1) / kBlock : 4096);
        k_copy_f32<<<blocks, kBlock, 0, s>>>(in, out, n);
        return hip_check(hipGetLastError(), "k_copy_f32");
    }
    float *tmp = static_cast<float *>(ws);
    switch (kernel / 2) {
    case 1: return run<1>(in, out, M, N, lambda, iterations, tmp, s);
    case 2: return run<2>(in, out, M, N, lambda, iterations, tmp, s);
    case 3: return run<3>(in, out, M, N, lambda, iterations, tmp, s);
    default: return run<4>(in, out, M, N, lambda, iterations, tmp, s);
    }
}

}  // namespace pl
