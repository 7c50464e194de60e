// Bilateral triangle-normal filter on the organized mesh (Sec. 2.3 Eqs. 3-6;
// neighbourhood of Sec. 5.2) and the gather of the result onto T.
//
// The quad is the unit of work, as in the paper: one thread owns quad (u, v)
// and filters both of its triangles, which share every neighbour load.  A
// workgroup stages an 8 x 32 tile of quads plus an R-quad halo of normals and
// centroids in LDS; off-grid quads and triangles with a NaN normal or
// centroid are staged as a centroid at +inf and a zero normal, which gives
// them an infinite exponent, an exactly-zero weight and a zero contribution.
//
// Weights are evaluated as w = 2^(m - e) with
//     e = ||c_i - c_j||^2 * log2(e)/(2 sigma_l^2) + ||n_i - n_j||^2 * log2(e)/(2 sigma_a^2)
// and m the smallest exponent seen so far in the window.  The sum is
// renormalised, so the common factor 2^m cancels; keeping the largest term
// at 1 means FP32 never underflows to an all-zero sum where the exact sum is
// non-zero.  m is tracked per window row (an online rescale, one exp2 per
// row) so no exponent has to be kept for the whole window.
#include "common.h"

#include <float.h>

namespace pl {

namespace {

constexpr int TQH = 8;
constexpr int TQW = 32;
constexpr int kBlock = TQH * TQW;

struct BilGeom {
    int Mq, Nq;
    int tiles_x, ntiles;
};

template <typename NT>
__device__ __forceinline__ void load6(const NT *p, float *o) {
#pragma unroll
    for (int i = 0; i < 6; ++i) o[i] = ld_f(p + i);
}

template <int R, typename NT>
__global__ __launch_bounds__(kBlock) void k_bilateral(const NT *__restrict__ nin,
                                                      const float *__restrict__ cen,
                                                      NT *__restrict__ nout, BilGeom g,
                                                      float ka, float kb,
                                                      const int32_t *__restrict__ tri_map,
                                                      NT *__restrict__ nT) {
    constexpr int H = TQH + 2 * R, W = TQW + 2 * R;
    constexpr int RW = 2 * (2 * R + 1);       // neighbour triangles per window row
    __shared__ float4 sn[2][H * W];           // normal xyz, w = 1 if usable
    __shared__ float4 sc[2][H * W];           // centroid xyz
    const float inf = __builtin_inff();
    const int tile = xcd_remap(blockIdx.x, g.ntiles);
    const int qy0 = (tile / g.tiles_x) * TQH, qx0 = (tile % g.tiles_x) * TQW;
    const int oy = qy0 - R, ox = qx0 - R;

    for (int idx = threadIdx.x; idx < H * W; idx += kBlock) {
        const int ly = idx / W, lx = idx - ly * W;
        const int qy = oy + ly, qx = ox + lx;
        float4 n0 = make_float4(0.f, 0.f, 0.f, 0.f), n1 = n0;
        float4 c0 = make_float4(inf, inf, inf, 0.f), c1 = c0;
        if (qy >= 0 && qy < g.Mq && qx >= 0 && qx < g.Nq) {
            const size_t q = (size_t)qy * g.Nq + qx;
            float n[6], c[6];
            load6(nin + 6 * q, n);
            load6(cen + 6 * q, c);
            bool ok0 = true, ok1 = true;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                ok0 = ok0 && !is_nan_bits(n[i]) && !is_nan_bits(c[i]);
                ok1 = ok1 && !is_nan_bits(n[3 + i]) && !is_nan_bits(c[3 + i]);
            }
            if (ok0) { n0 = make_float4(n[0], n[1], n[2], 1.f); c0 = make_float4(c[0], c[1], c[2], 0.f); }
            if (ok1) { n1 = make_float4(n[3], n[4], n[5], 1.f); c1 = make_float4(c[3], c[4], c[5], 0.f); }
        }
        sn[0][idx] = n0; sn[1][idx] = n1;
        sc[0][idx] = c0; sc[1][idx] = c1;
    }
    __syncthreads();

    const int ty = threadIdx.x / TQW, tx = threadIdx.x - ty * TQW;
    const int qy = qy0 + ty, qx = qx0 + tx;
    if (qy >= g.Mq || qx >= g.Nq) return;
    const int ly = ty + R, lx = tx + R;
    const float4 ni0 = sn[0][ly * W + lx], ni1 = sn[1][ly * W + lx];
    const float4 ci0 = sc[0][ly * W + lx], ci1 = sc[1][ly * W + lx];

    float m0 = FLT_MAX, m1 = FLT_MAX;
    float s0x = 0.f, s0y = 0.f, s0z = 0.f, s1x = 0.f, s1y = 0.f, s1z = 0.f;
    // One window row at a time keeps only 2(2R+1) exponents per triangle live.
#pragma unroll 1
    for (int dy = -R; dy <= R; ++dy) {
        float e0[RW], e1[RW];
        float4 nj[RW];
        float r0 = inf, r1 = inf;
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) {
            const bool self = dy == 0 && dx == 0;      // own quad: not a neighbour
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int j = 2 * (dx + R) + kk;
                const int a = (ly + dy) * W + lx + dx;
                const float4 n = sn[kk][a], c = sc[kk][a];
                nj[j] = n;
                {
                    const float ax = ci0.x - c.x, ay = ci0.y - c.y, az = ci0.z - c.z;
                    const float bx = ni0.x - n.x, by = ni0.y - n.y, bz = ni0.z - n.z;
                    const float dc2 = fmaf(ax, ax, fmaf(ay, ay, az * az));
                    const float dn2 = fmaf(bx, bx, fmaf(by, by, bz * bz));
                    e0[j] = self ? inf : fmaf(dn2, kb, dc2 * ka);
                }
                {
                    const float ax = ci1.x - c.x, ay = ci1.y - c.y, az = ci1.z - c.z;
                    const float bx = ni1.x - n.x, by = ni1.y - n.y, bz = ni1.z - n.z;
                    const float dc2 = fmaf(ax, ax, fmaf(ay, ay, az * az));
                    const float dn2 = fmaf(bx, bx, fmaf(by, by, bz * bz));
                    e1[j] = self ? inf : fmaf(dn2, kb, dc2 * ka);
                }
                r0 = fminf(r0, e0[j]);
                r1 = fminf(r1, e1[j]);
            }
        }
        const float m0n = fminf(m0, r0), m1n = fminf(m1, r1);
        const float sc0 = __builtin_amdgcn_exp2f(m0n - m0), sc1 = __builtin_amdgcn_exp2f(m1n - m1);
        m0 = m0n; m1 = m1n;
        s0x *= sc0; s0y *= sc0; s0z *= sc0;
        s1x *= sc1; s1y *= sc1; s1z *= sc1;
#pragma unroll
        for (int j = 0; j < RW; ++j) {
            // unusable neighbours and the own quad have e = inf: weight exactly 0
            const float w0 = __builtin_amdgcn_exp2f(m0 - e0[j]);
            const float w1 = __builtin_amdgcn_exp2f(m1 - e1[j]);
            s0x = fmaf(w0, nj[j].x, s0x); s0y = fmaf(w0, nj[j].y, s0y); s0z = fmaf(w0, nj[j].z, s0z);
            s1x = fmaf(w1, nj[j].x, s1x); s1y = fmaf(w1, nj[j].y, s1y); s1z = fmaf(w1, nj[j].z, s1z);
        }
    }

    const size_t q = (size_t)qy * g.Nq + qx;
    float out[6];
    // triangle 0
    {
        const float l2 = fmaf(s0x, s0x, fmaf(s0y, s0y, s0z * s0z));
        const bool filt = ni0.w != 0.f && m0 < FLT_MAX && l2 > 0.f;
        if (filt) {
            const float k = __builtin_amdgcn_rsqf(l2);
            out[0] = s0x * k; out[1] = s0y * k; out[2] = s0z * k;
        }
        NT *o = nout + 6 * q;
        const NT *in = nin + 6 * q;
        if (filt) { st_f(o, out[0]); st_f(o + 1, out[1]); st_f(o + 2, out[2]); }
        else { o[0] = in[0]; o[1] = in[1]; o[2] = in[2]; }
    }
    {
        const float l2 = fmaf(s1x, s1x, fmaf(s1y, s1y, s1z * s1z));
        const bool filt = ni1.w != 0.f && m1 < FLT_MAX && l2 > 0.f;
        if (filt) {
            const float k = __builtin_amdgcn_rsqf(l2);
            out[3] = s1x * k; out[4] = s1y * k; out[5] = s1z * k;
        }
        NT *o = nout + 6 * q + 3;
        const NT *in = nin + 6 * q + 3;
        if (filt) { st_f(o, out[3]); st_f(o + 1, out[4]); st_f(o + 2, out[5]); }
        else { o[0] = in[0]; o[1] = in[1]; o[2] = in[2]; }
    }
    if (tri_map) {
        const int r0 = tri_map[2 * q], r1 = tri_map[2 * q + 1];
        const NT *o = nout + 6 * q;
        if (r0 >= 0) { nT[3 * (size_t)r0] = o[0]; nT[3 * (size_t)r0 + 1] = o[1]; nT[3 * (size_t)r0 + 2] = o[2]; }
        if (r1 >= 0) { nT[3 * (size_t)r1] = o[3]; nT[3 * (size_t)r1 + 1] = o[4]; nT[3 * (size_t)r1 + 2] = o[5]; }
    }
}

template <typename NT>
__global__ __launch_bounds__(256) void k_copy_gather(const NT *__restrict__ nin,
                                                    NT *__restrict__ nout, size_t Q,
                                                    const int32_t *__restrict__ tri_map,
                                                    NT *__restrict__ nT) {
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < Q; q += (size_t)gridDim.x * 256) {
        NT v[6];
#pragma unroll
        for (int i = 0; i < 6; ++i) { v[i] = nin[6 * q + i]; nout[6 * q + i] = v[i]; }
        if (tri_map) {
            const int r0 = tri_map[2 * q], r1 = tri_map[2 * q + 1];
            if (r0 >= 0) { nT[3 * (size_t)r0] = v[0]; nT[3 * (size_t)r0 + 1] = v[1]; nT[3 * (size_t)r0 + 2] = v[2]; }
            if (r1 >= 0) { nT[3 * (size_t)r1] = v[3]; nT[3 * (size_t)r1 + 1] = v[4]; nT[3 * (size_t)r1 + 2] = v[5]; }
        }
    }
}

template <int R, typename NT>
pl_status run(const NT *nin, const float *cen, int M, int N, float sl, float sa,
              int iterations, NT *nout, const int32_t *tri_map, NT *nT, NT *tmp,
              hipStream_t s) {
    BilGeom g;
    g.Mq = M - 1;
    g.Nq = N - 1;
    g.tiles_x = (g.Nq + TQW - 1) / TQW;
    g.ntiles = g.tiles_x * ((g.Mq + TQH - 1) / TQH);
    const float log2e = 1.4426950408889634f;
    const float ka = log2e / (2.0f * sl * sl);
    const float kb = log2e / (2.0f * sa * sa);
    const NT *cur = nin;
    for (int it = 0; it < iterations; ++it) {
        const bool last = it == iterations - 1;
        NT *dst = ((iterations - 1 - it) % 2 == 0) ? nout : tmp;
        k_bilateral<R, NT><<<g.ntiles, kBlock, 0, s>>>(cur, cen, dst, g, ka, kb,
                                                       last ? tri_map : nullptr, nT);
        if (pl_status st = hip_check(hipGetLastError(), "k_bilateral")) return st;
        cur = dst;
    }
    return PL_OK;
}

template <typename NT>
pl_status dispatch(const NT *nin, const float *cen, int M, int N, int kernel, float sl,
                   float sa, int iterations, NT *nout, const int32_t *tri_map, NT *nT,
                   NT *tmp, hipStream_t s) {
    if (iterations == 0) {
        const size_t Q = (size_t)(M - 1) * (N - 1);
        const size_t want = (Q + 255) / 256;
        const int blocks = (int)(want < 4096 ? want : 4096);
        k_copy_gather<NT><<<blocks, 256, 0, s>>>(nin, nout, Q, tri_map, nT);
        return hip_check(hipGetLastError(), "k_copy_gather");
    }
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
