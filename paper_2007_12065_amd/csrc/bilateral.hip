// Bilateral triangle-normal filter on the organized mesh (Sec. 2.3 Eqs. 3-6;
// neighbourhood of Sec. 5.2) and the gather of the result onto T.
//
// Work decomposition.  The quad is the unit of work, as in the paper: a
// thread owns quad (u, v) and filters both of its triangles, which share
// every neighbour load.  A workgroup owns an 8 x 32 tile of quads.  It stages
// the tile plus a halo of R*F quads (R = kernel/2, F = sweeps fused in this
// launch) in LDS and runs the F Jacobi sweeps there: sweep f updates the
// region that is still exact after f steps, and the last sweep writes the
// tile to global memory (and gathers it onto T when asked).  Fusing sweeps
// trades a little redundant halo work for one HBM round trip of the normals
// and one launch per fused sweep.
//
// Arithmetic.  With log2(e) folded in, the weight of neighbour j is
//     w_j = 2^-e_j,  e_j = ka ||c_i - c_j||^2 + kb ||n_i - n_j||^2,
//     ka = log2(e) / (2 sigma_l^2),  kb = log2(e) / (2 sigma_a^2).
// Both squared distances are formed from component differences (exact for
// nearby float32 values), then scaled: fourteen FMA-class instructions per
// pair, one exp2 and four FMAs to accumulate.  Expanding the normal term as
// |n_i|^2 + |n_j|^2 - 2 n_i.n_j, or pre-scaling the centroids by sqrt(ka),
// would save instructions but rounds before the subtraction, which costs
// ~1e-5 relative weight accuracy.
//
// Underflow.  Eq. 6 renormalises, so a common factor of the weights cancels.
// Since e_j >= 0 every weight is <= 1 and nothing overflows; if the whole
// neighbourhood is so far away that the total weight drops below 2^-60, the
// triangle is recomputed with every exponent shifted by the smallest one
// (the same value in exact arithmetic), which keeps the largest term at 1.
// Only the lanes that need it take that path.
//
// Missing data.  Off-grid quads and triangles with a NaN normal or centroid
// are staged with an infinite centroid and a zero normal: their exponent is
// +inf, their weight exactly 0 and their contribution 0.  A triangle that is
// itself missing is copied through unchanged (its input bits).
//
// Float16 storage.  Normals produced by an intermediate fused sweep are
// rounded to float16, exactly as if they had been stored between launches,
// so the result does not depend on how many sweeps a launch fuses.
#include "common.h"

#include <float.h>

namespace pl {

namespace {

constexpr int TQH = 8;
constexpr int TQW = 32;
constexpr int kBlock = TQH * TQW;
constexpr float kUnderflow = 8.673617e-19f;    // 2^-60

struct BilGeom {
    int Mq, Nq;
    int tiles_x, ntiles;
};

template <typename NT> __device__ __forceinline__ float round_storage(float x);
template <> __device__ __forceinline__ float round_storage<float>(float x) { return x; }
template <> __device__ __forceinline__ float round_storage<__half>(float x) {
    return __half2float(__float2half_rn(x));
}

#ifndef PL_BIL_FOLDED
#define PL_BIL_FOLDED 0        // expand ||n_i - n_j||^2 (fewer ops, more rounding)
#endif
#ifndef PL_BIL_FUSE
#define PL_BIL_FUSE 1          // sweeps fused per launch for the 3x3 window
#endif
#ifndef PL_BIL_UNROLL_ROW
#define PL_BIL_UNROLL_ROW 1    // unroll the neighbours of one window row
#endif

struct Own {
    float cx, cy, cz;          // centroid
    float nx, ny, nz;          // n_i (folded form: -2 kb n_i)
    float q;                   // kb (folded form: kb |n_i|^2)
    float ka;
};

__device__ __forceinline__ Own own_of(const float4 c, const float4 n, float ka, float kb) {
    Own o;
    o.cx = c.x; o.cy = c.y; o.cz = c.z;
    o.ka = ka;
#if PL_BIL_FOLDED
    const float m = -2.0f * kb;
    o.nx = m * n.x; o.ny = m * n.y; o.nz = m * n.z;
    o.q = n.w;
#else
    o.nx = n.x; o.ny = n.y; o.nz = n.z;
    o.q = kb;
#endif
    return o;
}

// Exponent of the pair (own, neighbour), in log2 units.
#if PL_BIL_FOLDED
__device__ __forceinline__ float pair_e(const Own &o, const float4 c, const float4 n) {
    float t = n.w + o.q;
    t = fmaf(o.nx, n.x, fmaf(o.ny, n.y, fmaf(o.nz, n.z, t)));
    const float dx = o.cx - c.x, dy = o.cy - c.y, dz = o.cz - c.z;
    return fmaf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)), o.ka, t);
}
#else
__device__ __forceinline__ float pair_e(const Own &o, const float4 c, const float4 n) {
    const float ax = o.nx - n.x, ay = o.ny - n.y, az = o.nz - n.z;
    const float dn2 = fmaf(ax, ax, fmaf(ay, ay, az * az));
    const float dx = o.cx - c.x, dy = o.cy - c.y, dz = o.cz - c.z;
    const float dc2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    return fmaf(dc2, o.ka, dn2 * o.q);
}
#endif

struct Acc {
    float x, y, z, w;
};

__device__ __forceinline__ void accumulate(Acc &s, const Own &o, const float4 c, const float4 n) {
    const float w = __builtin_amdgcn_exp2f(-pair_e(o, c, n));
    s.w += w;
    s.x = fmaf(w, n.x, s.x);
    s.y = fmaf(w, n.y, s.y);
    s.z = fmaf(w, n.z, s.z);
}

// The rare path: every exponent shifted by the smallest usable one.
template <int R>
__device__ __forceinline__ Acc shifted_sum(const Own o, const float4 *sc, const float4 *sn,
                                        int a0, int pitch, int plane) {
    const float inf = __builtin_inff();
    float m = inf;
#pragma unroll 1
    for (int dy = -R; dy <= R; ++dy)
#pragma unroll 1
        for (int dx = -R; dx <= R; ++dx) {
            if (dy == 0 && dx == 0) continue;
            for (int kk = 0; kk < 2; ++kk) {
                const int b = a0 + dy * pitch + dx + kk * plane;
                m = fminf(m, pair_e(o, sc[b], sn[b]));
            }
        }
    Acc s{0.f, 0.f, 0.f, 0.f};
    if (!(m < inf)) return s;               // no usable neighbour
#pragma unroll 1
    for (int dy = -R; dy <= R; ++dy)
#pragma unroll 1
        for (int dx = -R; dx <= R; ++dx) {
            if (dy == 0 && dx == 0) continue;
            for (int kk = 0; kk < 2; ++kk) {
                const int b = a0 + dy * pitch + dx + kk * plane;
                const float4 n = sn[b];
                const float w = __builtin_amdgcn_exp2f(m - pair_e(o, sc[b], n));
                s.w += w;
                s.x = fmaf(w, n.x, s.x);
                s.y = fmaf(w, n.y, s.y);
                s.z = fmaf(w, n.z, s.z);
            }
        }
    return s;
}

// New normal of one triangle from its accumulated sum; `cur` is its current
// value (returned when it has no usable neighbour or the sum vanishes).
template <typename NT>
__device__ __forceinline__ float4 finish(Acc s, float4 cur, float kb) {
    const float l2 = fmaf(s.x, s.x, fmaf(s.y, s.y, s.z * s.z));
    if (!(s.w > 0.f) || !(l2 > 0.f)) return cur;
    const float k = __builtin_amdgcn_rsqf(l2);
    float4 r;
    r.x = round_storage<NT>(s.x * k);
    r.y = round_storage<NT>(s.y * k);
    r.z = round_storage<NT>(s.z * k);
    r.w = kb * fmaf(r.x, r.x, fmaf(r.y, r.y, r.z * r.z));
    return r;
}

// Filter both triangles of the quad at LDS index a.
template <int R, typename NT>
__device__ __forceinline__ void filter_quad(const float4 *sc, const float4 *sn, int a, int pitch,
                                            int plane, float ka, float kb, float4 &r0,
                                            float4 &r1) {
    const float4 c0 = sc[a], c1 = sc[plane + a];
    const float4 n0 = sn[a], n1 = sn[plane + a];
    const Own o0 = own_of(c0, n0, ka, kb), o1 = own_of(c1, n1, ka, kb);
    Acc s0{0.f, 0.f, 0.f, 0.f}, s1{0.f, 0.f, 0.f, 0.f};
    // one window row per iteration keeps only that row's neighbours live
#pragma unroll 1
    for (int dy = -R; dy <= R; ++dy) {
#if PL_BIL_UNROLL_ROW
#pragma unroll
#else
#pragma unroll 1
#endif
        for (int dx = -R; dx <= R; ++dx) {
            if (dy == 0 && dx == 0) continue;     // the own quad is not a neighbour
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                const int b = a + dy * pitch + dx + kk * plane;
                const float4 c = sc[b], n = sn[b];
                accumulate(s0, o0, c, n);
                accumulate(s1, o1, c, n);
            }
        }
    }
    const bool ok0 = c0.w != 0.f, ok1 = c1.w != 0.f;
    if (ok0 && !(s0.w >= kUnderflow)) s0 = shifted_sum<R>(o0, sc, sn, a, pitch, plane);
    if (ok1 && !(s1.w >= kUnderflow)) s1 = shifted_sum<R>(o1, sc, sn, a, pitch, plane);
    r0 = ok0 ? finish<NT>(s0, n0, kb) : n0;
    r1 = ok1 ? finish<NT>(s1, n1, kb) : n1;
}

template <int R, int F, typename NT>
__global__ __launch_bounds__(kBlock) void k_bilateral(const NT *__restrict__ nin,
                                                      const float *__restrict__ cen,
                                                      NT *__restrict__ nout, BilGeom g,
                                                      float ka, float kb,
                                                      const int32_t *__restrict__ tri_map,
                                                      NT *__restrict__ nT) {
    constexpr int H = TQH + 2 * R * F, W = TQW + 2 * R * F, S = H * W;
    __shared__ float4 s_c[2 * S];                      // centroids, w = 1 if usable
    __shared__ float4 s_n[2 * S];                      // normals, w = kb |n|^2
    __shared__ float4 s_m[F > 1 ? 2 * S : 1];          // second normal buffer
    const float inf = __builtin_inff();
    const int tile = xcd_remap(blockIdx.x, g.ntiles);
    const int qy0 = (tile / g.tiles_x) * TQH, qx0 = (tile % g.tiles_x) * TQW;
    const int oy = qy0 - R * F, ox = qx0 - R * F;

    for (int idx = threadIdx.x; idx < S; idx += kBlock) {
        const int ly = idx / W, lx = idx - ly * W;
        const int qy = oy + ly, qx = ox + lx;
        float4 c0 = make_float4(inf, inf, inf, 0.f), c1 = c0;
        float4 n0 = make_float4(0.f, 0.f, 0.f, 0.f), n1 = n0;
        if (qy >= 0 && qy < g.Mq && qx >= 0 && qx < g.Nq) {
            const size_t q = (size_t)qy * g.Nq + qx;
            float n[6], c[6];
#pragma unroll
            for (int i = 0; i < 6; ++i) { n[i] = ld_f(nin + 6 * q + i); c[i] = cen[6 * q + i]; }
            bool ok0 = true, ok1 = true;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                ok0 = ok0 && !is_nan_bits(n[i]) && !is_nan_bits(c[i]);
                ok1 = ok1 && !is_nan_bits(n[3 + i]) && !is_nan_bits(c[3 + i]);
            }
            if (ok0) {
                c0 = make_float4(c[0], c[1], c[2], 1.f);
                n0 = make_float4(n[0], n[1], n[2], kb * fmaf(n[0], n[0], fmaf(n[1], n[1], n[2] * n[2])));
            }
            if (ok1) {
                c1 = make_float4(c[3], c[4], c[5], 1.f);
                n1 = make_float4(n[3], n[4], n[5], kb * fmaf(n[3], n[3], fmaf(n[4], n[4], n[5] * n[5])));
            }
        }
        s_c[idx] = c0; s_c[S + idx] = c1;
        s_n[idx] = n0; s_n[S + idx] = n1;
    }
    __syncthreads();

    const float4 *cur = s_n;
    float4 *nxt = s_m;
    // intermediate sweeps: LDS to LDS over the shrinking exact region
    for (int f = 1; f < F; ++f) {
        const int lo = R * f;
        const int Hf = H - 2 * lo, Wf = W - 2 * lo;
        for (int idx = threadIdx.x; idx < Hf * Wf; idx += kBlock) {
            const int ry = idx / Wf;
            const int a = (lo + ry) * W + lo + (idx - ry * Wf);
            float4 r0, r1;
            filter_quad<R, NT>(s_c, cur, a, W, S, ka, kb, r0, r1);
            nxt[a] = r0;
            nxt[S + a] = r1;
        }
        __syncthreads();
        float4 *t = const_cast<float4 *>(cur);
        cur = nxt;
        nxt = t;
    }

    // last sweep: the tile itself, straight to global memory
    const int ty = threadIdx.x / TQW, tx = threadIdx.x - ty * TQW;
    const int qy = qy0 + ty, qx = qx0 + tx;
    if (qy >= g.Mq || qx >= g.Nq) return;
    const int a = (ty + R * F) * W + tx + R * F;
    float4 r[2];
    filter_quad<R, NT>(s_c, cur, a, W, S, ka, kb, r[0], r[1]);
    const size_t q = (size_t)qy * g.Nq + qx;
    NT v[6];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        if (s_c[k * S + a].w != 0.f) {
            st_f(&v[3 * k], r[k].x); st_f(&v[3 * k + 1], r[k].y); st_f(&v[3 * k + 2], r[k].z);
        } else {                       // missing triangle: input bits unchanged
            v[3 * k] = nin[6 * q + 3 * k];
            v[3 * k + 1] = nin[6 * q + 3 * k + 1];
            v[3 * k + 2] = nin[6 * q + 3 * k + 2];
        }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) nout[6 * q + i] = v[i];
    if (tri_map) {
        const int t0 = tri_map[2 * q], t1 = tri_map[2 * q + 1];
        if (t0 >= 0) { nT[3 * (size_t)t0] = v[0]; nT[3 * (size_t)t0 + 1] = v[1]; nT[3 * (size_t)t0 + 2] = v[2]; }
        if (t1 >= 0) { nT[3 * (size_t)t1] = v[3]; nT[3 * (size_t)t1 + 1] = v[4]; nT[3 * (size_t)t1 + 2] = v[5]; }
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

// Sweeps fused per launch for a window radius: the halo grows by R per
// fused sweep, so only the 3x3 window fuses (16% redundant work at F = 2).
int max_fused(int R) { return R == 1 ? PL_BIL_FUSE : 1; }

template <int R, int F, typename NT>
pl_status launch_one(const NT *cur, const float *cen, NT *dst, const BilGeom &g, float ka,
                     float kb, const int32_t *tri_map, NT *nT, hipStream_t s) {
    k_bilateral<R, F, NT><<<g.ntiles, kBlock, 0, s>>>(cur, cen, dst, g, ka, kb, tri_map, nT);
    return hip_check(hipGetLastError(), "k_bilateral");
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
    const int Fmax = max_fused(R);
    const int launches = (iterations + Fmax - 1) / Fmax;
    const NT *cur = nin;
    int left = iterations;
    for (int l = 0; l < launches; ++l) {
        const int F = left < Fmax ? left : Fmax;
        left -= F;
        const bool last = l == launches - 1;
        NT *dst = ((launches - 1 - l) % 2 == 0) ? nout : tmp;
        const int32_t *tm = last ? tri_map : nullptr;
        pl_status st;
        if (F == 2 && R == 1) st = launch_one<1, 2, NT>(cur, cen, dst, g, ka, kb, tm, nT, s);
        else st = launch_one<R, 1, NT>(cur, cen, dst, g, ka, kb, tm, nT, s);
        if (st) return st;
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
