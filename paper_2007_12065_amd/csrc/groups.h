// Group assignment (Sec. 7.1, Alg. 4): device body shared by the
// single-call kernel and the batched path.  One label per triangle of T, the
// index of the most similar dominant plane normal, or 255 when an edge of the
// triangle is longer than l_max or the best similarity is below ang_min.
//
// Streaming work over T: each thread takes four consecutive triangles, so
// the triangle list and float32 normals arrive as 16-byte loads and the four
// labels leave as one 32-bit store.  The vertices are gathered from the
// point array (a triangle's vertices sit in two neighbouring image rows, so
// consecutive triangles share cache lines).  The dominant normals are read
// at wave-uniform addresses (scalar loads), so the loop over them costs
// three fused multiply-adds, a compare and two selects per normal and
// triangle.
//
// Every comparison is taken in float32 with the products written as fmaf in
// a fixed order (the build disables implicit contraction), which makes the
// labels a function of the float32 inputs alone.
#pragma once

#include "common.h"

namespace pl {

constexpr int kGroupBlock = 256;  // threads per workgroup
constexpr int kGroupPer = 4;      // triangles per thread
constexpr uint32_t kSentinel = 255u;

__device__ __forceinline__ float sq_dist(float ax, float ay, float az, float bx, float by,
                                         float bz) {
    const float dx = ax - bx, dy = ay - by, dz = az - bz;
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Labels of K triangles (vertex indices idx[3k..3k+2], normals
// nrm[3k..3k+2]).  An index outside [0, n_pts) or an edge that is NaN or
// longer than l_max gives the sentinel; a NaN normal beats no similarity and
// keeps it.  Every vertex load is issued before any arithmetic, and the loop
// over the dominant normals runs once for all K triangles, so each normal is
// loaded once per thread.  Requires n_pts > 0 (an index out of range loads
// point 0 and is then discarded).
template <int K>
__device__ __forceinline__ void labels(const float *__restrict__ pts, int n_pts, const int *idx,
                                       const float *nrm, const float *__restrict__ dom, int l,
                                       float lmax2, float ang_min, uint32_t *out) {
    float v[K][9];
    bool in_range[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        in_range[k] = true;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int i = idx[3 * k + c];
            const bool ok = (unsigned)i < (unsigned)n_pts;
            in_range[k] = in_range[k] & ok;
            const float *p = pts + 3 * (size_t)(ok ? i : 0);
            v[k][3 * c] = p[0];
            v[k][3 * c + 1] = p[1];
            v[k][3 * c + 2] = p[2];
        }
    }
    bool keep[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float *a = v[k], *b = v[k] + 3, *c = v[k] + 6;
        const float e0 = sq_dist(a[0], a[1], a[2], b[0], b[1], b[2]);
        const float e1 = sq_dist(b[0], b[1], b[2], c[0], c[1], c[2]);
        const float e2 = sq_dist(c[0], c[1], c[2], a[0], a[1], a[2]);
        // non-short-circuit: every load stays unconditional and in flight together
        keep[k] = in_range[k] & (e0 <= lmax2) & (e1 <= lmax2) & (e2 <= lmax2);
    }
    float best[K];
    uint32_t g[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        best[k] = -1.0f;
        g[k] = kSentinel;
    }
    for (int j = 0; j < l; ++j) {
        const float dx = dom[3 * j], dy = dom[3 * j + 1], dz = dom[3 * j + 2];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float sim = fmaf(nrm[3 * k], dx, fmaf(nrm[3 * k + 1], dy, nrm[3 * k + 2] * dz));
            if (sim > best[k]) {
                g[k] = (uint32_t)j;
                best[k] = sim;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = (!keep[k] || best[k] < ang_min) ? kSentinel : g[k];
}

// One thread's rows [t0, t0 + 4) of T (those below min(*n_tri, cap)).
template <typename NT>
__device__ __forceinline__ void group_rows(const float *__restrict__ pts, int n_pts,
                                           const int32_t *__restrict__ tris,
                                           const NT *__restrict__ normals,
                                           const int32_t *__restrict__ n_tri, int cap,
                                           const float *__restrict__ dom, int l, float lmax2,
                                           float ang_min, uint8_t *__restrict__ groups, int t0) {
    if (t0 >= cap) return;
    // The rows of a whole group of four lie inside the arrays whatever |T|
    // is, so their loads are issued before the count arrives: the count and
    // the rows then cost one memory round trip, not two.
    const bool whole = t0 + kGroupPer <= cap;
    int idx[3 * kGroupPer];
    float nrm[3 * kGroupPer];
    if (whole) {
        // 3 x 16 B of indices, 3 x 16 B (float) or 24 B (half) of normals
        const int4 *tv = reinterpret_cast<const int4 *>(tris + 3 * (size_t)t0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int4 q = tv[k];
            idx[4 * k] = q.x;
            idx[4 * k + 1] = q.y;
            idx[4 * k + 2] = q.z;
            idx[4 * k + 3] = q.w;
        }
        if constexpr (sizeof(NT) == 4) {
            const float4 *nv = reinterpret_cast<const float4 *>(normals + 3 * (size_t)t0);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float4 q = nv[k];
                nrm[4 * k] = q.x;
                nrm[4 * k + 1] = q.y;
                nrm[4 * k + 2] = q.z;
                nrm[4 * k + 3] = q.w;
            }
        } else {
            const uint2 *nv = reinterpret_cast<const uint2 *>(normals + 3 * (size_t)t0);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const uint2 q = nv[k];
                const uint32_t w[2] = {q.x, q.y};
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    nrm[4 * k + 2 * h] = __half2float(__ushort_as_half((unsigned short)(w[h] & 0xffffu)));
                    nrm[4 * k + 2 * h + 1] = __half2float(__ushort_as_half((unsigned short)(w[h] >> 16)));
                }
            }
        }
    }
    const int n = min(max(*n_tri, 0), cap);
    if (t0 >= n) return;
    if (n_pts == 0) {  // no vertex index is in range
        for (int t = t0; t < min(t0 + kGroupPer, n); ++t) groups[t] = (uint8_t)kSentinel;
        return;
    }
    if (t0 + kGroupPer <= n) {  // four triangles of T (whole holds as n <= cap)
        uint32_t g[kGroupPer];
        labels<kGroupPer>(pts, n_pts, idx, nrm, dom, l, lmax2, ang_min, g);
        uint32_t out = 0;
#pragma unroll
        for (int k = 0; k < kGroupPer; ++k) out |= g[k] << (8 * k);
        *reinterpret_cast<uint32_t *>(groups + t0) = out;
        return;
    }
    // the last, partial group of T: element loads, byte stores, nothing
    // written at or past n
    for (int t = t0; t < n; ++t) {
        int idx1[3];
        float nrm1[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            idx1[c] = tris[3 * (size_t)t + c];
            nrm1[c] = ld_f(normals + 3 * (size_t)t + c);
        }
        uint32_t g;
        labels<1>(pts, n_pts, idx1, nrm1, dom, l, lmax2, ang_min, &g);
        groups[t] = (uint8_t)g;
    }
}

}  // namespace pl
