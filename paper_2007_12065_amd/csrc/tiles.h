// Per-tile device bodies shared by the single-frame kernels and the batched
// kernels, so that a frame gets bit-for-bit the same result
// whichever way it is launched.  Tile shapes and the number of fused sweeps
// are runtime values (LDS is dynamic), which lets the tuner pick them.
#pragma once

#include "common.h"

#include <float.h>
#include <type_traits>

namespace pl {

constexpr int kTileBlock = 256;        // threads per workgroup for every tile body

// ---------------------------------------------------------------------------
// Mesh (Sec. 4.2, Alg. 1 and Alg. 2), one quad row per call.
// ---------------------------------------------------------------------------

constexpr int kMeshChunk = 4 * kTileBlock;    // columns staged per pass

// Validity codes of quad row u (bit 0: first triangle, bit 1: second) and the
// row's triangle count.  All point loads of a 1024-column chunk are issued
// before any is used; point validity is staged in LDS.
struct MeshCountRowLds {
    uint8_t ok[2][kMeshChunk + 1];
};

__device__ __forceinline__ void mesh_count_row(const float *__restrict__ pts, int N, int u,
                                               uint8_t *__restrict__ codes,
                                               uint8_t *__restrict__ tri_valid,
                                               int *__restrict__ row_count,
                                               MeshCountRowLds &L) {
    auto &ok = L.ok;
    __shared__ int red[kTileBlock / kWave];
    const int Nq = N - 1;
    const float *r0 = pts + (size_t)u * N * 3;
    const float *r1 = r0 + (size_t)N * 3;
    int cnt = 0;
    for (int v0 = 0; v0 < Nq; v0 += kMeshChunk) {
        float x[2][5], y[2][5], z[2][5];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int v = v0 + threadIdx.x + j * kTileBlock;
            const bool in = (j < 4 || threadIdx.x == 0) && v < N && v <= v0 + kMeshChunk;
            x[0][j] = in ? r0[3 * v] : 0.f; y[0][j] = in ? r0[3 * v + 1] : 0.f; z[0][j] = in ? r0[3 * v + 2] : 0.f;
            x[1][j] = in ? r1[3 * v] : 0.f; y[1][j] = in ? r1[3 * v + 1] : 0.f; z[1][j] = in ? r1[3 * v + 2] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int l = threadIdx.x + j * kTileBlock;
            if (j < 4 || threadIdx.x == 0) {
#pragma unroll
                for (int r = 0; r < 2; ++r)
                    ok[r][l] = !(is_nan_bits(x[r][j]) || is_nan_bits(y[r][j]) || is_nan_bits(z[r][j]));
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int l = threadIdx.x + j * kTileBlock;
            const int v = v0 + l;
            if (v < Nq) {
                const int p1 = ok[0][l], p2 = ok[0][l + 1], p3 = ok[1][l + 1], p4 = ok[1][l];
                const int f = p1 & p2 & p3;          // first triangle (p3, p2, p1)
                const int s = p1 & p3 & p4;          // second triangle (p1, p4, p3)
                const size_t q = (size_t)u * Nq + v;
                codes[q] = (uint8_t)(f | (s << 1));
                if (tri_valid) {
                    tri_valid[2 * q] = (uint8_t)f;
                    tri_valid[2 * q + 1] = (uint8_t)s;
                }
                cnt += f + s;
            }
        }
        __syncthreads();
    }
    cnt = wave_sum(cnt);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
#pragma unroll
        for (int w = 0; w < kTileBlock / kWave; ++w) t += red[w];
        row_count[u] = t;
    }
}

// Block-wide exclusive scan of three counters packed in 21-bit fields (a
// pass of 1024 quads holds at most 2048 triangles per row).
__device__ __forceinline__ unsigned long long mesh_block_scan(unsigned long long x,
                                                             unsigned long long *total) {
    __shared__ unsigned long long wsum[kTileBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    unsigned long long incl = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const unsigned long long y = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += y;
    }
    __syncthreads();
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    unsigned long long before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kTileBlock / kWave; ++w) {
        const unsigned long long t = wsum[w];
        before += w < wid ? t : 0ull;
        all += t;
    }
    *total = all;
    return before + incl - x;
}

__device__ __forceinline__ int popc2(int c) { return (c & 1) + ((c >> 1) & 1); }

constexpr int kEmitQ = 4;                        // consecutive quads per thread
constexpr int kEmitChunk = kEmitQ * kTileBlock;  // quads per pass
constexpr unsigned long long kField = (1ull << 21) - 1;

// Cooperative copy of `count` staged ints to global memory: consecutive
// lanes write consecutive words, so every store instruction is coalesced.
__device__ __forceinline__ void emit_flush(const int *stage, int32_t *__restrict__ dst, int count) {
    __syncthreads();
    for (int k = threadIdx.x; k < count; k += kTileBlock) st_stream(&dst[k], stage[k]);
    __syncthreads();
}

// T_map, T and HE of quad row u.  The row's place in T is the sum of the
// counts of the rows above it; the codes of rows u-1 and u+1 give the
// indices of the Top and Bottom twins.  Each thread owns four consecutive
// quads of a 1024-quad pass (one block scan per pass, serial prefix inside
// the thread).  A thread's outputs are strided in memory (up to 96 bytes per
// lane), so each of the pass's three contiguous output ranges -- its T_map
// entries, its rows of T, its rows of HE -- is assembled in LDS and then
// written with coalesced stores.  The last row writes |T|.
struct MeshEmitRowLds {
    int stage[3 * 2 * kEmitChunk];
};

__device__ __forceinline__ void mesh_emit_row(const uint8_t *__restrict__ codes,
                                              const int *__restrict__ row_count, int Mq, int N,
                                              int u, int32_t *__restrict__ tri_map,
                                              int32_t *__restrict__ tris,
                                              int32_t *__restrict__ he, int cap,
                                              int32_t *__restrict__ n_tri, MeshEmitRowLds &L) {
    __shared__ int red[kTileBlock / kWave];
    int *stage = L.stage;
    const int Nq = N - 1;
    const uint8_t *cr0 = codes + (size_t)u * Nq;
    const uint8_t *crm = u > 0 ? cr0 - Nq : cr0;        // row u-1
    const uint8_t *crp = u + 1 < Mq ? cr0 + Nq : cr0;   // row u+1
    int above = 0;
    for (int r = threadIdx.x; r < u - 1; r += kTileBlock) above += row_count[r];
    above = wave_sum(above);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = above;
    __syncthreads();
    int basem = 0;
#pragma unroll
    for (int w = 0; w < kTileBlock / kWave; ++w) basem += red[w];
    const int base0 = basem + (u > 0 ? row_count[u - 1] : 0);
    const int basep = base0 + row_count[u];
    if (u == Mq - 1 && threadIdx.x == 0) *n_tri = basep;
    int carry0 = 0, carrym = 0, carryp = 0;
    for (int v0 = 0; v0 < Nq; v0 += kEmitChunk) {
        const int vb = v0 + kEmitQ * threadIdx.x;
        int c0[kEmitQ], cm[kEmitQ], cp[kEmitQ];
        int t0 = 0, tm = 0, tp = 0;
#pragma unroll
        for (int j = 0; j < kEmitQ; ++j) {
            const int v = vb + j;
            const bool in = v < Nq;
            c0[j] = in ? cr0[v] : 0;
            cm[j] = (in && u > 0) ? crm[v] : 0;
            cp[j] = (in && u + 1 < Mq) ? crp[v] : 0;
            t0 += popc2(c0[j]);
            tm += popc2(cm[j]);
            tp += popc2(cp[j]);
        }
        const int cl_first = (vb > 0 && vb - 1 < Nq) ? cr0[vb - 1] : 0;
        const int cr_last = vb + kEmitQ < Nq ? cr0[vb + kEmitQ] : 0;
        unsigned long long total;
        const unsigned long long ex = mesh_block_scan(
            (unsigned long long)t0 | ((unsigned long long)tm << 21) | ((unsigned long long)tp << 42),
            &total);
        const int pass0 = base0 + carry0;                    // first triangle of this pass
        const int r00 = pass0 + (int)(ex & kField);          // this thread's first triangle
        const int rm0 = basem + carrym + (int)((ex >> 21) & kField);
        const int rp0 = basep + carryp + (int)((ex >> 42) & kField);
        const int nq = min(kEmitChunk, Nq - v0);              // quads in this pass
        const int nt = (int)(total & kField);                 // triangles in this pass
        const int nw = max(0, min(nt, cap - pass0));          // of them below cap

        // T_map: two entries per quad, -1 for an invalid triangle
        {
            int r0 = r00;
#pragma unroll
            for (int j = 0; j < kEmitQ; ++j) {
                const int v = vb + j;
                if (v < Nq) {
                    const int f = c0[j] & 1, s = (c0[j] >> 1) & 1;
                    stage[2 * (v - v0)] = f ? r0 : -1;
                    stage[2 * (v - v0) + 1] = s ? r0 + f : -1;
                }
                r0 += popc2(c0[j]);
            }
            emit_flush(stage, tri_map + 2 * ((size_t)u * Nq + v0), 2 * nq);
        }
        // T: first triangle (p3, p2, p1), second (p1, p4, p3)
        {
            int r0 = r00;
#pragma unroll
            for (int j = 0; j < kEmitQ; ++j) {
                const int v = vb + j;
                const int f = c0[j] & 1, s = (c0[j] >> 1) & 1;
                const int i1 = u * N + v, i2 = i1 + 1, i3 = i1 + N + 1, i4 = i1 + N;
                const int a = 3 * (r0 - pass0);
                if (f) { stage[a] = i3; stage[a + 1] = i2; stage[a + 2] = i1; }
                if (s) { stage[a + 3 * f] = i1; stage[a + 3 * f + 1] = i4; stage[a + 3 * f + 2] = i3; }
                r0 += f + s;
            }
            emit_flush(stage, tris + 3 * (size_t)pass0, 3 * nw);
        }
        // HE: Right = (u, v+1, 1), Top = (u-1, v, 1), Left = (u, v-1, 0),
        // Bottom = (u+1, v, 0); twin indices from the running prefix sums
        if (he) {
            int r0 = r00, rm = rm0, rp = rp0;
#pragma unroll
            for (int j = 0; j < kEmitQ; ++j) {
                const int f = c0[j] & 1, s = (c0[j] >> 1) & 1;
                const int cr = j + 1 < kEmitQ ? c0[j + 1] : cr_last;
                const int cl = j > 0 ? c0[j - 1] : cl_first;
                const int right = (cr & 2) ? r0 + f + s + (cr & 1) : -1;
                const int left = (cl & 1) ? r0 - popc2(cl) : -1;
                const int top = (cm[j] & 2) ? rm + (cm[j] & 1) : -1;
                const int bottom = (cp[j] & 1) ? rp : -1;
                const int rF = r0, rS = r0 + f;
                const int a = 3 * (r0 - pass0);
                if (f) {
                    stage[a] = right >= 0 ? 3 * right : -1;
                    stage[a + 1] = top >= 0 ? 3 * top + 1 : -1;
                    stage[a + 2] = s ? 3 * rS + 2 : -1;
                }
                if (s) {
                    stage[a + 3 * f] = left >= 0 ? 3 * left : -1;
                    stage[a + 3 * f + 1] = bottom >= 0 ? 3 * bottom + 1 : -1;
                    stage[a + 3 * f + 2] = f ? 3 * rF + 2 : -1;
                }
                r0 += f + s;
                rm += popc2(cm[j]);
                rp += popc2(cp[j]);
            }
            emit_flush(stage, he + 3 * (size_t)pass0, 3 * nw);
        }
        carry0 += nt;
        carrym += (int)((total >> 21) & kField);
        carryp += (int)((total >> 42) & kField);
    }
}

// ---------------------------------------------------------------------------
// The same mesh over row segments of kMeshSeg quads, one quad per thread (the
// single-frame kernels): a 480x640 frame is then 1,437 workgroups instead of
// 479 rows, enough waves to cover the memory latency of these two short
// stages.  Segment s of quad row u covers columns [s kMeshSeg, (s+1) kMeshSeg)
// of every row alike, so with segments numbered row-major (k = u S + s, S
// segments per row) the first triangle of segment k is the sum of the counts
// of segments 0 .. k-1, and the twins in rows u-1 and u+1 start at the same
// sums for k - S and k + S.  The outputs equal the whole-row bodies' above.
// ---------------------------------------------------------------------------

constexpr int kMeshSeg = kTileBlock;
constexpr int kMeshSegMax = 8192;    // segments per frame up to which the segment bodies are used

__host__ __device__ constexpr int mesh_segments(int Nq) { return (Nq + kMeshSeg - 1) / kMeshSeg; }

// Validity codes of segment s of quad row u and its triangle count
// seg_count[u S + s].
struct MeshCountSegLds {
    uint8_t ok[2][kMeshSeg + 1];
};

__device__ __forceinline__ void mesh_count_seg(const float *__restrict__ pts, int N, int u, int s,
                                               int S, uint8_t *__restrict__ codes,
                                               uint8_t *__restrict__ tri_valid,
                                               int *__restrict__ seg_count, MeshCountSegLds &L) {
    auto &ok = L.ok;
    __shared__ int red[kTileBlock / kWave];
    const int Nq = N - 1;
    const int v0 = s * kMeshSeg;
    const float *r0 = pts + (size_t)u * N * 3;
    const float *r1 = r0 + (size_t)N * 3;
    // points v0 .. v0 + kMeshSeg of both rows (the last one by thread 0),
    // all loads issued before any is used
    float x[2][2], y[2][2], z[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int v = v0 + (int)threadIdx.x + j * kMeshSeg;
        const bool in = (j == 0 || threadIdx.x == 0) && v < N;
        x[0][j] = in ? r0[3 * v] : 0.f; y[0][j] = in ? r0[3 * v + 1] : 0.f; z[0][j] = in ? r0[3 * v + 2] : 0.f;
        x[1][j] = in ? r1[3 * v] : 0.f; y[1][j] = in ? r1[3 * v + 1] : 0.f; z[1][j] = in ? r1[3 * v + 2] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        if (j == 0 || threadIdx.x == 0) {
#pragma unroll
            for (int r = 0; r < 2; ++r)
                ok[r][threadIdx.x + j * kMeshSeg] =
                    !(is_nan_bits(x[r][j]) || is_nan_bits(y[r][j]) || is_nan_bits(z[r][j]));
        }
    }
    __syncthreads();
    const int v = v0 + (int)threadIdx.x;
    int cnt = 0;
    if (v < Nq) {
        const int l = threadIdx.x;
        const int p1 = ok[0][l], p2 = ok[0][l + 1], p3 = ok[1][l + 1], p4 = ok[1][l];
        const int f = p1 & p2 & p3;          // first triangle (p3, p2, p1)
        const int g = p1 & p3 & p4;          // second triangle (p1, p4, p3)
        const size_t q = (size_t)u * Nq + v;
        codes[q] = (uint8_t)(f | (g << 1));
        if (tri_valid) {
            tri_valid[2 * q] = (uint8_t)f;
            tri_valid[2 * q + 1] = (uint8_t)g;
        }
        cnt = f + g;
    }
    cnt = wave_sum(cnt);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
#pragma unroll
        for (int w = 0; w < kTileBlock / kWave; ++w) t += red[w];
        seg_count[u * S + s] = t;
    }
}

// T_map, T and HE of segment s of quad row u (the whole-row emit restricted
// to one quad per thread; see mesh_emit_row for the twin rules).  The last
// segment of the last row writes |T|.
struct MeshEmitSegLds {
    int stage[3 * 2 * kMeshSeg];
};

__device__ __forceinline__ void mesh_emit_seg(const uint8_t *__restrict__ codes,
                                              const int *__restrict__ seg_count, int Mq, int N,
                                              int u, int s, int S, int32_t *__restrict__ tri_map,
                                              int32_t *__restrict__ tris,
                                              int32_t *__restrict__ he, int cap,
                                              int32_t *__restrict__ n_tri, MeshEmitSegLds &L) {
    __shared__ int red[kTileBlock / kWave];
    int *stage = L.stage;
    const int Nq = N - 1;
    const int v0 = s * kMeshSeg;
    const int ku = u * S + s;                 // this segment
    const int lo = u > 0 ? ku - S : ku;       // the first of the segments above and here
    int a = 0;
    for (int k = threadIdx.x; k < lo; k += kTileBlock) a += seg_count[k];
    a = wave_sum(a);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = a;
    __syncthreads();
    int sum_lo = 0;
#pragma unroll
    for (int w = 0; w < kTileBlock / kWave; ++w) sum_lo += red[w];
    const int basem = sum_lo;                 // first triangle of segment ku - S (u > 0)
    int base0 = sum_lo;                       // first triangle of this segment
    if (u > 0)
        for (int k = ku - S; k < ku; ++k) base0 += seg_count[k];
    int basep = base0;                        // first triangle of segment ku + S
    if (u + 1 < Mq)
        for (int k = ku; k < ku + S; ++k) basep += seg_count[k];
    if (u == Mq - 1 && s == S - 1 && threadIdx.x == 0) *n_tri = base0 + seg_count[ku];

    const uint8_t *cr0 = codes + (size_t)u * Nq;
    const int v = v0 + (int)threadIdx.x;
    const bool in = v < Nq;
    const int c0 = in ? cr0[v] : 0;
    const int cm = (in && u > 0) ? cr0[v - Nq] : 0;
    const int cp = (in && u + 1 < Mq) ? cr0[v + Nq] : 0;
    const int cl = (in && v > 0) ? cr0[v - 1] : 0;
    const int cr = v + 1 < Nq ? cr0[v + 1] : 0;
    unsigned long long total;
    const unsigned long long ex = mesh_block_scan(
        (unsigned long long)popc2(c0) | ((unsigned long long)popc2(cm) << 21) |
            ((unsigned long long)popc2(cp) << 42),
        &total);
    const int r0 = base0 + (int)(ex & kField);           // this quad's first triangle
    const int rm = basem + (int)((ex >> 21) & kField);
    const int rp = basep + (int)((ex >> 42) & kField);
    const int nq = min(kMeshSeg, Nq - v0);                // quads in this segment
    const int nt = (int)(total & kField);                 // triangles in this segment
    const int nw = max(0, min(nt, cap - base0));          // of them below cap
    const int f = c0 & 1, g = (c0 >> 1) & 1;

    // T_map: two entries per quad, -1 for an invalid triangle
    if (in) {
        stage[2 * threadIdx.x] = f ? r0 : -1;
        stage[2 * threadIdx.x + 1] = g ? r0 + f : -1;
    }
    emit_flush(stage, tri_map + 2 * ((size_t)u * Nq + v0), 2 * nq);
    // T: first triangle (p3, p2, p1), second (p1, p4, p3)
    {
        const int i1 = u * N + v, i2 = i1 + 1, i3 = i1 + N + 1, i4 = i1 + N;
        const int at = 3 * (r0 - base0);
        if (f) { stage[at] = i3; stage[at + 1] = i2; stage[at + 2] = i1; }
        if (g) { stage[at + 3 * f] = i1; stage[at + 3 * f + 1] = i4; stage[at + 3 * f + 2] = i3; }
        emit_flush(stage, tris + 3 * (size_t)base0, 3 * nw);
    }
    // HE: Right = (u, v+1, 1), Top = (u-1, v, 1), Left = (u, v-1, 0),
    // Bottom = (u+1, v, 0)
    if (he) {
        const int right = (cr & 2) ? r0 + f + g + (cr & 1) : -1;
        const int left = (cl & 1) ? r0 - popc2(cl) : -1;
        const int top = (cm & 2) ? rm + (cm & 1) : -1;
        const int bottom = (cp & 1) ? rp : -1;
        const int at = 3 * (r0 - base0);
        if (f) {
            stage[at] = right >= 0 ? 3 * right : -1;
            stage[at + 1] = top >= 0 ? 3 * top + 1 : -1;
            stage[at + 2] = g ? 3 * (r0 + f) + 2 : -1;
        }
        if (g) {
            stage[at + 3 * f] = left >= 0 ? 3 * left : -1;
            stage[at + 3 * f + 1] = bottom >= 0 ? 3 * bottom + 1 : -1;
            stage[at + 3 * f + 2] = f ? 3 * r0 + 2 : -1;
        }
        emit_flush(stage, he + 3 * (size_t)base0, 3 * nw);
    }
}

// ---------------------------------------------------------------------------
// Laplacian (Sec. 2.3 Eqs. 1-2 on the image neighbourhood of Sec. 5.1):
// F Jacobi sweeps of one TH x TW tile, temporally blocked in LDS.
//
// The tile plus a halo of R*F pixels is staged as float4 (x, y, z, pad);
// sweep f updates the region that is still exact after f steps (shrinking by
// R per side) between two LDS buffers, and the centre is written back.
// Invalid pixels (any NaN coordinate) and pixels outside the image are staged
// as (0, 0, 0, +inf): the pad makes the squared distance +inf, whose
// reciprocal square root is exactly 0, so they drop out of both sums without
// a branch.  Pixels of the border band are staged with pad -0.0, which adds
// nothing to a distance: they are neighbours like any other, but only a +0.0
// pad (bits all zero) marks a pixel that is updated.  Invalid pixels and the
// border band are never updated; invalid pixels are written back from the
// input bits.  F = 0 copies the tile.
// LDS: 2 * (TH + 2RF) * (TW + 2RF) float4.
// ---------------------------------------------------------------------------

__host__ __device__ constexpr size_t lap_lds_bytes(int R, int F, int TH, int TW) {
    return 2 * sizeof(float4) * (size_t)(TH + 2 * R * F) * (size_t)(TW + 2 * R * F);
}

template <int R>
__device__ __forceinline__ void lap_tile(const float *__restrict__ src, float *__restrict__ dst,
                                         int M, int N, float lam, int F, int TH, int TW,
                                         int ty0, int tx0, float4 *lds) {
    const int halo = R * F;
    const int H = TH + 2 * halo, W = TW + 2 * halo;
    float4 *A = lds;
    float4 *B = lds + H * W;
    const int oy = ty0 - halo, ox = tx0 - halo;
    const float inf = __builtin_inff();

    const DivBy byW(W);
    for (int idx = threadIdx.x; idx < H * W; idx += kTileBlock) {
        const int ly = byW.div(idx), lx = idx - ly * W;
        const int gy = oy + ly, gx = ox + lx;
        float4 p = make_float4(0.f, 0.f, 0.f, inf);
        if (gy >= 0 && gy < M && gx >= 0 && gx < N) {
            const float *q = src + 3 * ((size_t)gy * N + gx);
            const float x = q[0], y = q[1], z = q[2];
            const bool inner = gy >= R && gy < M - R && gx >= R && gx < N - R;
            if (!(is_nan_bits(x) || is_nan_bits(y) || is_nan_bits(z)))
                p = make_float4(x, y, z, inner ? 0.f : -0.f);
        }
        A[idx] = p;
    }
    __syncthreads();

    for (int f = 1; f <= F; ++f) {
        const int lo = R * f;
        const int Hf = H - 2 * lo, Wf = W - 2 * lo;
        const DivBy byWf(Wf);
        for (int idx = threadIdx.x; idx < Hf * Wf; idx += kTileBlock) {
            const int ry = byWf.div(idx);
            const int ly = lo + ry, lx = lo + (idx - ry * Wf);
            const float4 c = A[ly * W + lx];
            float4 o = c;
            const bool active = __float_as_uint(c.w) == 0u;   // valid, not in the border band
            if (active) {
                float ws = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
                // The weighted sums; with `skip` set, coincident neighbours
                // (d2 = 0, weight 1/0) are left out.  Without the test such a neighbour makes ws
                // infinite -- nothing else can, every other weight being at
                // most 1/sqrt(the smallest float) -- so the point is summed
                // again with it (rare: duplicated points), and every result
                // is the same as with the test throughout.
                auto sums = [&](auto skip) {
                    ws = 0.f; sx = 0.f; sy = 0.f; sz = 0.f;
                    // 3x3: fully unrolled; larger windows: one row of the
                    // window per iteration, so only that row's neighbours are live
                    constexpr int kRowUnroll = R == 1 ? 3 : 1;
#pragma unroll kRowUnroll
                    for (int dy = -R; dy <= R; ++dy) {
#pragma unroll
                        for (int dx = -R; dx <= R; ++dx) {
                            if (dy == 0 && dx == 0) continue;
                            const float4 p = A[(ly + dy) * W + lx + dx];
                            const float ex = p.x - c.x, ey = p.y - c.y, ez = p.z - c.z;
                            const float d2 = fmaf(ex, ex, fmaf(ey, ey, fmaf(ez, ez, p.w)));
                            float w = __builtin_amdgcn_rsqf(d2);     // 1/||v_j - v_i||
                            if constexpr (decltype(skip)::value) w = d2 > 0.f ? w : 0.f;
                            ws += w;
                            sx = fmaf(w, ex, sx);
                            sy = fmaf(w, ey, sy);
                            sz = fmaf(w, ez, sz);
                        }
                    }
                };
                sums(std::false_type{});
                if (!(ws < inf)) sums(std::true_type{});
                if (ws > 0.f) {
                    const float k = lam * __builtin_amdgcn_rcpf(ws);
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

    const DivBy byTW(TW);
    for (int idx = threadIdx.x; idx < TH * TW; idx += kTileBlock) {
        const int ry = byTW.div(idx), rx = idx - ry * TW;
        const int gy = ty0 + ry, gx = tx0 + rx;
        if (gy >= M || gx >= N) continue;
        const size_t off = 3 * ((size_t)gy * N + gx);
        const float4 c = A[(ry + halo) * W + rx + halo];
        if (c.w == 0.f) {                   // +0 or -0: a valid pixel
            dst[off] = c.x; dst[off + 1] = c.y; dst[off + 2] = c.z;
        } else {
            dst[off] = src[off]; dst[off + 1] = src[off + 1]; dst[off + 2] = src[off + 2];
        }
    }
    __syncthreads();                 // LDS is reused by the next tile
}

// ---------------------------------------------------------------------------
// Triangle centroids and normals (Sec. 5.2) of one quad.
// ---------------------------------------------------------------------------

struct V3 {
    float x, y, z;
};

__device__ __forceinline__ bool ok3(const V3 &a) {
    return !(is_nan_bits(a.x) || is_nan_bits(a.y) || is_nan_bits(a.z));
}

// centroid (a + b + c) / 3 and unit normal of (b - a) x (c - a); NaN normal
// when the cross product vanishes.
__device__ __forceinline__ void tri_geom(const V3 &a, const V3 &b, const V3 &c, V3 &cen, V3 &nrm) {
    const float third = 1.0f / 3.0f;
    cen.x = (a.x + b.x + c.x) * third;
    cen.y = (a.y + b.y + c.y) * third;
    cen.z = (a.z + b.z + c.z) * third;
    const float e1x = b.x - a.x, e1y = b.y - a.y, e1z = b.z - a.z;
    const float e2x = c.x - a.x, e2y = c.y - a.y, e2z = c.z - a.z;
    // two rounded products and a difference (contraction is off, so the same
    // bits wherever this is inlined): when two corners coincide the edges are
    // equal and the products cancel exactly, so a zero-area triangle gets a
    // zero cross product and a NaN normal.  A fused form would leave the
    // rounding error of one product there instead.
    const float nx = e1y * e2z - e1z * e2y;
    const float ny = e1z * e2x - e1x * e2z;
    const float nz = e1x * e2y - e1y * e2x;
    const float l2 = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
    if (l2 > 0.f) {
        const float k = __builtin_amdgcn_rsqf(l2);
        nrm = V3{nx * k, ny * k, nz * k};
    } else {
        nrm = V3{qnan(), qnan(), qnan()};
    }
}

// Centroids and normals of both triangles of a quad with corners p1 = (u, v),
// p2 = (u, v+1), p3 = (u+1, v+1), p4 = (u+1, v); NaN for a missing triangle.
__device__ __forceinline__ void quad_geom(const V3 &p1, const V3 &p2, const V3 &p3, const V3 &p4,
                                          V3 &c0, V3 &n0, V3 &c1, V3 &n1) {
    const bool v1 = ok3(p1), v2 = ok3(p2), v3 = ok3(p3), v4 = ok3(p4);
    const V3 nan3{qnan(), qnan(), qnan()};
    c0 = nan3; n0 = nan3; c1 = nan3; n1 = nan3;
    if (v1 & v2 & v3) tri_geom(p3, p2, p1, c0, n0);     // first triangle
    if (v1 & v3 & v4) tri_geom(p1, p4, p3, c1, n1);     // second triangle
}

// Quad (qy, qx) of a frame with N points per row: centroids and normals.
__device__ __forceinline__ void quad_geom_at(const float *__restrict__ pts, int N, int qy, int qx,
                                             V3 &c0, V3 &n0, V3 &c1, V3 &n1) {
    const float *r0 = pts + 3 * ((size_t)qy * N + qx);
    const float *r1 = r0 + 3 * (size_t)N;
    quad_geom(V3{r0[0], r0[1], r0[2]}, V3{r0[3], r0[4], r0[5]}, V3{r1[3], r1[4], r1[5]},
              V3{r1[0], r1[1], r1[2]}, c0, n0, c1, n1);
}

// Up to kTileBlock consecutive quads [q0, q0 + nq), one per thread, q0 a
// multiple of kTileBlock.  Quad q = (u, v) has its top corners at point
// index q + u, so the block's top corners are one contiguous run of points
// and its bottom corners the run N points further; both runs are read with
// coalesced word loads into LDS (at most 2 kTileBlock points each, reached
// only when N = 2).  A quad's outputs (6 centroid floats, 6 normals) would be
// 24-byte strided per thread, so both are assembled in the same LDS and
// written with coalesced 8-byte (float32) or 4-byte (float16 pairs) stores.
struct NormalsStage {
    float f[2][3 * 2 * kTileBlock];
};

template <typename NT>
__device__ __forceinline__ void normals_block(const float *__restrict__ pts, int N, int Nq, size_t q0,
                                              int nq, NT *__restrict__ normals,
                                              float *__restrict__ centroids, NormalsStage &st) {
    // 6 Q < 2^31 (shape check): 32-bit index arithmetic
    const unsigned ua = (unsigned)q0 / (unsigned)Nq, ub = ((unsigned)q0 + nq - 1) / (unsigned)Nq;
    const size_t P0 = q0 + ua;                              // top-left corner of quad q0
    const int L = (int)(nq + 1 + (ub - ua));                // points per run
    const float *top = pts + 3 * P0, *bot = top + 3 * (size_t)N;
    constexpr int kLoads = 3 * 2 * kTileBlock / kTileBlock;   // all in flight at once
    float wt[kLoads], wb[kLoads];
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
        const int k = j * kTileBlock + threadIdx.x;
        wt[j] = k < 3 * L ? top[k] : 0.f;
        wb[j] = k < 3 * L ? bot[k] : 0.f;
    }
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
        const int k = j * kTileBlock + threadIdx.x;
        if (k < 3 * L) {
            st.f[0][k] = wt[j];
            st.f[1][k] = wb[j];
        }
    }
    __syncthreads();
    V3 c0, n0, c1, n1;
    if ((int)threadIdx.x < nq) {
        const unsigned q = (unsigned)q0 + threadIdx.x;
        const int o = 3 * (int)(q + q / (unsigned)Nq - (unsigned)P0);
        const float *t = st.f[0] + o, *b = st.f[1] + o;
        quad_geom(V3{t[0], t[1], t[2]}, V3{t[3], t[4], t[5]}, V3{b[3], b[4], b[5]},
                  V3{b[0], b[1], b[2]}, c0, n0, c1, n1);
    }
    __syncthreads();
    if ((int)threadIdx.x < nq) {
        float *co = st.f[0] + 6 * threadIdx.x;
        co[0] = c0.x; co[1] = c0.y; co[2] = c0.z;
        co[3] = c1.x; co[4] = c1.y; co[5] = c1.z;
        NT *no = reinterpret_cast<NT *>(st.f[1]) + 6 * threadIdx.x;
        st_f(no + 0, n0.x); st_f(no + 1, n0.y); st_f(no + 2, n0.z);
        st_f(no + 3, n1.x); st_f(no + 4, n1.y); st_f(no + 5, n1.z);
    }
    __syncthreads();
    float *gc = centroids + 6 * q0;
    for (int k = threadIdx.x; k < 3 * nq; k += kTileBlock)
        st_stream2(gc + 2 * k, st.f[0][2 * k], st.f[0][2 * k + 1]);
    if (sizeof(NT) == 4) {
        float *g = reinterpret_cast<float *>(normals + 6 * q0);
        for (int k = threadIdx.x; k < 3 * nq; k += kTileBlock)
            st_stream2(g + 2 * k, st.f[1][2 * k], st.f[1][2 * k + 1]);
    } else {
        const uint32_t *s1 = reinterpret_cast<const uint32_t *>(st.f[1]);
        uint32_t *g1 = reinterpret_cast<uint32_t *>(normals + 6 * q0);
        for (int k = threadIdx.x; k < 3 * nq; k += kTileBlock) st_stream(&g1[k], s1[k]);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Bilateral normal filter (Sec. 2.3 Eqs. 3-6; neighbourhood of Sec. 5.2):
// F Jacobi sweeps of one TQH x TQW tile of quads, temporally blocked in LDS.
//
// A thread owns a quad and filters both of its triangles, which share every
// neighbour load (the paper's unit of work).  With log2(e) folded into
//     ka = log2(e) / (2 sigma_l^2),  kb = log2(e) / (2 sigma_a^2),
// a neighbour's weight is w = 2^-e, e = ka ||c_i - c_j||^2 + kb ||n_i - n_j||^2.
// Both squared distances come from component differences (exact for nearby
// float32 values) before scaling; expanding them or pre-scaling the
// centroids saves instructions but costs ~1e-5 relative weight accuracy.
//
// Eq. 6 renormalises, so a common factor of the weights cancels: every
// weight is taken as w = 2^(48 - e) (the same value in exact arithmetic).
// The shift is a constant, so a pair's weight does not depend on which of
// its triangles is being filtered; with e >= 0 no weight exceeds 2^48, which
// keeps the sums and the squared norm of Eq. 6 finite for windows up to
// 9 x 9 (160 neighbours), and terms down to e = 174 stay normal floats.  If
// the weighted sum of normals drops below 2^-60 in norm (always when every
// neighbour is at e > 108; otherwise only where the normals nearly cancel),
// that triangle is recomputed with every exponent shifted by the smallest
// one, which puts the largest term at 1.
// Such triangles are isolated ones (about 7 per thousand on the LiDAR
// frames, 4 per 10^4 on the RGB-D ones), so instead of the lane
// redoing its window alone -- which held up its whole wave -- the lane
// queues the triangle in LDS, and after the sweep one wave per queued
// triangle takes its neighbours over the wave's lanes: the smallest exponent
// by a wave minimum, then the shifted weights and weighted normals summed
// over the lanes in a fixed tree.  The result depends on the triangle's
// window only, not on the tile.
//
// Summation order.  The window's displacements split into D+ (dy = 0 and
// dx > 0, or dy > 0) and their negatives; a triangle sums its terms in a
// fixed order: for each d of D+, the two triangles of quad a+d, then the two
// of quad a-d.  The order is the same for every tile shape and fusion depth,
// so float32 results are too.
//
// Off-grid quads and triangles with a NaN normal or centroid are staged with
// an infinite centroid and a zero normal: infinite exponent, weight exactly 0,
// contribution 0.  A triangle that is itself missing is copied through (its
// input bits).  Float16-stored normals produced by an intermediate sweep are
// re-rounded to float16, as if stored between launches, so results do not
// depend on F.  F = 0 copies the tile (and gathers).
// LDS: (TQH + 2RF) * (TQW + 2RF) float4 times 4 (centroids and normals of
// both triangles) or, with F > 1, times 6 (a second normal buffer), and the
// queue of underflowed triangles (one int per triangle of the region, and
// its count).
// ---------------------------------------------------------------------------

constexpr float kBilUnderflow2 = 0x1p-120f;       // (2^-60)^2
// register budget of the bilateral kernels: at least 6 waves per SIMD
// (<= 80 VGPRs), more than the LDS of a typical tile lets reside anyway
constexpr int kBilWavesPerSimd = 6;
constexpr float kBilShift = 48.f;                 // every weight is 2^(48 - e)
constexpr int kBilMaxSweeps = 8;                  // fused sweeps per launch at most
#ifndef PL_BIL_PARTS_K3
#define PL_BIL_PARTS_K3 1
#endif
#ifndef PL_BIL_PARTS_K5
#define PL_BIL_PARTS_K5 4
#endif
#ifndef PL_BIL_FRAME_WAVES
#define PL_BIL_FRAME_WAVES 1
#endif
#ifndef PL_BIL_BATCH_WAVES
#define PL_BIL_BATCH_WAVES 0
#endif
// Whether a kernel runs the parts of a quad's sum on its waves (windows of
// 5x5 and up): the single-frame kernels do, the batched ones (many rounds
// of workgroups deep, where wave 0 closing the quads alone idles the others)
// keep them on lanes.
__host__ __device__ constexpr bool bil_waves(int R, bool batch) {
    return R >= 2 && (batch ? PL_BIL_BATCH_WAVES : PL_BIL_FRAME_WAVES) != 0;
}
// floats of the parts' exchange when the parts run on waves: the partial
// sums of parts 1.. of 64 quads
__host__ __device__ constexpr int bil_xch_floats(int R) {
    return R >= 2 ? (PL_BIL_PARTS_K5 - 1) * 6 * 64 : 0;
}
__host__ __device__ constexpr size_t bil_lds_bytes(int R, int F, int TQH, int TQW, bool waves) {
    return (F > 1 ? 6 : 4) * sizeof(float4) * (size_t)(TQH + 2 * R * F) * (size_t)(TQW + 2 * R * F) +
           sizeof(int) * (2 * (size_t)(TQH + 2 * R * F) * (size_t)(TQW + 2 * R * F) + kBilMaxSweeps + 1) +
           sizeof(int) * (size_t)TQH * TQW +    // T ranks of the tile (gather from the mesh codes)
           (waves ? sizeof(float) * (size_t)bil_xch_floats(R) : 0);
}

// The mesh's codes and per-segment counts (pl_mesh_opc's first pass): with
// them the gather finds each triangle's place in T itself instead of reading
// T_map, so the pass can run in the same launch as the mesh emit.
struct GatherCodes {
    const uint8_t *codes;       // [Mq][Nq] validity codes (bit k: triangle k)
    const int *seg_count;       // [Mq][S] valid triangles per row segment
    int S;                      // segments per quad row (mesh_segments(Nq))
};

// Output stores of the filter: streaming for float32 normals, plain for
// float16 (measured on float32 only).
__device__ __forceinline__ void bil_store(float *p, float v) { st_stream(p, v); }
__device__ __forceinline__ void bil_store(__half *p, __half v) { *p = v; }

template <typename NT> __device__ __forceinline__ float round_storage(float x);
template <> __device__ __forceinline__ float round_storage<float>(float x) { return x; }
template <> __device__ __forceinline__ float round_storage<__half>(float x) {
    return __half2float(__float2half_rn(f32_rounded(x)));
}

struct BilOwn {
    float cx, cy, cz;
    float nx, ny, nz;
    float ka, kb;
};

__device__ __forceinline__ float bil_pair_e(const BilOwn &o, const float4 c, const float4 n) {
    const float ax = o.nx - n.x, ay = o.ny - n.y, az = o.nz - n.z;
    const float dn2 = fmaf(ax, ax, fmaf(ay, ay, az * az));
    const float dx = o.cx - c.x, dy = o.cy - c.y, dz = o.cz - c.z;
    const float dc2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    return fmaf(dc2, o.ka, dn2 * o.kb);
}

// Sum of weighted neighbour normals.  Eq. 6 renormalises it, so the sum of
// the weights is not needed; the underflow test uses the vector's norm,
// which never exceeds the total weight (unit normals).
struct BilAcc {
    float x, y, z;
};

// s += 2^(m - e) * n
__device__ __forceinline__ void bil_add(BilAcc &s, float m, float e, const float4 n) {
    const float w = __builtin_amdgcn_exp2f(m - e);
    s.x = fmaf(w, n.x, s.x);
    s.y = fmaf(w, n.y, s.y);
    s.z = fmaf(w, n.z, s.z);
}

// The i-th displacement of D+: dy = 0, dx = 1..R, then dy = 1..R, dx = -R..R.
template <int R>
__device__ __forceinline__ void bil_dplus(int i, int &dy, int &dx) {
    if (i < R) {
        dy = 0;
        dx = i + 1;
    } else {
        const int j = i - R;
        dy = 1 + j / (2 * R + 1);
        dx = j % (2 * R + 1) - R;
    }
}
template <int R> constexpr int bil_ndplus() { return 2 * R * R + 2 * R; }

__device__ __forceinline__ float bil_norm2(const BilAcc &s) {
    return fmaf(s.x, s.x, fmaf(s.y, s.y, s.z * s.z));
}

template <typename NT>
__device__ __forceinline__ float4 bil_finish(BilAcc s, float4 cur) {
    const float l2 = bil_norm2(s);
    if (!(l2 > 0.f)) return cur;            // no usable neighbour
    const float k = __builtin_amdgcn_rsqf(l2);
    return make_float4(round_storage<NT>(s.x * k), round_storage<NT>(s.y * k),
                       round_storage<NT>(s.z * k), cur.w);
}

// Weight of a triangle pair (Eqs. 4-5 with log2(e) folded into ka and kb),
// shifted by the constant 2^48: 2^(48 - e).  The value depends on the pair
// only: swapping the triangles changes the sign of every difference exactly
// and none of the squares.  A pair with an off-grid or missing triangle has
// e = +inf and weight 0 (NaN only when both are missing; no sum uses that).
__device__ __forceinline__ float bil_w(const float4 ci, const float4 ni, const float4 cj,
                                       const float4 nj, float ka, float kb) {
    const float ax = ni.x - nj.x, ay = ni.y - nj.y, az = ni.z - nj.z;
    const float dn2 = fmaf(ax, ax, fmaf(ay, ay, az * az));
    const float dx = ci.x - cj.x, dy = ci.y - cj.y, dz = ci.z - cj.z;
    const float dc2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    return __builtin_amdgcn_exp2f(-fmaf(dc2, ka, fmaf(dn2, kb, -kBilShift)));
}

// s += w n
__device__ __forceinline__ void bil_acc(BilAcc &s, float w, const float4 n) {
    s.x = fmaf(w, n.x, s.x);
    s.y = fmaf(w, n.y, s.y);
    s.z = fmaf(w, n.z, s.z);
}

// Eq. 6 for one triangle: a missing one (c.w = 0) is copied through; pend:
// the weighted sum fell below 2^-60 in norm (the triangle goes to the queue
// and r is not set).  Every total weight below 2^-60 is caught, since the
// norm is at most the total weight.
template <typename NT>
__device__ __forceinline__ float4 bil_close(const float4 c, const float4 n, BilAcc s, bool &pend) {
    const bool ok = c.w != 0.f;
    pend = ok && !(bil_norm2(s) >= kBilUnderflow2);
    return ok ? bil_finish<NT>(s, n) : n;
}

__device__ __forceinline__ float wave_min_f(float x) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) x = fminf(x, __shfl_xor(x, m, kWave));
    return x;
}

__device__ __forceinline__ float wave_sum_f(float x) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) x += __shfl_xor(x, m, kWave);
    return x;
}

// The underflowed triangle k of the quad at LDS index a, by one whole wave:
// lane l takes neighbours j = l, l + 64, ... in the main pass's order (j / 4
// the displacement of D+, bit 1 the side, bit 0 the triangle), the shift is
// the smallest exponent (a wave minimum, exact), and the shifted sums are
// added lane by lane in a fixed butterfly.  Every lane returns the result.
template <int R, typename NT>
__device__ __forceinline__ float4 bil_fallback_wave(const float4 *sc, const float4 *sn, int a,
                                                    int k, int pitch, int plane, float ka,
                                                    float kb) {
    constexpr int kN = 4 * bil_ndplus<R>();               // neighbours
    constexpr int kPer = (kN + kWave - 1) / kWave;         // per lane
    const int lane = (int)threadIdx.x & (kWave - 1);
    const float4 c = sc[k * plane + a], n = sn[k * plane + a];
    const BilOwn o{c.x, c.y, c.z, n.x, n.y, n.z, ka, kb};
    const float inf = __builtin_inff();
    float e[kPer];
    float4 nj[kPer];
    float mn = inf;
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
        const int j = lane + t * kWave;
        e[t] = inf;
        nj[t] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j < kN) {
            int dy, dx;
            bil_dplus<R>(j >> 2, dy, dx);
            const int off = dy * pitch + dx;
            const int b = ((j >> 1) & 1) ? a - off : a + off;
            const int kk = j & 1;
            const float4 cj = sc[b + kk * plane];
            nj[t] = sn[b + kk * plane];
            e[t] = bil_pair_e(o, cj, nj[t]);
            mn = fminf(mn, e[t]);
        }
    }
    mn = wave_min_f(mn);
    BilAcc s{0.f, 0.f, 0.f};
    if (mn < inf) {
#pragma unroll
        for (int t = 0; t < kPer; ++t) bil_add(s, mn, e[t], nj[t]);
    }
    s.x = wave_sum_f(s.x);
    s.y = wave_sum_f(s.y);
    s.z = wave_sum_f(s.z);
    return bil_finish<NT>(s, n);
}

// Queue of underflowed triangles in LDS: entries 2 a + k (at most two per
// quad of the staged region, so it cannot overflow) and one count per sweep
// (sweep f counts into count[f], so no count is reset in between).
struct BilQueue {
    int *entry;
    int *count;
};

__device__ __forceinline__ void bil_push(const BilQueue &qu, int a, int k, int sweep) {
    const int i = atomicAdd(&qu.count[sweep], 1);
    qu.entry[i] = 2 * a + k;
}

// Parts per quad: the displacements of D+ are dealt over P parts (part p
// takes i = p, p + P, ...), whose partial sums are then added in a fixed
// tree -- (s_0 + s_1) for P = 2, ((s_0 + s_1) + (s_2 + s_3)) for P = 4 --
// identical on every lane of the quad (addition commutes exactly).  Larger
// windows take more parts: a 5x5 window has 48 neighbours per triangle, and
// a LiDAR frame of 64 x 1024 quads filled only one wave per SIMD at one lane
// per quad.  A kernel runs the P parts on PP lanes (PP dividing P): a lane
// keeps the partial sums of its P / PP parts apart and adds them in the same
// tree, so every kernel gives the same bits whatever its PP.  The single-
// frame kernels put the four parts of a 5x5-and-up quad on the workgroup's
// four waves instead (bil_sweep_waves, same tree again); the batch, many
// rounds deep and bound by VALU issue, runs them on one lane, which needs no
// lane tree and closes and stores each quad once.
template <int R> constexpr int bil_parts() { return R == 1 ? PL_BIL_PARTS_K3 : PL_BIL_PARTS_K5; }
#ifndef PL_BIL_BATCH_LANES_K5
#define PL_BIL_BATCH_LANES_K5 1
#endif
// lanes per quad (0: parts on waves) of the single-frame kernels
template <int R> constexpr int bil_frame_lanes() {
    return bil_waves(R, false) ? 0 : bil_parts<R>();
}
// lanes per quad (0: parts on waves) of the batched kernels
template <int R> constexpr int bil_batch_lanes() {
    return bil_waves(R, true) ? 0 : (R == 1 ? bil_parts<1>() : PL_BIL_BATCH_LANES_K5);
}
static_assert(bil_ndplus<1>() % PL_BIL_PARTS_K3 == 0 && bil_ndplus<2>() % PL_BIL_PARTS_K5 == 0 &&
                  bil_ndplus<3>() % PL_BIL_PARTS_K5 == 0 && bil_ndplus<4>() % PL_BIL_PARTS_K5 == 0,
              "the parts of a quad share |D+| evenly");

// The tree over the P parts of a quad held as P / PP sets on PP lanes (part
// p = lane + k PP is set k): its steps with m < PP add across lanes, the
// rest across sets, each term its own value plus its partner's.
template <int P, int PP>
__device__ __forceinline__ BilAcc bil_reduce(BilAcc (&s)[P / PP]) {
    constexpr int NS = P / PP;
#pragma unroll
    for (int m = 1; m < PP; m <<= 1) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            s[k].x += __shfl_xor(s[k].x, m, kWave);
            s[k].y += __shfl_xor(s[k].y, m, kWave);
            s[k].z += __shfl_xor(s[k].z, m, kWave);
        }
    }
#pragma unroll
    for (int m = 1; m < NS; m <<= 1) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            if (k & m) continue;
            const int o = k ^ m;
            const BilAcc u{s[k].x + s[o].x, s[k].y + s[o].y, s[k].z + s[o].z};
            s[k] = u;
            s[o] = u;
        }
    }
    return s[0];
}

// The terms of the i-th displacement d of D+ for both triangles of the quad
// at LDS index a (own centroids c, normals n): the two triangles of quad
// a + d, then the two of quad a - d.
template <int R>
__device__ __forceinline__ void bil_disp(const float4 *sc, const float4 *sn, int a, int pitch,
                                         int plane, float ka, float kb, int i, const float4 c0,
                                         const float4 c1, const float4 n0, const float4 n1,
                                         BilAcc &s0, BilAcc &s1) {
    int dy, dx;
    bil_dplus<R>(i, dy, dx);
    const int off = dy * pitch + dx;
    const int bp = a + off, bm = a - off;
    const float4 pc0 = sc[bp], pc1 = sc[plane + bp], p0 = sn[bp], p1 = sn[plane + bp];
    const float4 mc0 = sc[bm], mc1 = sc[plane + bm], m0 = sn[bm], m1 = sn[plane + bm];
    bil_acc(s0, bil_w(c0, n0, pc0, p0, ka, kb), p0);
    bil_acc(s0, bil_w(c0, n0, pc1, p1, ka, kb), p1);
    bil_acc(s0, bil_w(mc0, m0, c0, n0, ka, kb), m0);
    bil_acc(s0, bil_w(mc1, m1, c0, n0, ka, kb), m1);
    bil_acc(s1, bil_w(c1, n1, pc0, p0, ka, kb), p0);
    bil_acc(s1, bil_w(c1, n1, pc1, p1, ka, kb), p1);
    bil_acc(s1, bil_w(mc0, m0, c1, n1, ka, kb), m0);
    bil_acc(s1, bil_w(mc1, m1, c1, n1, ka, kb), m1);
}

// Both triangles of the quad at LDS index a, in the fixed summation order:
// for each d of D+ (part p's share of them), the two triangles of quad
// a + d, then the two of quad a - d; the parts' partial sums are added in a
// fixed tree.  This lane (`lane` of PP) runs parts lane, lane + PP, ...: the
// i-th displacement belongs to part i mod P, whose set here is
// (i mod P) / PP.  A pair weight takes its lower quad's triangle first
// (bil_w is symmetric anyway).  Every lane of the quad returns the same r0,
// r1 and pending flags.
template <int R, typename NT, int PP>
__device__ __forceinline__ void bil_sum_quad(const float4 *sc, const float4 *sn, int a,
                                                int pitch, int plane, float ka, float kb,
                                                int lane, float4 &r0, float4 &r1, bool &pend0,
                                                bool &pend1) {
    constexpr int ND = bil_ndplus<R>(), P = bil_parts<R>(), NS = P / PP;
    static_assert(P % PP == 0, "the lanes of a quad share its parts evenly");
    const float4 c0 = sc[a], c1 = sc[plane + a], n0 = sn[a], n1 = sn[plane + a];
    BilAcc s0[NS], s1[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        s0[k] = BilAcc{0.f, 0.f, 0.f};
        s1[k] = BilAcc{0.f, 0.f, 0.f};
    }
#pragma unroll 1
    for (int j0 = 0; j0 < ND / PP; j0 += NS) {
#pragma unroll
        for (int k = 0; k < NS; ++k)            // displacement j0 + k: set k
            bil_disp<R>(sc, sn, a, pitch, plane, ka, kb, (j0 + k) * PP + lane, c0, c1, n0, n1,
                        s0[k], s1[k]);
    }
    r0 = bil_close<NT>(c0, n0, bil_reduce<P, PP>(s0), pend0);
    r1 = bil_close<NT>(c1, n1, bil_reduce<P, PP>(s1), pend1);
}

// One sweep over the OH x OW region at (oy0, ox0) of the staged tile;
// out(ry, rx, a, r0, r1, pend0, pend1) takes each quad's results (ry, rx
// within the region).  Ends with a barrier.
template <int R, typename NT, int PP, typename Out>
__device__ __forceinline__ void bil_sweep(const float4 *sc, const float4 *sn, int pitch, int plane,
                                          int oy0, int ox0, int OH, int OW, float ka, float kb,
                                          Out &&out) {
    const int slot = (int)threadIdx.x / PP, lane = (int)threadIdx.x % PP;
    const DivBy byOW(OW);
    for (int idx = slot; idx < OH * OW; idx += kTileBlock / PP) {
        const int ry = byOW.div(idx), rx = idx - ry * OW;
        const int a = (oy0 + ry) * pitch + ox0 + rx;
        float4 r0, r1;
        bool p0, p1;
        bil_sum_quad<R, NT, PP>(sc, sn, a, pitch, plane, ka, kb, lane, r0, r1, p0, p1);
        out(ry, rx, a, r0, r1, p0, p1);
    }
    __syncthreads();
}

// The same sweep with the P parts of a quad on the workgroup's P waves
// (wave w runs part w of 64 quads at a time): the displacement index is the
// same on every lane of a wave, so its decoding and the neighbour offsets
// are scalar work; waves 1.. leave their partial sums in `xch`, and wave 0
// adds them in the tree of bil_reduce -- ((s_0 + s_1) + (s_2 + s_3)) --
// closes the quad and calls out, alone.  Same bits as the lane form.
template <int R, typename NT, typename Out>
__device__ __forceinline__ void bil_sweep_waves(const float4 *sc, const float4 *sn, int pitch,
                                                int plane, int oy0, int ox0, int OH, int OW,
                                                float ka, float kb, float *xch, Out &&out) {
    constexpr int ND = bil_ndplus<R>(), P = bil_parts<R>();
    static_assert(P == 4 && P == kTileBlock / kWave, "one wave per part, tree of four");
    static_assert(bil_xch_floats(R) == (P - 1) * 6 * kWave, "exchange size");
    const int part = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int lane = (int)threadIdx.x & (kWave - 1);
    const DivBy byOW(OW);
    const int n = OH * OW;
    for (int base = 0; base < n; base += kWave) {
        const int idx = base + lane;
        const bool have = idx < n;
        const int ry = have ? byOW.div(idx) : 0, rx = have ? idx - ry * OW : 0;
        const int a = (oy0 + ry) * pitch + ox0 + rx;
        BilAcc s0{0.f, 0.f, 0.f}, s1{0.f, 0.f, 0.f};
        float4 c0, c1, n0, n1;
        if (have) {
            c0 = sc[a]; c1 = sc[plane + a]; n0 = sn[a]; n1 = sn[plane + a];
#pragma unroll 1
            for (int j = 0; j < ND / P; ++j)
                bil_disp<R>(sc, sn, a, pitch, plane, ka, kb, j * P + part, c0, c1, n0, n1, s0, s1);
        }
        if (part != 0) {
            float *x = xch + (part - 1) * 6 * kWave + lane;
            x[0] = s0.x; x[kWave] = s0.y; x[2 * kWave] = s0.z;
            x[3 * kWave] = s1.x; x[4 * kWave] = s1.y; x[5 * kWave] = s1.z;
        }
        __syncthreads();
        if (part == 0 && have) {
            const float *x1 = xch + lane, *x2 = x1 + 6 * kWave, *x3 = x2 + 6 * kWave;
            const BilAcc t0{(s0.x + x1[0]) + (x2[0] + x3[0]),
                            (s0.y + x1[kWave]) + (x2[kWave] + x3[kWave]),
                            (s0.z + x1[2 * kWave]) + (x2[2 * kWave] + x3[2 * kWave])};
            const BilAcc t1{(s1.x + x1[3 * kWave]) + (x2[3 * kWave] + x3[3 * kWave]),
                            (s1.y + x1[4 * kWave]) + (x2[4 * kWave] + x3[4 * kWave]),
                            (s1.z + x1[5 * kWave]) + (x2[5 * kWave] + x3[5 * kWave])};
            bool p0, p1;
            const float4 r0 = bil_close<NT>(c0, n0, t0, p0);
            const float4 r1 = bil_close<NT>(c1, n1, t1, p1);
            out(ry, rx, a, r0, r1, p0, p1);
        }
        if (base + kWave < n) __syncthreads();   // xch is reused by the next 64 quads
    }
    __syncthreads();
}

// T ranks of a tile's quads for the gather: rank[ty TQW + tx] is the index
// in T of quad (qy0 + ty, qx0 + tx)'s first valid triangle, with the quad's
// code in bits 30..31 (T has fewer than 2^30 triangles).  T is the valid
// triangles in GID order, so the rank is the number of valid triangles in
// the segments before the quad's row segment, plus those before it in its
// segment: each wave takes tile rows, sums the counts of the segments
// before the row's first column and the codes from that segment's start,
// then scans the row.  Quads off the grid get code 0.  No barrier: the
// caller's next one publishes the ranks.
__device__ __forceinline__ void bil_gather_ranks(const GatherCodes &gc, int Mq, int Nq, int qy0,
                                                 int qx0, int TQH, int TQW, int *rank) {
    const int lane = (int)threadIdx.x & (kWave - 1), wave = (int)threadIdx.x / kWave;
    const int s0 = qx0 / kMeshSeg;
    // segments before the tile's first row: the same for every row of it
    const int k0 = qy0 * gc.S;
    int before = 0;
    for (int k = lane; k < k0; k += kWave) before += gc.seg_count[k];
    before = wave_sum(before);
    for (int ty = wave; ty < TQH; ty += kTileBlock / kWave) {
        const int u = qy0 + ty;
        if (u >= Mq) {
            for (int tx = lane; tx < TQW; tx += kWave) rank[ty * TQW + tx] = 0;
            continue;
        }
        const uint8_t *row = gc.codes + (size_t)u * Nq;
        // the rows between, the row's segments before s0, and its codes
        // from the segment's first column up to qx0
        int c = 0;
        for (int k = k0 + lane; k < u * gc.S + s0; k += kWave) c += gc.seg_count[k];
        for (int v = s0 * kMeshSeg + lane; v < qx0; v += kWave) c += popc2(row[v]);
        int run = before + wave_sum(c);
        for (int t0 = 0; t0 < TQW; t0 += kWave) {
            const int tx = t0 + lane, v = qx0 + tx;
            const int code = tx < TQW && v < Nq ? row[v] : 0;
            const int n = popc2(code);
            const int incl = wave_inclusive_scan(n);
            if (tx < TQW) rank[ty * TQW + tx] = (run + incl - n) | (code << 30);
            run += __shfl(incl, kWave - 1, kWave);
        }
    }
}

// FromPts: the raw normals and centroids are not read but computed here from
// the (smoothed) points `pts` exactly as normals_quad computes and stores
// them (normals rounded to NT), and the tile's centroids are written to
// `cen` -- the batched path's first pass, which then needs no normals
// stage.  Otherwise nin / cen are the stored raw normals and centroids.
// PP: lanes per quad for the parts of its sum (bil_parts); 0 puts the parts
// on the workgroup's waves instead (bil_sweep_waves; windows of 5x5 and up).
template <int R, typename NT, bool FromPts = false, bool ByCodes = false, int PP = bil_parts<R>()>
__device__ __forceinline__ void bil_tile(const NT *__restrict__ nin, const float *__restrict__ cen,
                                         NT *__restrict__ nout, int Mq, int Nq, float ka, float kb,
                                         int F, int TQH, int TQW, int qy0, int qx0,
                                         const int32_t *__restrict__ tri_map, NT *__restrict__ nT,
                                         float4 *lds, const float *__restrict__ pts = nullptr,
                                         float *__restrict__ cen_out = nullptr,
                                         GatherCodes gc = GatherCodes{nullptr, nullptr, 0}) {
    const int halo = R * F;
    const int H = TQH + 2 * halo, W = TQW + 2 * halo, S = H * W;
    float4 *s_c = lds;                  // [2][S] centroids, w = 1 if usable
    float4 *s_n = lds + 2 * S;          // [2][S] normals
    float4 *s_m = lds + 4 * S;          // [2][S] second normal buffer (F > 1)
    // queue of underflowed triangles: 2S entries, then one count per sweep
    int *qbase = reinterpret_cast<int *>(lds + (F > 1 ? 6 : 4) * S);
    const BilQueue qu{qbase, qbase + 2 * S};
    if (threadIdx.x < kBilMaxSweeps + 1) qu.count[threadIdx.x] = 0;
    // T ranks of the tile when the gather takes them from the mesh codes
    int *rank = qbase + 2 * S + kBilMaxSweeps + 1;
    // the parts' exchange (parts on waves)
    float *xch = reinterpret_cast<float *>(rank + TQH * TQW);
    constexpr bool waves = PP == 0;
    static_assert(!waves || R >= 2, "parts on waves for windows of 5x5 and up");
    constexpr bool by_codes = ByCodes;
    if constexpr (by_codes) {
        bil_gather_ranks(gc, Mq, Nq, qy0, qx0, TQH, TQW, rank);
        if (F == 0) __syncthreads();
    }
    // index in T of triangle k of tile quad (ty, tx), or -1 (none, or no gather)
    auto t_index = [&](int ty, int tx, size_t q, int k) -> int {
        if constexpr (by_codes) {
            const unsigned r = (unsigned)rank[ty * TQW + tx];
            const int code = (int)(r >> 30), base = (int)(r & 0x3fffffffu);
            if (!((code >> k) & 1)) return -1;
            return base + (k == 1 ? (code & 1) : 0);
        } else {
            return tri_map ? tri_map[2 * q + k] : -1;
        }
    };
    const float inf = __builtin_inff();
    const int oy = qy0 - halo, ox = qx0 - halo;

    if (F > 0) {
        const DivBy byW(W);
        for (int idx = threadIdx.x; idx < S; idx += kTileBlock) {
            const int ly = byW.div(idx), lx = idx - ly * W;
            const int qy = oy + ly, qx = ox + lx;
            float4 c0 = make_float4(inf, inf, inf, 0.f), c1 = c0;
            float4 n0 = make_float4(0.f, 0.f, 0.f, 0.f), n1 = n0;
            if (qy >= 0 && qy < Mq && qx >= 0 && qx < Nq) {
                const size_t q = (size_t)qy * Nq + qx;
                float n[6], c[6];
                if constexpr (FromPts) {
                    V3 g[4];
                    quad_geom_at(pts, Nq + 1, qy, qx, g[0], g[1], g[2], g[3]);
                    c[0] = g[0].x; c[1] = g[0].y; c[2] = g[0].z; c[3] = g[2].x; c[4] = g[2].y; c[5] = g[2].z;
                    n[0] = round_storage<NT>(g[1].x); n[1] = round_storage<NT>(g[1].y);
                    n[2] = round_storage<NT>(g[1].z); n[3] = round_storage<NT>(g[3].x);
                    n[4] = round_storage<NT>(g[3].y); n[5] = round_storage<NT>(g[3].z);
                } else {
#pragma unroll
                    for (int i = 0; i < 6; ++i) { n[i] = ld_f(nin + 6 * q + i); c[i] = cen[6 * q + i]; }
                }
                bool ok0 = true, ok1 = true;
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    ok0 = ok0 && !is_nan_bits(n[i]) && !is_nan_bits(c[i]);
                    ok1 = ok1 && !is_nan_bits(n[3 + i]) && !is_nan_bits(c[3 + i]);
                }
                if (ok0) { c0 = make_float4(c[0], c[1], c[2], 1.f); n0 = make_float4(n[0], n[1], n[2], 0.f); }
                if (ok1) { c1 = make_float4(c[3], c[4], c[5], 1.f); n1 = make_float4(n[3], n[4], n[5], 0.f); }
            }
            s_c[idx] = c0; s_c[S + idx] = c1;
            s_n[idx] = n0; s_n[S + idx] = n1;
        }
        __syncthreads();
    }

    const float4 *cur = s_n;
    float4 *nxt = s_m;
    // PP lanes per quad: quad slot and lane within the quad; parts on
    // waves: the lane is the slot, the wave the part (only part 0 stores)
    constexpr int QL = waves ? 1 : PP;                       // lanes per quad
    const int slot = waves ? (int)threadIdx.x % kWave : (int)threadIdx.x / QL;
    const int part = waves ? (int)threadIdx.x / kWave : (int)threadIdx.x % QL;
    const int wave = (int)threadIdx.x / kWave, lane = (int)threadIdx.x & (kWave - 1);
    // one sweep over the OH x OW region at (o0, o0) of the staged tile
    auto sweep = [&](int o0, int OH, int OW, auto &&out) {
        if constexpr (waves)
            bil_sweep_waves<R, NT>(s_c, cur, W, S, o0, o0, OH, OW, ka, kb, xch, out);
        else
            bil_sweep<R, NT, PP>(s_c, cur, W, S, o0, o0, OH, OW, ka, kb, out);
    };
    // intermediate sweeps: LDS to LDS over the shrinking exact region
    for (int f = 1; f < F; ++f) {
        const int lo = R * f;
        sweep(lo, H - 2 * lo, W - 2 * lo,
              [&](int, int, int a, float4 r0, float4 r1, bool p0, bool p1) {
                  if (part != 0) return;
                  if (p0) bil_push(qu, a, 0, f); else nxt[a] = r0;
                  if (p1) bil_push(qu, a, 1, f); else nxt[S + a] = r1;
              });
        const int nq = qu.count[f];
        for (int e = wave; e < nq; e += kTileBlock / kWave) {
            const int a = qu.entry[e] >> 1, k = qu.entry[e] & 1;
            const float4 r = bil_fallback_wave<R, NT>(s_c, cur, a, k, W, S, ka, kb);
            if (lane == 0) nxt[k * S + a] = r;
        }
        __syncthreads();
        float4 *t = const_cast<float4 *>(cur);
        cur = nxt;
        nxt = t;
    }

    // last sweep (or the copy when F = 0): the tile itself, to global memory
    auto emit = [&](int ty, int tx, int a, float4 r0, float4 r1, bool p0, bool p1) {
        const int qy = qy0 + ty, qx = qx0 + tx;
        if (part != 0 || qy >= Mq || qx >= Nq) return;   // the quad's first lane stores
        const size_t q = (size_t)qy * Nq + qx;
        const float4 r[2] = {r0, r1};
        const bool pend[2] = {p0, p1};
        NT v[6];
        NT raw[6];                           // raw normals as stored (FromPts)
        if constexpr (FromPts) {
            V3 c0, n0, c1, n1;
            quad_geom_at(pts, Nq + 1, qy, qx, c0, n0, c1, n1);
            cen_out[6 * q + 0] = c0.x; cen_out[6 * q + 1] = c0.y; cen_out[6 * q + 2] = c0.z;
            cen_out[6 * q + 3] = c1.x; cen_out[6 * q + 4] = c1.y; cen_out[6 * q + 5] = c1.z;
            st_f(&raw[0], n0.x); st_f(&raw[1], n0.y); st_f(&raw[2], n0.z);
            st_f(&raw[3], n1.x); st_f(&raw[4], n1.y); st_f(&raw[5], n1.z);
        }
        // the stored raw normal i of this quad
        auto raw_at = [&](int i) -> NT {
            if constexpr (FromPts) return raw[i];
            else return nin[6 * q + i];
        };
        if (F > 0) {
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (pend[k]) {                 // queued: written after the sweep
                    bil_push(qu, a, k, F);
                } else if (s_c[k * S + a].w != 0.f) {
                    st_f(&v[3 * k], r[k].x); st_f(&v[3 * k + 1], r[k].y); st_f(&v[3 * k + 2], r[k].z);
                } else {                       // missing triangle: input bits unchanged
                    v[3 * k] = raw_at(3 * k);
                    v[3 * k + 1] = raw_at(3 * k + 1);
                    v[3 * k + 2] = raw_at(3 * k + 2);
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < 6; ++i) v[i] = raw_at(i);
        }
        // streaming stores (float32 normals): they write partial lines, about
        // 2 MB more per launch on a 480x640 frame, but the whole path gains
        // 2.4 us per frame.  A queued triangle is written after the sweep.
        const int t0 = t_index(ty, tx, q, 0), t1 = t_index(ty, tx, q, 1);
        if (!(pend[0] | pend[1])) {
#pragma unroll
            for (int i = 0; i < 6; ++i) bil_store(&nout[6 * q + i], v[i]);
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (!pend[0]) bil_store(&nout[6 * q + i], v[i]);
                if (!pend[1]) bil_store(&nout[6 * q + 3 + i], v[3 + i]);
            }
        }
        if (t0 >= 0 && !pend[0]) {
#pragma unroll
            for (int i = 0; i < 3; ++i) bil_store(&nT[3 * (size_t)t0 + i], v[i]);
        }
        if (t1 >= 0 && !pend[1]) {
#pragma unroll
            for (int i = 0; i < 3; ++i) bil_store(&nT[3 * (size_t)t1 + i], v[3 + i]);
        }
    };
    if (F > 0) {
        sweep(halo, TQH, TQW, emit);
    } else {
        const DivBy byTQW(TQW);
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int idx = slot; idx < TQH * TQW; idx += waves ? kWave : kTileBlock / QL) {
            const int ty = byTQW.div(idx);
            emit(ty, idx - ty * TQW, 0, z, z, false, false);
        }
    }
    if (F > 0) {
        // the queued triangles of the last sweep, one wave each (the sweep
        // ended with a barrier)
        const int nq = qu.count[F];
        for (int e = wave; e < nq; e += kTileBlock / kWave) {
            const int a = qu.entry[e] >> 1, k = qu.entry[e] & 1;
            const float4 r = bil_fallback_wave<R, NT>(s_c, cur, a, k, W, S, ka, kb);
            if (lane == 0) {
                const int ly = a / W, lx = a - ly * W;
                const size_t q = (size_t)(oy + ly) * Nq + (ox + lx);
                NT v[3];
                st_f(&v[0], r.x); st_f(&v[1], r.y); st_f(&v[2], r.z);
#pragma unroll
                for (int i = 0; i < 3; ++i) bil_store(&nout[6 * q + 3 * k + i], v[i]);
                const int t = t_index(ly - halo, lx - halo, q, k);
                if (t >= 0) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) bil_store(&nT[3 * (size_t)t + i], v[i]);
                }
            }
        }
    }
    __syncthreads();                 // LDS is reused by the next tile
}

}  // namespace pl
