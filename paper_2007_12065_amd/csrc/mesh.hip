// Organized-point-cloud mesh extraction (Sec. 4.2, Alg. 1 and Alg. 2) as an
// ordered compaction over quad rows.
//
//   k_mesh_count : one workgroup per quad row.  Tests the points of rows u
//                  and u+1 for NaN (all loads of a 1024-column chunk in
//                  flight at once, validity staged in LDS), stores a 2-bit
//                  code per quad (bit 0: first triangle valid, bit 1:
//                  second) and the row's triangle count.
//   k_mesh_emit  : one workgroup per quad row.  Sums the counts of the rows
//                  above it (a few hundred to a few thousand integers, L2
//                  hits) to place its rows in T, re-scans the codes of rows
//                  u-1, u, u+1 (bytes) so every triangle knows its own index
//                  and its four cross-quad neighbours' indices, then writes
//                  T_map, T and HE in one pass; the last row writes |T|.
//
// Triangle indices come from prefix sums in GID order, so T is in exactly
// the append order of Alg. 1 and every output is bit-exact and
// deterministic.
#include "common.h"

namespace pl {

namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;

__device__ __forceinline__ bool point_valid(const float *p) {
    return !(is_nan_bits(p[0]) || is_nan_bits(p[1]) || is_nan_bits(p[2]));
}

constexpr int kChunk = 4 * kBlock;     // columns per pass of k_mesh_count

__global__ __launch_bounds__(kBlock) void k_mesh_count(
    const float *__restrict__ pts, int N, uint8_t *__restrict__ codes,
    uint8_t *__restrict__ tri_valid, int *__restrict__ row_count) {
    __shared__ uint8_t ok[2][kChunk + 1];
    __shared__ int red[kWaves];
    const int u = blockIdx.x;
    const int Nq = N - 1;
    const float *r0 = pts + (size_t)u * N * 3;
    const float *r1 = r0 + (size_t)N * 3;
    int cnt = 0;
    for (int v0 = 0; v0 < Nq; v0 += kChunk) {
        // validity of points v0 .. v0 + kChunk of both rows, all loads issued
        // before any is used
        float x[2][5], y[2][5], z[2][5];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int v = v0 + threadIdx.x + j * kBlock;
            const bool in = (j < 4 || threadIdx.x == 0) && v < N && v <= v0 + kChunk;
            x[0][j] = in ? r0[3 * v] : 0.f; y[0][j] = in ? r0[3 * v + 1] : 0.f; z[0][j] = in ? r0[3 * v + 2] : 0.f;
            x[1][j] = in ? r1[3 * v] : 0.f; y[1][j] = in ? r1[3 * v + 1] : 0.f; z[1][j] = in ? r1[3 * v + 2] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int l = threadIdx.x + j * kBlock;
            if (j < 4 || threadIdx.x == 0) {
#pragma unroll
                for (int r = 0; r < 2; ++r)
                    ok[r][l] = !(is_nan_bits(x[r][j]) || is_nan_bits(y[r][j]) || is_nan_bits(z[r][j]));
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int l = threadIdx.x + j * kBlock;
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
        for (int w = 0; w < kWaves; ++w) t += red[w];
        row_count[u] = t;
    }
}

// Block-wide exclusive scan of a packed triple of 10-bit counters (each
// chunk holds at most 2 * kBlock = 512 triangles per row, so no field
// overflows).  Returns the exclusive prefix; *total receives the sum.
__device__ __forceinline__ int block_exclusive_scan(int x, int *total) {
    __shared__ int wsum[kWaves];
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int incl = wave_inclusive_scan(x);
    __syncthreads();                       // wsum reuse across calls
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int t = wsum[w];
        before += w < wid ? t : 0;
        all += t;
    }
    *total = all;
    return before + incl - x;
}

__device__ __forceinline__ int popc2(int c) { return (c & 1) + ((c >> 1) & 1); }

__global__ __launch_bounds__(kBlock) void k_mesh_emit(
    const uint8_t *__restrict__ codes, const int *__restrict__ row_count, int Mq, int N,
    int32_t *__restrict__ tri_map, int32_t *__restrict__ tris,
    int32_t *__restrict__ he, int cap, int32_t *__restrict__ n_tri) {
    __shared__ int red[kWaves];
    const int u = blockIdx.x;
    const int Nq = N - 1;
    const uint8_t *cr0 = codes + (size_t)u * Nq;
    const uint8_t *crm = u > 0 ? cr0 - Nq : cr0;        // row u-1
    const uint8_t *crp = u + 1 < Mq ? cr0 + Nq : cr0;   // row u+1
    // index in T of the first triangle of rows u-1, u, u+1
    int above = 0;
    for (int r = threadIdx.x; r < u - 1; r += kBlock) above += row_count[r];
    above = wave_sum(above);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = above;
    __syncthreads();
    int basem = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) basem += red[w];
    const int cm_row = u > 0 ? row_count[u - 1] : 0;
    const int base0 = basem + cm_row;
    const int basep = base0 + row_count[u];
    if (u == Mq - 1 && threadIdx.x == 0) *n_tri = basep;
    int carry0 = 0, carrym = 0, carryp = 0;
    for (int v0 = 0; v0 < Nq; v0 += kBlock) {
        const int v = v0 + threadIdx.x;
        const bool in = v < Nq;
        const int c0 = in ? cr0[v] : 0;
        const int cm = (in && u > 0) ? crm[v] : 0;
        const int cp = (in && u + 1 < Mq) ? crp[v] : 0;
        const int n0 = popc2(c0);
        int total;
        const int ex = block_exclusive_scan(n0 | (popc2(cm) << 10) | (popc2(cp) << 20), &total);
        const int p0 = ex & 1023, pm = (ex >> 10) & 1023, pp = (ex >> 20) & 1023;
        if (in) {
            const int f = c0 & 1, s = (c0 >> 1) & 1;
            const int rank0 = base0 + carry0 + p0;       // index of (u,v,0) if valid
            const int rF = f ? rank0 : -1;
            const int rS = s ? rank0 + f : -1;
            const size_t q = (size_t)u * Nq + v;
            *reinterpret_cast<int2 *>(tri_map + 2 * q) = make_int2(rF, rS);
            const int i1 = u * N + v, i2 = i1 + 1, i3 = i1 + N + 1, i4 = i1 + N;
            if (f && rF < cap) {
                tris[3 * rF + 0] = i3; tris[3 * rF + 1] = i2; tris[3 * rF + 2] = i1;
            }
            if (s && rS < cap) {
                tris[3 * rS + 0] = i1; tris[3 * rS + 1] = i4; tris[3 * rS + 2] = i3;
            }
            if (he) {
                // Right = (u, v+1, 1), Top = (u-1, v, 1), Left = (u, v-1, 0),
                // Bottom = (u+1, v, 0); indices from the prefix sums.
                const int cr = v + 1 < Nq ? cr0[v + 1] : 0;
                const int cl = v > 0 ? cr0[v - 1] : 0;
                const int right = (cr & 2) ? rank0 + n0 + (cr & 1) : -1;
                const int left = (cl & 1) ? rank0 - popc2(cl) : -1;
                const int top = (cm & 2) ? basem + carrym + pm + (cm & 1) : -1;
                const int bottom = (cp & 1) ? basep + carryp + pp : -1;
                if (f && rF < cap) {
                    he[3 * rF + 0] = right >= 0 ? 3 * right : -1;
                    he[3 * rF + 1] = top >= 0 ? 3 * top + 1 : -1;
                    he[3 * rF + 2] = s ? 3 * rS + 2 : -1;
                }
                if (s && rS < cap) {
                    he[3 * rS + 0] = left >= 0 ? 3 * left : -1;
                    he[3 * rS + 1] = bottom >= 0 ? 3 * bottom + 1 : -1;
                    he[3 * rS + 2] = f ? 3 * rF + 2 : -1;
                }
            }
        }
        carry0 += total & 1023;
        carrym += (total >> 10) & 1023;
        carryp += (total >> 20) & 1023;
    }
}

struct MeshWs {
    uint8_t *codes;
    int *row_count;
};

MeshWs carve(void *ws, int M, int N) {
    const size_t Q = (size_t)(M - 1) * (N - 1);
    uint8_t *b = static_cast<uint8_t *>(ws);
    MeshWs w;
    w.codes = b;
    w.row_count = reinterpret_cast<int *>(b + align_up(Q, 256));
    return w;
}

}  // namespace

size_t mesh_workspace(int M, int N) {
    const size_t Q = (size_t)(M - 1) * (N - 1);
    return align_up(Q, 256) + align_up(sizeof(int) * (M - 1), 256);
}

pl_status launch_mesh(const float *pts, int M, int N, uint8_t *tri_valid,
                      int32_t *tri_map, int32_t *triangles, int32_t *halfedges,
                      int32_t cap, int32_t *n_tri, void *ws, hipStream_t s) {
    const int Mq = M - 1;
    MeshWs w = carve(ws, M, N);
    k_mesh_count<<<Mq, kBlock, 0, s>>>(pts, N, w.codes, tri_valid, w.row_count);
    if (pl_status st = hip_check(hipGetLastError(), "k_mesh_count")) return st;
    k_mesh_emit<<<Mq, kBlock, 0, s>>>(w.codes, w.row_count, Mq, N, tri_map, triangles,
                                      halfedges, cap, n_tri);
    return hip_check(hipGetLastError(), "k_mesh_emit");
}

}  // namespace pl
