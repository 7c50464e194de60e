// Vertex update from filtered normals: the second stage of the bilateral
// mesh denoising the paper cites with Eqs. (3)-(6) (Sun et al., 2007), which
// Polylidar3D skips (Sec. 5.2).  Each sweep moves every vertex by the mean,
// over the valid triangles of T_FC that contain it, of the correction that
// puts it on the plane through the triangle's centroid with the triangle's
// filtered normal:
//     x <- x + (1 / |F|) sum_f n_f (n_f . (c_f - x)).
//
// On the implicit right-cut mesh vertex (r, c) lies in at most six
// triangles: both triangles of quad (r, c) (as p1) and of quad (r-1, c-1)
// (as p3), the first triangle of quad (r, c-1) (as p2) and the second of
// quad (r-1, c) (as p4).  Their vertices are the point and six of its eight
// grid neighbours, so one thread per point reads a 3 x 3 neighbourhood (the
// rows overlap between threads and come from cache) and the six normals.
// Sweeps are Jacobi: each reads the previous sweep's points.
#include "vu.h"

namespace pl {

namespace {

constexpr int kVuBlock = 256;

struct P3 {
    float x, y, z;
};

__device__ __forceinline__ P3 ld_p(const float *__restrict__ pts, int N, int r, int c) {
    const float *p = pts + 3 * ((size_t)r * N + c);
    return {p[0], p[1], p[2]};
}

__device__ __forceinline__ bool p_ok(P3 p) {
    return !(is_nan_bits(p.x) || is_nan_bits(p.y) || is_nan_bits(p.z));
}

// Adds triangle (a, b, d) with normal n to the sums if it counts.
template <typename NT>
__device__ __forceinline__ void vu_add(P3 x, P3 a, P3 b, P3 d, const NT *__restrict__ n,
                                       float &sx, float &sy, float &sz, int &count) {
    const float nx = ld_f(n), ny = ld_f(n + 1), nz = ld_f(n + 2);
    if (!(p_ok(a) && p_ok(b) && p_ok(d)) || is_nan_bits(nx) || is_nan_bits(ny) || is_nan_bits(nz))
        return;
    // the centroid through a multiply by the rounded 1/3 (within an ulp of
    // the quotient; an IEEE division would cost ten instructions a component)
    constexpr float kThird = 1.0f / 3.0f;
    const float cx = fmaf(a.x + b.x + d.x, kThird, -x.x);
    const float cy = fmaf(a.y + b.y + d.y, kThird, -x.y);
    const float cz = fmaf(a.z + b.z + d.z, kThird, -x.z);
    const float proj = fmaf(nx, cx, fmaf(ny, cy, nz * cz));
    sx = fmaf(nx, proj, sx);
    sy = fmaf(ny, proj, sy);
    sz = fmaf(nz, proj, sz);
    ++count;
}

template <typename NT>
__global__ __launch_bounds__(kVuBlock) void k_vertex_update(const float *__restrict__ in,
                                                            float *__restrict__ out, int M, int N,
                                                            const NT *__restrict__ normals) {
    // one thread per point, row-major over the frame (a 1-D grid: any M);
    // contiguous runs of points per XCD, so the normals of the quad rows
    // that neighbouring point rows share are fetched once into one L2
    const long long idx =
        (long long)xcd_remap((int)blockIdx.x, (int)gridDim.x) * kVuBlock + threadIdx.x;
    if (idx >= (long long)M * N) return;
    const int r = (int)(idx / N), c = (int)(idx - (long long)r * N);
    const P3 x = ld_p(in, N, r, c);
    float *o = out + 3 * ((size_t)r * N + c);
    float sx = 0.0f, sy = 0.0f, sz = 0.0f;
    int count = 0;
    if (p_ok(x)) {
        const int Nq = N - 1;
        const bool up = r > 0, down = r < M - 1, left = c > 0, right = c < N - 1;
        const P3 nan3 = {qnan(), qnan(), qnan()};
        // the six neighbours the incident triangles use
        const P3 pr = right ? ld_p(in, N, r, c + 1) : nan3;
        const P3 pl_ = left ? ld_p(in, N, r, c - 1) : nan3;
        const P3 pd = down ? ld_p(in, N, r + 1, c) : nan3;
        const P3 pu = up ? ld_p(in, N, r - 1, c) : nan3;
        const P3 pdr = (down && right) ? ld_p(in, N, r + 1, c + 1) : nan3;
        const P3 pul = (up && left) ? ld_p(in, N, r - 1, c - 1) : nan3;
        auto nrm = [&](int u, int v, int k) { return normals + 3 * (2 * ((size_t)u * Nq + v) + k); };
        // triangle k = 0 of quad (u, v) is (p3, p2, p1), k = 1 is (p1, p4, p3)
        if (down && right) {            // quad (r, c): x = p1
            vu_add(x, pdr, pr, x, nrm(r, c, 0), sx, sy, sz, count);
            vu_add(x, x, pd, pdr, nrm(r, c, 1), sx, sy, sz, count);
        }
        if (down && left)               // quad (r, c-1): x = p2, in its first triangle
            vu_add(x, pd, x, pl_, nrm(r, c - 1, 0), sx, sy, sz, count);
        if (up && left) {               // quad (r-1, c-1): x = p3
            vu_add(x, x, pu, pul, nrm(r - 1, c - 1, 0), sx, sy, sz, count);
            vu_add(x, pul, pl_, x, nrm(r - 1, c - 1, 1), sx, sy, sz, count);
        }
        if (up && right)                // quad (r-1, c): x = p4, in its second triangle
            vu_add(x, pu, x, pr, nrm(r - 1, c, 1), sx, sy, sz, count);
    }
    if (count) {
        const float inv = __builtin_amdgcn_rcpf((float)count);   // count in 1..6
        st_stream(&o[0], fmaf(sx, inv, x.x));
        st_stream(&o[1], fmaf(sy, inv, x.y));
        st_stream(&o[2], fmaf(sz, inv, x.z));
    } else {
        st_stream(&o[0], x.x);
        st_stream(&o[1], x.y);
        st_stream(&o[2], x.z);
    }
}

}  // namespace

size_t vertex_update_workspace(int M, int N, int iterations) {
    return iterations > 1 ? align_up(12 * (size_t)M * N, 256) : 0;
}

pl_status launch_vertex_update(const float *in, float *out, int M, int N, const void *normals,
                               pl_dtype ndt, int iterations, void *ws, hipStream_t s) {
    const size_t bytes = 12 * (size_t)M * N;
    if (iterations == 0)
        return hip_check(hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
    const unsigned grid = (unsigned)(((size_t)M * N + kVuBlock - 1) / kVuBlock);
    const float *src = in;
    for (int it = 0; it < iterations; ++it) {
        // the last sweep lands in `out`; earlier ones alternate with the workspace
        float *dst = ((iterations - 1 - it) % 2 == 0) ? out : static_cast<float *>(ws);
        if (ndt == PL_F32)
            k_vertex_update<float><<<grid, kVuBlock, 0, s>>>(src, dst, M, N,
                                                             static_cast<const float *>(normals));
        else
            k_vertex_update<__half><<<grid, kVuBlock, 0, s>>>(src, dst, M, N,
                                                              static_cast<const __half *>(normals));
        if (pl_status st = hip_check(hipGetLastError(), "k_vertex_update")) return st;
        src = dst;
    }
    return PL_OK;
}

}  // namespace pl
