// Triangle centroids and normals over the implicit full mesh T_FC (Sec. 5.2).
// One thread per quad: four corner loads (shared through L1/L2 with the
// neighbouring quads), two centroids and two normals written contiguously in
// GID order.  Pure streaming work: 12 B/point in, 2 x 12 B/triangle out.
#include "common.h"

namespace pl {

namespace {

constexpr int kBlock = 256;

struct V3 {
    float x, y, z;
};

__device__ __forceinline__ V3 ld3(const float *p) { return V3{p[0], p[1], p[2]}; }
__device__ __forceinline__ bool ok3(const V3 &a) {
    return !(is_nan_bits(a.x) || is_nan_bits(a.y) || is_nan_bits(a.z));
}

// centroid (a + b + c) / 3 and unit normal of (b - a) x (c - a); NaN normal
// when the cross product vanishes.
__device__ __forceinline__ void tri(const V3 &a, const V3 &b, const V3 &c, V3 &cen, V3 &nrm) {
    const float third = 1.0f / 3.0f;
    cen.x = (a.x + b.x + c.x) * third;
    cen.y = (a.y + b.y + c.y) * third;
    cen.z = (a.z + b.z + c.z) * third;
    const float e1x = b.x - a.x, e1y = b.y - a.y, e1z = b.z - a.z;
    const float e2x = c.x - a.x, e2y = c.y - a.y, e2z = c.z - a.z;
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

template <typename NT>
__global__ __launch_bounds__(kBlock) void k_tri_normals(const float *__restrict__ pts, int N,
                                                        int Nq, size_t Q,
                                                        NT *__restrict__ normals,
                                                        float *__restrict__ centroids) {
    const size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= Q) return;
    const int u = (int)(q / Nq), v = (int)(q - (size_t)u * Nq);
    const float *r0 = pts + 3 * ((size_t)u * N + v);
    const float *r1 = r0 + 3 * (size_t)N;
    const V3 p1 = ld3(r0), p2 = ld3(r0 + 3), p3 = ld3(r1 + 3), p4 = ld3(r1);
    const bool v1 = ok3(p1), v2 = ok3(p2), v3 = ok3(p3), v4 = ok3(p4);
    const V3 nan3{qnan(), qnan(), qnan()};
    V3 c0 = nan3, n0 = nan3, c1 = nan3, n1 = nan3;
    if (v1 & v2 & v3) tri(p3, p2, p1, c0, n0);     // first triangle
    if (v1 & v3 & v4) tri(p1, p4, p3, c1, n1);     // second triangle
    float *co = centroids + 6 * q;
    co[0] = c0.x; co[1] = c0.y; co[2] = c0.z;
    co[3] = c1.x; co[4] = c1.y; co[5] = c1.z;
    NT *no = normals + 6 * q;
    st_f(no + 0, n0.x); st_f(no + 1, n0.y); st_f(no + 2, n0.z);
    st_f(no + 3, n1.x); st_f(no + 4, n1.y); st_f(no + 5, n1.z);
}

}  // namespace

pl_status launch_tri_normals(const float *pts, int M, int N, void *normals, pl_dtype ndt,
                             float *centroids, hipStream_t s) {
    const int Nq = N - 1;
    const size_t Q = (size_t)(M - 1) * Nq;
    const int blocks = (int)((Q + kBlock - 1) / kBlock);
    if (ndt == PL_F32)
        k_tri_normals<float><<<blocks, kBlock, 0, s>>>(pts, N, Nq, Q,
                                                       static_cast<float *>(normals), centroids);
    else
        k_tri_normals<__half><<<blocks, kBlock, 0, s>>>(pts, N, Nq, Q,
                                                        static_cast<__half *>(normals), centroids);
    return hip_check(hipGetLastError(), "k_tri_normals");
}

}  // namespace pl
