// Group assignment over one triangle list (pl_group_assign): one launch,
// four triangles of T per thread (the body is in groups.h).
#include "groups.h"

namespace pl {

namespace {

template <typename NT>
__global__ __launch_bounds__(kGroupBlock) void k_group_assign(
    const float *__restrict__ pts, int n_pts, const int32_t *__restrict__ tris,
    const NT *__restrict__ normals, const int32_t *__restrict__ n_tri, int cap,
    const float *__restrict__ dom, int l, float lmax2, float ang_min,
    uint8_t *__restrict__ groups) {
    // each XCD takes one contiguous eighth of T, so the vertex rows that
    // neighbouring workgroups share meet in one L2
    const int chunk = xcd_remap((int)blockIdx.x, (int)gridDim.x);
    group_rows<NT>(pts, n_pts, tris, normals, n_tri, cap, dom, l, lmax2, ang_min, groups,
                   (chunk * kGroupBlock + (int)threadIdx.x) * kGroupPer);
}

}  // namespace

int group_assign_blocks(int cap) {
    const long per_block = (long)kGroupBlock * kGroupPer;
    return (int)(((long)cap + per_block - 1) / per_block);
}

pl_status launch_group_assign(const float *pts, int n_pts, const int32_t *tris,
                              const void *normals, pl_dtype ndt, const int32_t *n_tri, int cap,
                              const float *dom, int l, float l_max, float ang_min,
                              uint8_t *groups, hipStream_t s) {
    if (cap == 0) return PL_OK;
    const float lmax2 = l_max * l_max;
    const int blocks = group_assign_blocks(cap);
    if (ndt == PL_F32)
        k_group_assign<float><<<blocks, kGroupBlock, 0, s>>>(
            pts, n_pts, tris, static_cast<const float *>(normals), n_tri, cap, dom, l, lmax2,
            ang_min, groups);
    else
        k_group_assign<__half><<<blocks, kGroupBlock, 0, s>>>(
            pts, n_pts, tris, static_cast<const __half *>(normals), n_tri, cap, dom, l, lmax2,
            ang_min, groups);
    return hip_check(hipGetLastError(), "k_group_assign");
}

}  // namespace pl
