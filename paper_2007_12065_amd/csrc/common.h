// Internal helpers shared by the gfx950 kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/pl.h"

namespace pl {

constexpr int kWave = 64;        // CDNA wavefront width
constexpr int kNumXcd = 8;       // MI355X: 8 accelerator complex dies, 32 CUs each

// NaN test on the bit pattern: exponent all ones, mantissa non-zero.  Immune
// to any fast-math or finite-math compiler flag.
__device__ __forceinline__ bool is_nan_bits(float x) {
    return (__float_as_uint(x) & 0x7fffffffu) > 0x7f800000u;
}

__device__ __forceinline__ float qnan() { return __uint_as_float(0x7fc00000u); }

// Workgroups are dispatched round-robin over the XCDs (workgroup b runs on
// XCD b mod 8), and each XCD has its own L2.  Remap the dispatch index so
// each XCD receives a contiguous range of tiles: neighbouring tiles, which
// share halo data, then hit the same L2.  A bijection on [0, n).
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int xcd = b % kNumXcd;
    const int idx = b / kNumXcd;
    const int q = n / kNumXcd;
    const int rem = n % kNumXcd;
    const int start = xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
    return start + idx;
}

// The same dealing when only the first `total` numbers of a larger grid carry
// work: each XCD takes a contiguous eighth of [0, total), so all eight share
// the work however small `total` is; workgroups past their XCD's range get
// -1.  With grid >= total each XCD is dealt ceil((grid - x) / 8) >=
// ceil((total - x) / 8) workgroups, enough for its range: every number in
// [0, total) is taken exactly once.
__device__ __forceinline__ int xcd_remap_active(int b, int total) {
    const int xcd = b % kNumXcd;
    const int idx = b / kNumXcd;
    const int q = total / kNumXcd;
    const int rem = total % kNumXcd;
    if (idx >= q + (xcd < rem ? 1 : 0)) return -1;
    const int start = xcd < rem ? xcd * (q + 1) : rem * (q + 1) + (xcd - rem) * q;
    return start + idx;
}

// Division of a small non-negative index by a workgroup-uniform divisor d:
// with m = ceil(2^32 / d), floor(i / d) = umulhi(i, m) for every i < 2^32 / d
// (the error term i (m d - 2^32) / (d 2^32) stays below 1 / d).  Tile
// indices are far below that bound.
struct DivBy {
    unsigned m;
    __device__ __forceinline__ explicit DivBy(int d) : m(0xFFFFFFFFu / (unsigned)d + 1u) {}
    __device__ __forceinline__ int div(int i) const { return (int)__umulhi((unsigned)i, m); }
};

// Inclusive prefix sum across one 64-wide wavefront.
__device__ __forceinline__ int wave_inclusive_scan(int x) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) x += __shfl_xor(x, d, kWave);
    return x;
}

// Half storage helpers (normals in PL_F16 mode).
__device__ __forceinline__ float ld_f(const float *p) { return *p; }
__device__ __forceinline__ float ld_f(const __half *p) { return __half2float(*p); }
__device__ __forceinline__ void st_f(float *p, float v) { *p = v; }
// The value as a rounded float32, opaque to the optimiser (an empty asm with
// a VGPR operand, no instruction): without it the compiler may fuse the
// product that produced v into the float->half conversion (v_fma_mix*),
// rounding once to half instead of to float and then to half -- and do so in
// some inlining contexts only, so that one tile body would give different
// float16 bits in different kernels.
__device__ __forceinline__ float f32_rounded(float v) {
    asm volatile("" : "+v"(v));
    return v;
}
__device__ __forceinline__ void st_f(__half *p, float v) { *p = __float2half_rn(f32_rounded(v)); }

// Streaming stores for outputs a kernel writes once and never reads back: the
// non-temporal hint sends them on towards memory instead of leaving them
// dirty in L2 for the write-back at the kernel's end.  Same bits as a plain
// store; the next kernel reads them after its own cache acquire.  Used where
// it measured faster (480x640 frame: mesh emit 8.6 -> 7.2 us, normals 5.7
// -> 4.7 us, vertex update 7.6 -> 6.5 us, same bytes; the bilateral's
// float32 outputs: 2.4 us less per frame over the whole path, although their
// strided pieces then reach memory as partial lines); the Laplacian's
// outputs (no change) keep plain stores.
__device__ __forceinline__ void st_stream(float *p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_stream(int32_t *p, int32_t v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_stream(uint32_t *p, uint32_t v) { __builtin_nontemporal_store(v, p); }
// two consecutive floats, 8-byte aligned, in one store
__device__ __forceinline__ void st_stream2(float *p, float a, float b) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    f2v v;
    v.x = a;
    v.y = b;
    __builtin_nontemporal_store(v, reinterpret_cast<f2v *>(p));
}

// ---- host side -----------------------------------------------------------

void set_error(const char *fmt, ...);
pl_status hip_check(hipError_t e, const char *what);

// Launchers implemented next to their kernels.  Arguments are validated by
// the ABI layer before these run.
pl_status launch_mesh(const float *pts, int M, int N, uint8_t *tri_valid,
                      int32_t *tri_map, int32_t *triangles, int32_t *halfedges,
                      int32_t cap, int32_t *n_tri, void *ws, hipStream_t s);
size_t mesh_workspace(int M, int N);
// The allocation-free mesh entry's scratch: capacity in bytes, and its device
// address on the device of stream `s` (looked up on the first call there).
size_t mesh_static_scratch_bytes();
pl_status mesh_static_scratch(hipStream_t s, void **out);

pl_status launch_laplacian(const float *in, float *out, int M, int N, int kernel,
                           float lambda, int iterations, void *ws, hipStream_t s);
size_t laplacian_workspace(int M, int N, int iterations);
int laplacian_fused_sweeps(int kernel);

pl_status launch_tri_normals(const float *pts, int M, int N, void *normals,
                             pl_dtype ndt, float *centroids, hipStream_t s);

pl_status launch_bilateral(const void *nin, const float *cen, pl_dtype ndt, int M,
                           int N, int kernel, float sigma_length, float sigma_angle,
                           int iterations, void *nout, const int32_t *tri_map,
                           void *normals_T, void *ws, hipStream_t s);
size_t bilateral_workspace(int M, int N, pl_dtype ndt, int iterations);

pl_status launch_group_assign(const float *pts, int n_pts, const int32_t *tris,
                              const void *normals, pl_dtype ndt, const int32_t *n_tri, int cap,
                              const float *dom, int l, float l_max, float ang_min,
                              uint8_t *groups, hipStream_t s);
int group_assign_blocks(int cap);

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t smooth_frame_workspace(const pl_frame &f, pl_dtype ndt);
pl_status launch_smooth_frame(const pl_frame &f, pl_dtype ndt, void *ws, hipStream_t s,
                              hipEvent_t *events = nullptr, int n_events = 0,
                              int32_t *kinds = nullptr, int n_kinds = 0,
                              int32_t *n_launches = nullptr);

size_t batch_workspace(const pl_frame *frames, int n, pl_dtype ndt);
pl_status batch_create(const pl_frame *frames, int n, pl_dtype ndt, void *ws, hipStream_t s,
                       pl_batch_s **out);
pl_status batch_run(const pl_batch_s *b, const uint8_t *active, hipStream_t s);
int batch_size(const pl_batch_s *b);
pl_status batch_capture(pl_batch_s *b, const uint8_t *active, int bound, hipStream_t s);
pl_status batch_replay(const pl_batch_s *b, int n_active, hipStream_t s);
void batch_destroy(pl_batch_s *b);

}  // namespace pl
