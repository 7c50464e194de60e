// extern "C" entry points of libpl.so: argument validation, then dispatch to
// the kernel launchers.  Nothing is enqueued when validation fails.
#include "common.h"
#include "ga.h"
#include "he.h"
#include "vu.h"
#include "tuning.h"

#include <algorithm>
#include <vector>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>

namespace pl {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

pl_status hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return PL_OK;
    set_error("%s: %s", what, hipGetErrorString(e));
    return PL_ERR_HIP;
}

#define PL_TRY(x)                          \
    do {                                   \
        if (pl_status _s = (x)) return _s; \
    } while (0)

namespace {

struct Range {
    const void *p;
    size_t bytes;
};

bool overlap(Range a, Range b) {
    if (!a.p || !b.p || !a.bytes || !b.bytes) return false;
    const uintptr_t a0 = (uintptr_t)a.p, b0 = (uintptr_t)b.p;
    return a0 < b0 + b.bytes && b0 < a0 + a.bytes;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

pl_status check_shape(int32_t M, int32_t N) {
    if (M < 2 || N < 2) {
        set_error("shape %d x %d: need M >= 2 and N >= 2", M, N);
        return PL_ERR_SHAPE;
    }
    if (6.0 * (double)(M - 1) * (double)(N - 1) >= 2147483648.0) {
        set_error("shape %d x %d: 6 (M-1)(N-1) must stay below 2^31", M, N);
        return PL_ERR_SHAPE;
    }
    return PL_OK;
}

pl_status check_kernel(int32_t k) {
    if (k < 3 || k > 9 || (k % 2) == 0) {
        set_error("kernel size %d: must be odd and in [3, 9]", k);
        return PL_ERR_KERNEL;
    }
    return PL_OK;
}

pl_status check_ptrs(std::initializer_list<std::pair<const void *, const char *>> ps) {
    for (auto &p : ps) {
        if (!p.first) {
            set_error("%s is NULL", p.second);
            return PL_ERR_ARG;
        }
        if (!aligned16(p.first)) {
            set_error("%s is not 16-byte aligned", p.second);
            return PL_ERR_ARG;
        }
    }
    return PL_OK;
}

pl_status check_ws(const void *ws, size_t have, size_t need) {
    if (need == 0) return PL_OK;
    if (!ws || have < need) {
        set_error("workspace of %zu bytes needed, %zu given", need, ws ? have : (size_t)0);
        return PL_ERR_WORKSPACE;
    }
    if (!aligned16(ws)) {
        set_error("workspace is not 16-byte aligned");
        return PL_ERR_ARG;
    }
    return PL_OK;
}

// Arguments of the mesh entry points (pl_mesh_opc, pl_mesh_opc_static).
pl_status check_mesh(const float *pts, int32_t M, int32_t N, uint8_t *tri_valid,
                     int32_t *tri_map, int32_t *triangles, int32_t *halfedges, int32_t cap,
                     int32_t *n_tri) {
    PL_TRY(check_shape(M, N));
    if (cap < 0) {
        set_error("cap %d < 0", cap);
        return PL_ERR_ARG;
    }
    PL_TRY(check_ptrs({{pts, "pts"}, {tri_map, "tri_map"}, {n_tri, "n_tri"}}));
    if (cap > 0) PL_TRY(check_ptrs({{triangles, "triangles"}}));
    if (halfedges && cap > 0) PL_TRY(check_ptrs({{halfedges, "halfedges"}}));
    if (tri_valid) PL_TRY(check_ptrs({{tri_valid, "tri_valid"}}));
    return PL_OK;
}

// No output of a mesh call may overlap the points or another output
// (`ws` is the workspace, if any).
pl_status check_mesh_alias(const float *pts, int32_t M, int32_t N, uint8_t *tri_valid,
                           int32_t *tri_map, int32_t *triangles, int32_t *halfedges,
                           int32_t cap, int32_t *n_tri, Range ws) {
    const size_t T = 2 * (size_t)(M - 1) * (N - 1);
    const Range in{pts, sizeof(float) * 3 * (size_t)M * N};
    const Range outs[] = {{tri_valid, tri_valid ? T : 0},
                          {tri_map, 4 * T},
                          {triangles, 12 * (size_t)cap},
                          {halfedges, halfedges ? 12 * (size_t)cap : 0},
                          {n_tri, 4},
                          ws};
    for (size_t i = 0; i < sizeof(outs) / sizeof(outs[0]); ++i) {
        if (overlap(in, outs[i])) {
            set_error("output %zu overlaps pts", i);
            return PL_ERR_ALIAS;
        }
        for (size_t j = i + 1; j < sizeof(outs) / sizeof(outs[0]); ++j)
            if (overlap(outs[i], outs[j])) {
                set_error("outputs %zu and %zu overlap", i, j);
                return PL_ERR_ALIAS;
            }
    }
    return PL_OK;
}

}  // namespace
}  // namespace pl

using namespace pl;

static_assert((int)PL_STAGE_LAPLACIAN == (int)pl::kStageLaplacian &&
                  (int)PL_STAGE_BILATERAL == (int)pl::kStageBilateral &&
                  (int)PL_STAGE_BATCH_LAPLACIAN == (int)pl::kStageBatchLaplacian &&
                  (int)PL_STAGE_BATCH_BILATERAL == (int)pl::kStageBatchBilateral &&
                  (int)PL_STAGE_LAPLACIAN_SMALL == (int)pl::kStageLaplacianSmall &&
                  (int)PL_STAGE_BILATERAL_SMALL == (int)pl::kStageBilateralSmall,
              "pl_stage and the tuning table's stages must agree");

extern "C" {

__attribute__((visibility("default"))) int32_t pl_version(void) { return 105; }

__attribute__((visibility("default"))) const char *pl_last_error(void) { return g_err; }

__attribute__((visibility("default"))) size_t pl_mesh_opc_workspace(int32_t M, int32_t N) {
    if (M < 2 || N < 2) return 0;
    return mesh_workspace(M, N);
}

__attribute__((visibility("default"))) pl_status pl_mesh_opc(
    const float *pts, int32_t M, int32_t N, uint8_t *tri_valid, int32_t *tri_map,
    int32_t *triangles, int32_t *halfedges, int32_t cap, int32_t *n_tri, void *ws,
    size_t ws_bytes, hipStream_t stream) {
    g_err[0] = 0;
    PL_TRY(check_mesh(pts, M, N, tri_valid, tri_map, triangles, halfedges, cap, n_tri));
    PL_TRY(check_ws(ws, ws_bytes, mesh_workspace(M, N)));
    PL_TRY(check_mesh_alias(pts, M, N, tri_valid, tri_map, triangles, halfedges, cap, n_tri,
                            {ws, mesh_workspace(M, N)}));
    return launch_mesh(pts, M, N, tri_valid, tri_map, triangles, cap > 0 ? halfedges : nullptr,
                       cap, n_tri, ws, stream);
}

__attribute__((visibility("default"))) pl_status pl_mesh_opc_static(
    const float *pts, int32_t M, int32_t N, uint8_t *tri_valid, int32_t *tri_map,
    int32_t *triangles, int32_t *halfedges, int32_t cap, int32_t *n_tri, hipStream_t stream) {
    g_err[0] = 0;
    PL_TRY(check_mesh(pts, M, N, tri_valid, tri_map, triangles, halfedges, cap, n_tri));
    const size_t need = mesh_workspace(M, N);
    if (need > mesh_static_scratch_bytes()) {
        set_error("shape %d x %d needs %zu bytes of mesh scratch; the static scratch of "
                  "pl_mesh_opc_static holds %zu (use pl_mesh_opc with a workspace)",
                  M, N, need, mesh_static_scratch_bytes());
        return PL_ERR_SHAPE;
    }
    PL_TRY(check_mesh_alias(pts, M, N, tri_valid, tri_map, triangles, halfedges, cap, n_tri,
                            {nullptr, 0}));
    void *scr = nullptr;
    PL_TRY(mesh_static_scratch(stream, &scr));
    return launch_mesh(pts, M, N, tri_valid, tri_map, triangles, cap > 0 ? halfedges : nullptr,
                       cap, n_tri, scr, stream);
}

__attribute__((visibility("default"))) size_t pl_laplacian_workspace(int32_t M, int32_t N,
                                                                     int32_t iterations) {
    if (M < 2 || N < 2 || iterations < 0) return 0;
    return laplacian_workspace(M, N, iterations);
}

__attribute__((visibility("default"))) int32_t pl_laplacian_fused_sweeps(int32_t kernel) {
    if (kernel < 3 || kernel > 9 || (kernel % 2) == 0) return 0;
    return laplacian_fused_sweeps(kernel);
}

__attribute__((visibility("default"))) pl_status pl_laplacian(
    const float *pts_in, float *pts_out, int32_t M, int32_t N, int32_t kernel, float lambda,
    int32_t iterations, void *ws, size_t ws_bytes, hipStream_t stream) {
    g_err[0] = 0;
    PL_TRY(check_shape(M, N));
    PL_TRY(check_kernel(kernel));
    if (!(lambda >= 0.f && lambda <= 1.f)) {
        set_error("lambda %g outside [0, 1]", (double)lambda);
        return PL_ERR_ARG;
    }
    if (iterations < 0) {
        set_error("iterations %d < 0", iterations);
        return PL_ERR_ARG;
    }
    PL_TRY(check_ptrs({{pts_in, "pts_in"}, {pts_out, "pts_out"}}));
    const size_t need = laplacian_workspace(M, N, iterations);
    PL_TRY(check_ws(ws, ws_bytes, need));
    const size_t bytes = sizeof(float) * 3 * (size_t)M * N;
    if (overlap({pts_in, bytes}, {pts_out, bytes}) || overlap({pts_in, bytes}, {ws, need}) ||
        overlap({pts_out, bytes}, {ws, need})) {
        set_error("pts_in, pts_out and the workspace must not overlap");
        return PL_ERR_ALIAS;
    }
    return launch_laplacian(pts_in, pts_out, M, N, kernel, lambda, iterations, ws, stream);
}

__attribute__((visibility("default"))) pl_status pl_tri_normals(const float *pts, int32_t M,
                                                                int32_t N, void *normals,
                                                                pl_dtype ndt, float *centroids,
                                                                hipStream_t stream) {
    g_err[0] = 0;
    PL_TRY(check_shape(M, N));
    if (ndt != PL_F32 && ndt != PL_F16) {
        set_error("unknown normal dtype %d", (int)ndt);
        return PL_ERR_ARG;
    }
    PL_TRY(check_ptrs({{pts, "pts"}, {normals, "normals"}, {centroids, "centroids"}}));
    const size_t T = 2 * (size_t)(M - 1) * (N - 1);
    const Range in{pts, sizeof(float) * 3 * (size_t)M * N};
    const Range nr{normals, T * 3 * (ndt == PL_F32 ? 4 : 2)};
    const Range cr{centroids, T * 12};
    if (overlap(in, nr) || overlap(in, cr) || overlap(nr, cr)) {
        set_error("pts, normals and centroids must not overlap");
        return PL_ERR_ALIAS;
    }
    return launch_tri_normals(pts, M, N, normals, ndt, centroids, stream);
}

__attribute__((visibility("default"))) size_t pl_bilateral_workspace(int32_t M, int32_t N,
                                                                     pl_dtype ndt,
                                                                     int32_t iterations) {
    if (M < 2 || N < 2 || iterations < 0 || (ndt != PL_F32 && ndt != PL_F16)) return 0;
    return bilateral_workspace(M, N, ndt, iterations);
}

__attribute__((visibility("default"))) pl_status pl_bilateral(
    const void *normals_in, const float *centroids, pl_dtype ndt, int32_t M, int32_t N,
    int32_t kernel, float sigma_length, float sigma_angle, int32_t iterations,
    void *normals_out, const int32_t *tri_map, void *normals_T, void *ws, size_t ws_bytes,
    hipStream_t stream) {
    g_err[0] = 0;
    PL_TRY(check_shape(M, N));
    PL_TRY(check_kernel(kernel));
    if (ndt != PL_F32 && ndt != PL_F16) {
        set_error("unknown normal dtype %d", (int)ndt);
        return PL_ERR_ARG;
    }
    if (!(sigma_length > 0.f) || !isfinite(sigma_length) || !(sigma_angle > 0.f) ||
        !isfinite(sigma_angle)) {
        set_error("sigmas must be finite and > 0 (got %g, %g)", (double)sigma_length,
                  (double)sigma_angle);
        return PL_ERR_ARG;
    }
    if (iterations < 0) {
        set_error("iterations %d < 0", iterations);
        return PL_ERR_ARG;
    }
    PL_TRY(check_ptrs({{normals_in, "normals_in"}, {centroids, "centroids"},
                       {normals_out, "normals_out"}}));
    if (tri_map) PL_TRY(check_ptrs({{tri_map, "tri_map"}, {normals_T, "normals_T"}}));
    const size_t need = bilateral_workspace(M, N, ndt, iterations);
    PL_TRY(check_ws(ws, ws_bytes, need));
    const size_t T = 2 * (size_t)(M - 1) * (N - 1);
    const size_t nb = T * 3 * (ndt == PL_F32 ? 4 : 2);
    const Range ins[] = {{normals_in, nb}, {centroids, T * 12}, {tri_map, tri_map ? T * 4 : 0}};
    const Range outs[] = {{normals_out, nb}, {normals_T, tri_map ? nb : 0}, {ws, need}};
    for (const Range &o : outs) {
        for (const Range &i : ins)
            if (overlap(i, o)) {
                set_error("an output of pl_bilateral overlaps an input");
                return PL_ERR_ALIAS;
            }
    }
    if (overlap(outs[0], outs[1]) || overlap(outs[0], outs[2]) || overlap(outs[1], outs[2])) {
        set_error("normals_out, normals_T and the workspace must not overlap");
        return PL_ERR_ALIAS;
    }
    return launch_bilateral(normals_in, centroids, ndt, M, N, kernel, sigma_length,
                            sigma_angle, iterations, normals_out, tri_map, normals_T, ws,
                            stream);
}

__attribute__((visibility("default"))) pl_status pl_tune_get(pl_stage stage, int32_t kernel,
                                                             int32_t *tile_rows,
                                                             int32_t *tile_cols, int32_t *fuse) {
    g_err[0] = 0;
    PL_TRY(check_kernel(kernel));
    if (stage < PL_STAGE_LAPLACIAN || stage > PL_STAGE_BILATERAL_SMALL) {
        set_error("unknown stage %d", (int)stage);
        return PL_ERR_ARG;
    }
    const TileCfg c = tile_cfg(static_cast<Stage>(stage), kernel / 2);
    if (tile_rows) *tile_rows = c.th;
    if (tile_cols) *tile_cols = c.tw;
    if (fuse) *fuse = c.fuse;
    return PL_OK;
}

__attribute__((visibility("default"))) pl_status pl_tune_set(pl_stage stage, int32_t kernel,
                                                             int32_t tile_rows,
                                                             int32_t tile_cols, int32_t fuse) {
    g_err[0] = 0;
    PL_TRY(check_kernel(kernel));
    if (stage < PL_STAGE_LAPLACIAN || stage > PL_STAGE_BILATERAL_SMALL) {
        set_error("unknown stage %d", (int)stage);
        return PL_ERR_ARG;
    }
    if (!set_tile_cfg(static_cast<Stage>(stage), kernel / 2,
                      TileCfg{tile_rows, tile_cols, fuse})) {
        set_error("tile %d x %d with %d fused sweeps is outside the kernels' limits", tile_rows,
                  tile_cols, fuse);
        return PL_ERR_ARG;
    }
    return PL_OK;
}

}  // extern "C"

namespace {

struct Span {
    uintptr_t a, b;     // [a, b)
    int frame;
    bool output;
};

// Full validation of a batch's frame list.
pl_status check_batch(const pl_frame *frames, int32_t n, pl_dtype ndt) {
    if (!frames || n < 1) {
        set_error("a batch needs at least one frame");
        return PL_ERR_ARG;
    }
    if (ndt != PL_F32 && ndt != PL_F16) {
        set_error("unknown normal dtype %d", (int)ndt);
        return PL_ERR_ARG;
    }
    std::vector<Span> spans;
    const size_t nb = ndt == PL_F32 ? 4 : 2;
    for (int i = 0; i < n; ++i) {
        const pl_frame &f = frames[i];
        if (pl_status st = check_shape(f.M, f.N)) {
            set_error("frame %d: %s", i, pl_last_error());
            return st;
        }
        if (check_kernel(f.kernel_lap) || check_kernel(f.kernel_bil)) {
            set_error("frame %d: kernel sizes %d / %d must be odd and in [3, 9]", i, f.kernel_lap,
                      f.kernel_bil);
            return PL_ERR_KERNEL;
        }
        if (!(f.lambda >= 0.f && f.lambda <= 1.f) || f.iters_lap < 0 || f.iters_bil < 0 ||
            !(f.sigma_length > 0.f) || !isfinite(f.sigma_length) || !(f.sigma_angle > 0.f) ||
            !isfinite(f.sigma_angle)) {
            set_error("frame %d: lambda, sigmas or sweep counts out of range", i);
            return PL_ERR_ARG;
        }
        const std::pair<const void *, const char *> req[] = {
            {f.pts, "pts"}, {f.pts_out, "pts_out"}, {f.normals, "normals"},
            {f.centroids, "centroids"}, {f.tri_map, "tri_map"}, {f.triangles, "triangles"},
            {f.n_tri, "n_tri"}, {f.normals_T, "normals_T"}};
        for (auto &r : req) {
            if (!r.first || !aligned16(r.first)) {
                set_error("frame %d: %s is NULL or not 16-byte aligned", i, r.second);
                return PL_ERR_ARG;
            }
        }
        if ((f.tri_valid && !aligned16(f.tri_valid)) || (f.halfedges && !aligned16(f.halfedges))) {
            set_error("frame %d: tri_valid / halfedges not 16-byte aligned", i);
            return PL_ERR_ARG;
        }
        if (f.groups) {
            if (!aligned16(f.groups) || f.n_dominant < 0 || f.n_dominant > 254 ||
                (f.n_dominant > 0 && (!f.dominant || !aligned16(f.dominant))) ||
                !(f.l_max >= 0.0f) || isnan(f.ang_min)) {
                set_error("frame %d: group assignment needs 16-byte aligned groups (and "
                          "dominant), 0..254 dominant normals, l_max >= 0 and ang_min a number",
                          i);
                return PL_ERR_ARG;
            }
        }
        const size_t P = (size_t)f.M * f.N, T = 2 * (size_t)(f.M - 1) * (f.N - 1);
        auto add = [&](const void *p, size_t bytes, bool out) {
            if (p && bytes) spans.push_back(Span{(uintptr_t)p, (uintptr_t)p + bytes, i, out});
        };
        add(f.pts, 12 * P, false);
        add(f.pts_out, 12 * P, true);
        add(f.normals, 3 * T * nb, true);
        add(f.centroids, 12 * T, true);
        add(f.tri_valid, T, true);
        add(f.tri_map, 4 * T, true);
        add(f.triangles, 12 * T, true);
        add(f.halfedges, 12 * T, true);
        add(f.n_tri, 4, true);
        add(f.normals_T, 3 * T * nb, true);
        if (f.groups) {
            add(f.groups, T, true);
            add(f.dominant, 12 * (size_t)f.n_dominant, false);
        }
    }
    std::sort(spans.begin(), spans.end(), [](const Span &x, const Span &y) { return x.a < y.a; });
    uintptr_t reach = 0;
    int holder = -1;
    bool holder_out = false;
    for (const Span &sp : spans) {
        // an overlap is allowed only between two inputs (frames may share pts)
        if (holder >= 0 && sp.a < reach && (sp.output || holder_out)) {
            set_error("buffers of frames %d and %d overlap (an output must not overlap anything)",
                      holder, sp.frame);
            return PL_ERR_ALIAS;
        }
        if (sp.b > reach) {
            reach = sp.b;
            holder = sp.frame;
            holder_out = sp.output;
        } else if (sp.output) {
            holder_out = true;
        }
    }
    return PL_OK;
}

pl_status smooth_frame_checked(const pl_frame *frame, pl_dtype ndt, void *ws, size_t ws_bytes,
                               hipStream_t stream, hipEvent_t *events, int32_t n_events,
                               int32_t *kinds, int32_t n_kinds, int32_t *n_launches) {
    g_err[0] = 0;
    PL_TRY(check_batch(frame, 1, ndt));
    const pl_frame &f = *frame;
    const size_t need = smooth_frame_workspace(f, ndt);
    PL_TRY(check_ws(ws, ws_bytes, need));
    const size_t P = (size_t)f.M * f.N, T = 2 * (size_t)(f.M - 1) * (f.N - 1);
    const size_t nb = 3 * T * (ndt == PL_F32 ? 4 : 2);
    const Range wr{ws, need};
    const Range bufs[] = {{f.pts, 12 * P},         {f.pts_out, 12 * P},
                          {f.normals, nb},         {f.centroids, 12 * T},
                          {f.tri_valid, f.tri_valid ? T : 0},
                          {f.tri_map, 4 * T},      {f.triangles, 12 * T},
                          {f.halfedges, f.halfedges ? 12 * T : 0},
                          {f.n_tri, 4},            {f.normals_T, nb},
                          {f.groups, f.groups ? T : 0},
                          {f.dominant, f.groups ? 12 * (size_t)f.n_dominant : 0}};
    for (const Range &b : bufs)
        if (overlap(wr, b)) {
            set_error("the workspace overlaps a buffer of the frame");
            return PL_ERR_ALIAS;
        }
    return launch_smooth_frame(f, ndt, ws, stream, events, n_events, kinds, n_kinds, n_launches);
}

}  // namespace

extern "C" {

__attribute__((visibility("default"))) size_t pl_smooth_frame_workspace(const pl_frame *frame,
                                                                        pl_dtype ndt) {
    if (check_batch(frame, 1, ndt)) return 0;
    return smooth_frame_workspace(*frame, ndt);
}

__attribute__((visibility("default"))) pl_status pl_smooth_frame(const pl_frame *frame,
                                                                 pl_dtype ndt, void *ws,
                                                                 size_t ws_bytes,
                                                                 hipStream_t stream) {
    return smooth_frame_checked(frame, ndt, ws, ws_bytes, stream, nullptr, 0, nullptr, 0,
                                nullptr);
}

__attribute__((visibility("default"))) pl_status pl_smooth_frame_events(
    const pl_frame *frame, pl_dtype ndt, void *ws, size_t ws_bytes, hipEvent_t *events,
    int32_t n_events, int32_t *kinds, int32_t n_kinds, int32_t *n_launches,
    hipStream_t stream) {
    if (n_events < 0 || n_kinds < 0 || (n_events > 0 && !events) || (n_kinds > 0 && !kinds)) {
        g_err[0] = 0;
        set_error("events / kinds: a positive count needs an array");
        return PL_ERR_ARG;
    }
    return smooth_frame_checked(frame, ndt, ws, ws_bytes, stream, events, n_events, kinds,
                                n_kinds, n_launches);
}

__attribute__((visibility("default"))) size_t pl_batch_workspace(const pl_frame *frames,
                                                                 int32_t n, pl_dtype ndt) {
    if (check_batch(frames, n, ndt)) return 0;
    return batch_workspace(frames, n, ndt);
}

__attribute__((visibility("default"))) pl_status pl_batch_create(const pl_frame *frames,
                                                                 int32_t n, pl_dtype ndt,
                                                                 void *ws, size_t ws_bytes,
                                                                 hipStream_t stream,
                                                                 pl_batch *out) {
    g_err[0] = 0;
    if (!out) {
        set_error("out is NULL");
        return PL_ERR_ARG;
    }
    *out = nullptr;
    PL_TRY(check_batch(frames, n, ndt));
    const size_t need = batch_workspace(frames, n, ndt);
    PL_TRY(check_ws(ws, ws_bytes, need));
    const uintptr_t w0 = (uintptr_t)ws, w1 = w0 + need;
    for (int i = 0; i < n; ++i) {
        const pl_frame &f = frames[i];
        const size_t P = (size_t)f.M * f.N;
        const uintptr_t a = (uintptr_t)f.pts;
        if (a < w1 && w0 < a + 12 * P) {
            set_error("frame %d: pts overlaps the workspace", i);
            return PL_ERR_ALIAS;
        }
    }
    return batch_create(frames, n, ndt, ws, stream, out);
}

__attribute__((visibility("default"))) pl_status pl_batch_run(pl_batch batch,
                                                              const uint8_t *active,
                                                              hipStream_t stream) {
    g_err[0] = 0;
    if (!batch) {
        set_error("batch is NULL");
        return PL_ERR_ARG;
    }
    return batch_run(batch, active, stream);
}

__attribute__((visibility("default"))) pl_status pl_batch_capture(pl_batch batch,
                                                                  const uint8_t *active,
                                                                  hipStream_t stream) {
    g_err[0] = 0;
    if (!batch) {
        set_error("batch is NULL");
        return PL_ERR_ARG;
    }
    return batch_capture(batch, active, batch_size(batch), stream);
}

__attribute__((visibility("default"))) pl_status pl_batch_replay(pl_batch batch,
                                                                 hipStream_t stream) {
    g_err[0] = 0;
    if (!batch) {
        set_error("batch is NULL");
        return PL_ERR_ARG;
    }
    return batch_replay(batch, batch_size(batch), stream);
}

__attribute__((visibility("default"))) pl_status pl_batch_capture_bounded(pl_batch batch,
                                                                          const uint8_t *active,
                                                                          int32_t max_active,
                                                                          hipStream_t stream) {
    g_err[0] = 0;
    if (!batch) {
        set_error("batch is NULL");
        return PL_ERR_ARG;
    }
    if (max_active < 1) {
        set_error("max_active must be at least 1, got %d", max_active);
        return PL_ERR_ARG;
    }
    return batch_capture(batch, active, max_active, stream);
}

__attribute__((visibility("default"))) pl_status pl_batch_replay_bounded(pl_batch batch,
                                                                         int32_t n_active,
                                                                         hipStream_t stream) {
    g_err[0] = 0;
    if (!batch) {
        set_error("batch is NULL");
        return PL_ERR_ARG;
    }
    return batch_replay(batch, n_active, stream);
}

__attribute__((visibility("default"))) void pl_batch_destroy(pl_batch batch) {
    batch_destroy(batch);
}

__attribute__((visibility("default"))) pl_status pl_group_assign(
    const float *pts, int32_t n_pts, const int32_t *triangles, const void *normals_T,
    pl_dtype ndt, const int32_t *n_tri, int32_t cap, const float *dominant, int32_t l,
    float l_max, float ang_min, uint8_t *groups, hipStream_t stream) {
    g_err[0] = 0;
    if (ndt != PL_F32 && ndt != PL_F16) {
        set_error("unknown normal dtype %d", (int)ndt);
        return PL_ERR_ARG;
    }
    if (n_pts < 0 || cap < 0) {
        set_error("n_pts %d, cap %d: must not be negative", n_pts, cap);
        return PL_ERR_ARG;
    }
    if (3.0 * (double)cap >= 2147483648.0 || 3.0 * (double)n_pts >= 2147483648.0) {
        set_error("n_pts %d, cap %d: 3 n_pts and 3 cap must stay below 2^31", n_pts, cap);
        return PL_ERR_SHAPE;
    }
    if (l < 0 || l > 254) {
        set_error("%d dominant normals: at most 254 (255 is the sentinel label)", l);
        return PL_ERR_ARG;
    }
    if (!(l_max >= 0.0f) || isnan(ang_min)) {
        set_error("l_max must be >= 0 and ang_min a number (got %g, %g)", (double)l_max,
                  (double)ang_min);
        return PL_ERR_ARG;
    }
    PL_TRY(check_ptrs({{n_tri, "n_tri"}}));
    if (n_pts > 0) PL_TRY(check_ptrs({{pts, "pts"}}));
    if (cap > 0)
        PL_TRY(check_ptrs({{triangles, "triangles"}, {normals_T, "normals_T"},
                           {groups, "groups"}}));
    if (l > 0) PL_TRY(check_ptrs({{dominant, "dominant"}}));
    const Range gr{groups, (size_t)cap};
    const Range ins[] = {{pts, 12 * (size_t)n_pts},
                         {triangles, 12 * (size_t)cap},
                         {normals_T, (size_t)cap * 3 * (ndt == PL_F32 ? 4 : 2)},
                         {n_tri, 4},
                         {dominant, 12 * (size_t)l}};
    for (const Range &r : ins)
        if (overlap(gr, r)) {
            set_error("groups must not overlap an input");
            return PL_ERR_ALIAS;
        }
    return launch_group_assign(pts, n_pts, triangles, normals_T, ndt, n_tri, cap, dominant, l,
                               l_max, ang_min, groups, stream);
}

__attribute__((visibility("default"))) size_t pl_ga_workspace(int32_t level) {
    if (level < 0 || level > kGaMaxLevel) return 0;
    return ga_level_workspace(level);
}

}  // extern "C"

namespace {

pl_status check_cells(const float *cells, int32_t n_cells) {
    if (!cells || n_cells < 1 || n_cells > kGaMaxCells) {
        set_error("cells: need 1..%d host cell normals", kGaMaxCells);
        return PL_ERR_ARG;
    }
    for (int32_t i = 0; i < n_cells; ++i) {
        const double x = cells[3 * i], y = cells[3 * i + 1], z = cells[3 * i + 2];
        const double r = sqrt(x * x + y * y + z * z);
        if (!(fabs(r - 1.0) <= 1e-5)) {
            set_error("cell %d is not a unit vector", i);
            return PL_ERR_ARG;
        }
    }
    return PL_OK;
}

pl_status check_ga_ws(void *ws, size_t ws_bytes, size_t need, hipStream_t stream, pl_ga *out) {
    if (!out) {
        set_error("out is NULL");
        return PL_ERR_ARG;
    }
    *out = nullptr;
    (void)stream;
    return check_ws(ws, ws_bytes, need);
}

}  // namespace

extern "C" {

__attribute__((visibility("default"))) size_t pl_ga_workspace_cells(const float *cells,
                                                                    int32_t n_cells) {
    if (check_cells(cells, n_cells)) return 0;
    return ga_cells_workspace(cells, n_cells);
}

__attribute__((visibility("default"))) pl_status pl_ga_create(int32_t level, void *ws,
                                                              size_t ws_bytes,
                                                              hipStream_t stream, pl_ga *out) {
    g_err[0] = 0;
    if (level < 0 || level > kGaMaxLevel) {
        set_error("level %d: must be in [0, %d]", level, kGaMaxLevel);
        if (out) *out = nullptr;
        return PL_ERR_ARG;
    }
    PL_TRY(check_ga_ws(ws, ws_bytes, ga_level_workspace(level), stream, out));
    return ga_create_level(level, ws, stream, out);
}

__attribute__((visibility("default"))) pl_status pl_ga_create_cells(const float *cells,
                                                                    int32_t n_cells, void *ws,
                                                                    size_t ws_bytes,
                                                                    hipStream_t stream,
                                                                    pl_ga *out) {
    g_err[0] = 0;
    if (out) *out = nullptr;
    PL_TRY(check_cells(cells, n_cells));
    PL_TRY(check_ga_ws(ws, ws_bytes, ga_cells_workspace(cells, n_cells), stream, out));
    return ga_create_cells(cells, n_cells, ws, stream, out);
}

__attribute__((visibility("default"))) int32_t pl_ga_cell_count(pl_ga ga) {
    return ga ? ga_cell_count(ga) : 0;
}

__attribute__((visibility("default"))) const float *pl_ga_cells(pl_ga ga) {
    return ga ? ga_cells(ga) : nullptr;
}

__attribute__((visibility("default"))) pl_status pl_ga_integrate(
    pl_ga ga, const void *normals, pl_dtype ndt, const int32_t *n_normals, int32_t cap,
    int32_t stride, uint32_t *counts, int32_t *cell_out, hipStream_t stream) {
    g_err[0] = 0;
    if (!ga) {
        set_error("ga is NULL");
        return PL_ERR_ARG;
    }
    if (ndt != PL_F32 && ndt != PL_F16) {
        set_error("unknown normal dtype %d", (int)ndt);
        return PL_ERR_ARG;
    }
    if (cap < 0 || stride < 1) {
        set_error("cap %d, stride %d: need cap >= 0 and stride >= 1", cap, stride);
        return PL_ERR_ARG;
    }
    if (3.0 * (double)cap >= 2147483648.0) {
        set_error("cap %d: 3 cap must stay below 2^31", cap);
        return PL_ERR_SHAPE;
    }
    PL_TRY(check_ptrs({{n_normals, "n_normals"}, {counts, "counts"}}));
    if (cap > 0) PL_TRY(check_ptrs({{normals, "normals"}}));
    if (cell_out) PL_TRY(check_ptrs({{cell_out, "cell_out"}}));
    const size_t rows = cap == 0 ? 0 : (size_t)(cap - 1) / stride + 1;
    const Range cr{counts, 4 * (size_t)ga_cell_count(ga)};
    const Range orr{cell_out, 4 * rows};
    const Range ins[] = {{normals, (size_t)cap * 3 * (ndt == PL_F32 ? 4 : 2)},
                         {n_normals, 4},
                         {ga_cells(ga), ga_bytes(ga)}};
    for (const Range &r : ins)
        if (overlap(cr, r) || overlap(orr, r)) {
            set_error("counts and cell_out must not overlap an input or the accumulator");
            return PL_ERR_ALIAS;
        }
    if (overlap(cr, orr)) {
        set_error("counts and cell_out overlap");
        return PL_ERR_ALIAS;
    }
    return ga_integrate(ga, normals, ndt, n_normals, cap, stride, counts, cell_out, stream);
}

__attribute__((visibility("default"))) void pl_ga_destroy(pl_ga ga) { ga_destroy(ga); }

__attribute__((visibility("default"))) size_t pl_user_halfedges_workspace(int32_t cap) {
    if (cap < 0 || 3.0 * (double)cap >= 2147483648.0) return 0;
    return cap == 0 ? 0 : user_halfedges_workspace(cap);
}

__attribute__((visibility("default"))) pl_status pl_user_halfedges(
    const int32_t *triangles, const int32_t *n_tri, int32_t cap, int32_t *halfedges, void *ws,
    size_t ws_bytes, hipStream_t stream) {
    g_err[0] = 0;
    if (cap < 0) {
        set_error("cap %d must not be negative", cap);
        return PL_ERR_ARG;
    }
    if (3.0 * (double)cap >= 2147483648.0) {
        set_error("cap %d: 3 cap must stay below 2^31", cap);
        return PL_ERR_SHAPE;
    }
    PL_TRY(check_ptrs({{n_tri, "n_tri"}}));
    if (cap > 0) PL_TRY(check_ptrs({{triangles, "triangles"}, {halfedges, "halfedges"}}));
    const size_t need = cap == 0 ? 0 : user_halfedges_workspace(cap);
    PL_TRY(check_ws(ws, ws_bytes, need));
    const Range tr{triangles, 12 * (size_t)cap}, nr{n_tri, 4}, hr{halfedges, 12 * (size_t)cap},
        wr{ws, need};
    if (overlap(hr, tr) || overlap(hr, nr) || overlap(hr, wr) || overlap(wr, tr) ||
        overlap(wr, nr)) {
        set_error("halfedges, the workspace and the inputs must not overlap");
        return PL_ERR_ALIAS;
    }
    return launch_user_halfedges(triangles, n_tri, cap, halfedges, ws, stream);
}

__attribute__((visibility("default"))) size_t pl_vertex_update_workspace(int32_t M, int32_t N,
                                                                         int32_t iterations) {
    if (M < 2 || N < 2 || iterations < 0) return 0;
    return vertex_update_workspace(M, N, iterations);
}

__attribute__((visibility("default"))) pl_status pl_vertex_update(
    const float *pts_in, float *pts_out, int32_t M, int32_t N, const void *normals, pl_dtype ndt,
    int32_t iterations, void *ws, size_t ws_bytes, hipStream_t stream) {
    g_err[0] = 0;
    PL_TRY(check_shape(M, N));
    if (ndt != PL_F32 && ndt != PL_F16) {
        set_error("unknown normal dtype %d", (int)ndt);
        return PL_ERR_ARG;
    }
    if (iterations < 0) {
        set_error("iterations %d must not be negative", iterations);
        return PL_ERR_ARG;
    }
    PL_TRY(check_ptrs({{pts_in, "pts_in"}, {pts_out, "pts_out"}, {normals, "normals"}}));
    const size_t need = vertex_update_workspace(M, N, iterations);
    PL_TRY(check_ws(ws, ws_bytes, need));
    const size_t P = (size_t)M * N, T = 2 * (size_t)(M - 1) * (N - 1);
    const Range in{pts_in, 12 * P}, out{pts_out, 12 * P}, nr{normals, T * 3 * (ndt == PL_F32 ? 4 : 2)},
        wr{ws, need};
    if (overlap(in, out) || overlap(out, nr) || overlap(wr, in) || overlap(wr, out) ||
        overlap(wr, nr)) {
        set_error("pts_out and the workspace must not overlap the inputs or each other");
        return PL_ERR_ALIAS;
    }
    return launch_vertex_update(pts_in, pts_out, M, N, normals, ndt, iterations, ws, stream);
}

__attribute__((visibility("default"))) pl_status pl_smooth_batch(const pl_frame *frames, int32_t n,
                                                                 pl_dtype ndt, void *ws,
                                                                 size_t ws_bytes,
                                                                 hipStream_t stream) {
    pl_batch b = nullptr;
    if (pl_status st = pl_batch_create(frames, n, ndt, ws, ws_bytes, stream, &b)) return st;
    const pl_status st = pl_batch_run(b, nullptr, stream);
    pl_batch_destroy(b);          // host-side plan only: the queued run reads `ws`
    return st;
}

}  // extern "C"
