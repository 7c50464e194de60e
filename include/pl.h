/*
 * pl.h -- C ABI of the MI355X (gfx950) organized-point-cloud meshing and
 * smoothing library (libpl.so).
 *
 * The operations are those of Polylidar3D (Castagno & Atkins, arXiv
 * 2007.12065): implicit right-cut meshing of an organized point cloud
 * (Sec. 4.2, Alg. 1 and Alg. 2), the Laplacian vertex filter (Sec. 2.3
 * Eqs. 1-2, applied as in Sec. 5.1), triangle centroids and normals, and the
 * bilateral triangle-normal filter (Sec. 2.3 Eqs. 3-6, applied as in
 * Sec. 5.2) with the gather of filtered normals onto the final mesh.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.   Every array argument is a DEVICE pointer allocated and owned by
 *           the caller; the library never keeps a pointer after a call
 *           returns and allocates no device memory.  Temporary storage is a
 *           caller-provided workspace whose size the matching *_workspace()
 *           function returns (0 means none is needed; ws may then be NULL).
 * Streams.  Every call only enqueues kernels on `stream` (NULL = the null
 *           stream) and returns without synchronising; results are ready when
 *           the stream reaches that point.  Scalars produced on the device
 *           (the triangle count) are written to device memory.
 * Points.   float32, row-major [M][N][3] (x, y, z), flat index i = u*N + v
 *           for row u and column v.  A point is invalid iff any coordinate is
 *           NaN (Sec. 4.2); infinities are outside the contract.
 * Triangles of the implicit full mesh T_FC (Sec. 4.2).  Quad (u, v),
 *           0 <= u < M-1, 0 <= v < N-1, has corners p1 = (u, v),
 *           p2 = (u, v+1), p3 = (u+1, v+1), p4 = (u+1, v).  Its first
 *           triangle (k = 0) is (p3, p2, p1), its second (k = 1) is
 *           (p1, p4, p3); GID = 2 (u (N-1) + v) + k.  Per-triangle arrays
 *           ("T_FC layout") are [M-1][N-1][2][3] in GID order.
 * Alignment. Every array pointer and the workspace must be 16-byte aligned
 *           (device allocations are); PL_ERR_ARG otherwise.
 * Errors.   Arguments are checked before anything is launched; on error
 *           nothing is enqueued and pl_last_error() describes the problem.
 *           PL_ERR_HIP means a launch failed after earlier launches of the
 *           same call may already have been enqueued.
 * Threads.  All entry points are re-entrant.  The error message is
 *           thread-local.
 */
#ifndef PL_H
#define PL_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PL_OK = 0,
    PL_ERR_ARG = -1,       /* NULL required pointer, lambda outside [0, 1],
                              sigma <= 0 or not finite, iterations < 0,
                              cap < 0, unknown dtype, more than 254
                              dominant normals, l_max < 0 or NaN           */
    PL_ERR_SHAPE = -2,     /* M < 2 or N < 2, or 6 (M-1)(N-1) >= 2^31;
                              for group assignment 3 n_pts or 3 cap >= 2^31 */
    PL_ERR_KERNEL = -3,    /* kernel size even, < 3 or > 9                  */
    PL_ERR_ALIAS = -4,     /* an output overlaps an input (Jacobi semantics) */
    PL_ERR_WORKSPACE = -5, /* ws NULL or ws_bytes below the required size   */
    PL_ERR_HIP = -6        /* a HIP launch failed                           */
} pl_status;

/* Storage type of triangle normals.  Arithmetic is float32 either way. */
/* Storage type of the normals.  A plain int32_t, not an enum type, so that a
   value outside the list reaches the library's check (PL_ERR_ARG) as it is. */
typedef int32_t pl_dtype;
enum { PL_F32 = 0, PL_F16 = 1 };

/* Version of this ABI (major * 100 + minor). */
int32_t pl_version(void);

/* Description of the last error on the calling thread ("" if none). */
const char *pl_last_error(void);

/*
 * Mesh extraction, Sec. 4.2: Alg. 1 (Extract Triangles from OPC) and Alg. 2
 * (Extract Half-Edges from OPC).
 *
 * pts        [M][N][3] float32 points, NaN = invalid.
 * tri_valid  optional (may be NULL): uint8 [2(M-1)(N-1)] in GID order,
 *            1 iff all three vertices of that T_FC triangle are valid.
 * tri_map    int32 [2(M-1)(N-1)]: T_map of Alg. 1, the index of each GID in
 *            T, or -1 if that triangle is not in T.
 * triangles  int32 [cap][3]: T, the valid triangles in increasing GID order,
 *            each as three flat point indices in the order above.
 * halfedges  optional (may be NULL): int32 [3 cap]: HE of Alg. 2; entry
 *            3t + j is the twin of half-edge j of triangle t (j runs from
 *            vertex j to vertex (j+1) mod 3), or -1 on a border.
 * cap        capacity of triangles/halfedges in triangles; 2(M-1)(N-1)
 *            always suffices.  Only triangles with index < cap are written;
 *            *n_tri still receives the full count, so *n_tri > cap reports
 *            truncation (twin indices may then refer to triangles >= cap).
 * n_tri      int32 device scalar: |T|.
 * Workspace: pl_mesh_opc_workspace(M, N) bytes.
 * Outputs are bit-exact and deterministic (an ordered compaction, no
 * atomics).
 */
size_t pl_mesh_opc_workspace(int32_t M, int32_t N);
pl_status pl_mesh_opc(const float *pts, int32_t M, int32_t N,
                      uint8_t *tri_valid, int32_t *tri_map, int32_t *triangles,
                      int32_t *halfedges, int32_t cap, int32_t *n_tri,
                      void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * pl_mesh_opc without a workspace, for callers that cannot allocate device
 * memory: code being captured into a HIP graph, tight serving loops, and
 * harnesses that forbid allocation.  Arguments, outputs and errors are those
 * of pl_mesh_opc, whose outputs it reproduces bit for bit; the validity codes
 * and segment counts that pl_mesh_opc keeps in the workspace live instead in
 * a static device array of 8 MiB (one per GPU, held until the process ends,
 * its address looked up on the first call on that GPU).
 * Limit: frames with pl_mesh_opc_workspace(M, N) <= 8 MiB (about 8.3
 * million quads, e.g. 2000 x 4096); larger frames get PL_ERR_SHAPE and
 * nothing is enqueued.  The call allocates nothing and writes no memory the
 * caller did not pass except that array; nothing in it needs clearing (every
 * code and count a call reads, the same call writes first).
 * Calls that overlap in time on one GPU (on different streams, or from
 * different threads) share the array and race: order them on one stream.
 * `stream` must belong to a device in 0..63.
 */
pl_status pl_mesh_opc_static(const float *pts, int32_t M, int32_t N,
                             uint8_t *tri_valid, int32_t *tri_map, int32_t *triangles,
                             int32_t *halfedges, int32_t cap, int32_t *n_tri,
                             hipStream_t stream);

/*
 * Laplacian vertex filter, Sec. 2.3 Eqs. (1)-(2) on the image-space
 * neighbourhood of Sec. 5.1, `iterations` Jacobi sweeps:
 *     v_o = v_i + lambda * sum_j w_j (v_j - v_i) / sum_j w_j,
 *     w_j = 1 / ||v_j - v_i||,
 * over the valid pixels j != i of the kernel x kernel window around i.
 * Neighbours at distance 0 are skipped; a pixel with no usable neighbour
 * keeps its value.  Invalid pixels and pixels within kernel/2 of the image
 * border are copied unchanged (bitwise).
 *
 * pts_in/pts_out  [M][N][3] float32; must not overlap.
 * kernel          odd window size, 3..9.
 * lambda          in [0, 1].
 * iterations      >= 0; 0 copies pts_in to pts_out.
 * Workspace: pl_laplacian_workspace(M, N, iterations) bytes.
 */
size_t pl_laplacian_workspace(int32_t M, int32_t N, int32_t iterations);

/* Sweeps the library fuses into one kernel launch for this window size
 * (ceil(iterations / this) launches per pl_laplacian call); 0 if the kernel
 * size is invalid.  Informational: results do not depend on it. */
int32_t pl_laplacian_fused_sweeps(int32_t kernel);

pl_status pl_laplacian(const float *pts_in, float *pts_out, int32_t M, int32_t N,
                       int32_t kernel, float lambda, int32_t iterations,
                       void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Triangle centroids and normals over T_FC, Sec. 5.2.  For each triangle
 * with vertices (a, b, c) in the order above:
 *     centroid = (a + b + c) / 3,   normal = (b - a) x (c - a) / ||.||.
 * Both are NaN if any vertex is invalid; the normal is NaN if the cross
 * product is zero.
 *
 * pts        [M][N][3] float32.
 * normals    T_FC layout, float32 [..][3] (ndt = PL_F32) or float16 [..][3]
 *            (ndt = PL_F16, rounded to nearest from the float32 result).
 * centroids  T_FC layout float32 [..][3].
 */
pl_status pl_tri_normals(const float *pts, int32_t M, int32_t N,
                         void *normals, pl_dtype ndt, float *centroids,
                         hipStream_t stream);

/*
 * Bilateral normal filter, Sec. 2.3 Eqs. (3)-(6) on the organized mesh of
 * Sec. 5.2, `iterations` Jacobi sweeps over the normals (centroids fixed):
 *     n_o = normalize( sum_j exp(-||c_i - c_j||^2 / (2 sigma_length^2)
 *                               -||n_i - n_j||^2 / (2 sigma_angle^2)) n_j ).
 * Neighbours of t_{u,v,k}: both triangles of every other quad (u+du, v+dv),
 * |du|, |dv| <= kernel/2, (du, dv) != (0, 0), on the grid, whose normal and
 * centroid are free of NaN (16 at kernel 3).  The result is renormalised to
 * unit length (the constant of Eq. 6 cancels); a triangle without
 * neighbours, or whose weighted sum vanishes, keeps its normal; a triangle
 * whose own normal or centroid holds a NaN is copied unchanged.
 *
 * normals_in   T_FC layout, storage type ndt.
 * centroids    T_FC layout float32.
 * normals_out  T_FC layout, storage type ndt; must not overlap the inputs.
 * tri_map      optional (NULL = no gather): T_map from pl_mesh_opc.
 * normals_T    required iff tri_map is given: [2(M-1)(N-1)][3] of type ndt;
 *              row T_map[g] receives the filtered normal of GID g for every
 *              g with T_map[g] >= 0 (Sec. 5.2); rows >= |T| are untouched.
 * kernel       odd window size in quads, 3..9.
 * sigma_length, sigma_angle  finite and > 0.
 * iterations   >= 0; 0 copies normals_in to normals_out (and gathers).
 * Workspace: pl_bilateral_workspace(M, N, ndt, iterations) bytes.
 */
size_t pl_bilateral_workspace(int32_t M, int32_t N, pl_dtype ndt, int32_t iterations);
pl_status pl_bilateral(const void *normals_in, const float *centroids, pl_dtype ndt,
                       int32_t M, int32_t N, int32_t kernel,
                       float sigma_length, float sigma_angle, int32_t iterations,
                       void *normals_out, const int32_t *tri_map, void *normals_T,
                       void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Group assignment, Sec. 7.1 Alg. 4: a label per triangle of T for the
 * planar segmentation.  Triangle t gets the index j of the dominant normal
 * n^d_j with the largest similarity n_t . n^d_j (the first such j among
 * equals), or 255 ("no group") when one of its edges is longer than l_max,
 * when that similarity is below ang_min, or when there is no dominant normal.
 * The comparisons are taken in float32 on the float32 values (float16
 * normals are widened exactly):
 *     edge test   fma(dx,dx, fma(dy,dy, dz*dz)) <= l_max*l_max for all
 *                 three edges, d = difference of the edge's endpoints;
 *                 a NaN coordinate fails it,
 *     similarity  fma(nx,djx, fma(ny,djy, nz*djz)), strict > against the
 *                 running best (which starts at -1),
 * so the labels are a function of the inputs alone.  A NaN normal gets 255;
 * a triangle with a vertex index outside [0, n_pts) gets 255.
 *
 * pts        float32 [n_pts][3]: the vertices (for a frame, the smoothed
 *            points [M][N][3], n_pts = M N).
 * triangles  int32 [cap][3]: T (pl_mesh_opc's layout).
 * normals_T  [cap][3] of type ndt: row t is the normal of triangle t
 *            (pl_bilateral's gathered output).
 * n_tri      int32 DEVICE scalar: |T|; rows t with
 *            t < min(*n_tri, cap) are labelled, the rest of `groups` is
 *            left untouched (read when the kernel runs, so the call can
 *            follow pl_mesh_opc on the same stream without a host sync).
 * cap        rows of triangles / normals_T / groups; 0 enqueues nothing.
 * dominant   float32 [l][3] device array of dominant unit normals, used as
 *            given; may be NULL when l = 0.
 * l          0..254.
 * l_max      >= 0 (may be +inf); ang_min any number but NaN.
 * groups     uint8 [cap] output; must not overlap an input.
 * All arrays are device memory owned by the caller; pts may be NULL when
 * n_pts = 0, and triangles, normals_T and groups when cap = 0.  No workspace, no
 * allocation; stream-ordered.  PL_ERR_ARG / PL_ERR_SHAPE / PL_ERR_ALIAS on
 * invalid arguments (nothing enqueued).
 */
pl_status pl_group_assign(const float *pts, int32_t n_pts, const int32_t *triangles,
                          const void *normals_T, pl_dtype ndt, const int32_t *n_tri,
                          int32_t cap, const float *dominant, int32_t l, float l_max,
                          float ang_min, uint8_t *groups, hipStream_t stream);

/*
 * Vertex update from filtered normals: the second stage of the bilateral
 * mesh denoising the paper cites with Eqs. (3)-(6) (Sun et al., 2007); the
 * paper itself skips it (Sec. 5.2) and prints no formula.  `iterations`
 * Jacobi sweeps of
 *     x_i <- x_i + (1 / |F_i|) sum_{f in F_i} n_f (n_f . (c_f - x_i)),
 * F_i the triangles of T_FC containing vertex i whose three vertices are
 * valid and whose normal n_f (from `normals`, fixed) has no NaN, c_f their
 * centroids from the current vertices.  An invalid point, or a vertex with
 * no such triangle, keeps its value (bitwise).
 *
 * pts_in/pts_out  [M][N][3] float32; must not overlap.
 * normals         T_FC layout of type ndt (e.g. pl_bilateral's output).
 * iterations      >= 0; 0 copies pts_in to pts_out.
 * Workspace: pl_vertex_update_workspace(M, N, iterations) bytes (one point
 * buffer when iterations > 1).
 */
size_t pl_vertex_update_workspace(int32_t M, int32_t N, int32_t iterations);
pl_status pl_vertex_update(const float *pts_in, float *pts_out, int32_t M, int32_t N,
                           const void *normals, pl_dtype ndt, int32_t iterations, void *ws,
                           size_t ws_bytes, hipStream_t stream);

/*
 * Half-edges of a user-provided mesh, Sec. 4.3: the twin of every half-edge
 * of T found through a hash table keyed by ordered point pairs.
 *
 * Half-edge 3t + j of triangle t runs from vertex j to vertex (j+1) mod 3;
 * its twin is a half-edge running the other way between the same two
 * points.  Edges shared by more than two triangles (meshes that violate the
 * second manifold condition) take the paper's option 1, keep the first pair:
 * half-edge h = (a, b) is paired only if no lower-indexed half-edge is also
 * (a, b), and then with the lowest-indexed half-edge (b, a) if there is one.
 * Half-edges from a point to itself are never paired.  The pairing is
 * symmetric, and on a two-manifold mesh it is the usual twin map (on
 * pl_mesh_opc's T it equals that call's HE).  The output is deterministic.
 *
 * triangles  int32 [cap][3] point indices (any int32 values; no point array
 *            is needed).
 * n_tri      int32 DEVICE scalar: |T|; triangles t < min(*n_tri, cap) are
 *            processed (e.g. pl_mesh_opc's count).
 * halfedges  int32 [3 cap] output; entries at or past 3 min(*n_tri, cap) are
 *            left untouched.
 * Workspace: pl_user_halfedges_workspace(cap) bytes, 0 when cap = 0.  Up
 * to 5.6 M triangles the edges are dealt to 2^k buckets by hash (2^k the
 * power of two at or above 3 cap / 2048) and each bucket is solved in one
 * workgroup's LDS: the workspace holds per-chunk bucket counts and starts,
 * bucket regions of 3072 entries of 12 bytes and an overflow list of 3 cap
 * entries (about 100 bytes per triangle at cap = 612k); five launches.
 * Larger capacities use one hash table of 4 cap slots of 16 bytes and a
 * slot index per half-edge; three launches.  PL_ERR_ARG / PL_ERR_SHAPE /
 * PL_ERR_WORKSPACE / PL_ERR_ALIAS on invalid arguments (nothing enqueued).
 * No allocation, graph-capturable (the workspace needs no clearing).
 */
size_t pl_user_halfedges_workspace(int32_t cap);
pl_status pl_user_halfedges(const int32_t *triangles, const int32_t *n_tri, int32_t cap,
                            int32_t *halfedges, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Gaussian accumulator, Sec. 6.1: the cells of a refined icosahedron
 * (Sec. 6.1.1, Table 1) and the integration of normals into them (Alg. 3).
 *
 * Level L (0..5) has 20 * 4^L triangular cells; each cell's surface normal is
 * the outward unit normal of its plane.  Integration adds one to the count of
 * the cell whose normal is nearest to each integrated normal: squared
 * Euclidean distance in float32, d = c - n,
 *     |d|^2 = fma(dx, dx, fma(dy, dy, dz * dz)),
 * the lowest cell index among equals.  The result is exactly that of a
 * brute-force search over all cells (the library finds the cell through a
 * precomputed table of candidates per direction bin, or over all cells for
 * normals whose length is outside [0.5, 2]).  A normal with a NaN or
 * infinite coordinate lands in no cell.
 *
 * pl_ga_workspace(level)      bytes of device workspace for a level-L
 *                             accumulator (0 if L is outside 0..5).  The
 *                             first call for a level builds its tables on
 *                             the host (tens of milliseconds at level 4);
 *                             they are kept for the process.
 * pl_ga_workspace_cells       the same for caller-given cell normals
 *                             (host float32 [n_cells][3], 1 <= n_cells <=
 *                             32768, each of unit length within 1e-5).
 * pl_ga_create[_cells]        uploads the cells and tables into `ws` (which
 *                             must stay allocated and untouched until
 *                             pl_ga_destroy); synchronises `stream` once.
 * pl_ga_cell_count, pl_ga_cells  the number of cells and a device pointer to
 *                             their normals, float32 [n_cells][3] inside ws.
 * pl_ga_integrate             integrates rows 0, stride, 2 stride, ... below
 *                             min(*n_normals, cap) of `normals` ([cap][3],
 *                             type ndt, device): counts (uint32 [n_cells],
 *                             device) are ADDED to (clear them first for a
 *                             fresh histogram); cell_out (optional, int32
 *                             [ceil(cap / stride)]) receives row j's cell (or
 *                             -1) at index j / stride for every integrated
 *                             row.  n_normals is an int32 device scalar (e.g.
 *                             pl_mesh_opc's |T| with normals_T).  No
 *                             allocation; stream-ordered.
 * pl_ga_destroy               releases the host-side handle.
 * Integrations through one accumulator must not overlap in time (they share
 * its scratch histograms in ws); different accumulators may add into the
 * same counts concurrently (atomic adds).
 */
typedef struct pl_ga_s *pl_ga;
size_t pl_ga_workspace(int32_t level);
size_t pl_ga_workspace_cells(const float *cells, int32_t n_cells);
pl_status pl_ga_create(int32_t level, void *ws, size_t ws_bytes, hipStream_t stream, pl_ga *out);
pl_status pl_ga_create_cells(const float *cells, int32_t n_cells, void *ws, size_t ws_bytes,
                             hipStream_t stream, pl_ga *out);
int32_t pl_ga_cell_count(pl_ga ga);
const float *pl_ga_cells(pl_ga ga);
pl_status pl_ga_integrate(pl_ga ga, const void *normals, pl_dtype ndt, const int32_t *n_normals,
                          int32_t cap, int32_t stride, uint32_t *counts, int32_t *cell_out,
                          hipStream_t stream);
void pl_ga_destroy(pl_ga ga);

/*
 * Tile shapes and sweep fusion ("tuning").  Every stage runs its kernel
 * over tiles of tile_rows x tile_cols (points for the Laplacian, quads for
 * the bilateral) and fuses up to `fuse` sweeps per launch.  float32 results
 * do not depend on these values (the arithmetic of every output is the same
 * whatever the tiling), and float16 results do not depend on `fuse`.  The
 * single-frame calls read the PL_STAGE_LAPLACIAN / PL_STAGE_BILATERAL
 * entries, or the PL_STAGE_*_SMALL ones for frames of at most 131072 points
 * (M * N <= 2^17: a 64 x 1024 frame fills the chip with other shapes than a
 * 480 x 640 one); batch plans read the PL_STAGE_BATCH_* entries when they
 * are created (a launch over many frames favours other shapes than one over
 * a single frame).  pl_laplacian_fused_sweeps reports the large-frame
 * entry.  The table is process-wide; pl_tune_set is meant for a
 * tuner run before work is enqueued (it does not affect launches already
 * enqueued or plans already created).
 * kernel      odd window size, 3..9.
 * tile_rows * tile_cols <= 16384; the LDS the shape needs must fit 156 KB.
 * Returns PL_ERR_KERNEL / PL_ERR_ARG for an invalid request.
 */
typedef int32_t pl_stage;     /* one of the values below (PL_ERR_ARG otherwise) */
enum {
    PL_STAGE_LAPLACIAN = 0,
    PL_STAGE_BILATERAL = 1,
    PL_STAGE_BATCH_LAPLACIAN = 2,
    PL_STAGE_BATCH_BILATERAL = 3,
    PL_STAGE_LAPLACIAN_SMALL = 4,
    PL_STAGE_BILATERAL_SMALL = 5
};
pl_status pl_tune_get(pl_stage stage, int32_t kernel, int32_t *tile_rows, int32_t *tile_cols,
                      int32_t *fuse);
pl_status pl_tune_set(pl_stage stage, int32_t kernel, int32_t tile_rows, int32_t tile_cols,
                      int32_t fuse);

/*
 * Batched path: a set of frames of any sizes and filter settings through the
 * whole pipeline (mesh, Laplacian, normals, bilateral, gather) with one
 * launch per stage (per sweep pass for the filters) over a tile queue built
 * on the device from the active frames.  Each frame's outputs
 * are exactly those of the single-frame calls with the same parameters:
 *   pl_mesh_opc(pts, M, N, tri_valid, tri_map, triangles, halfedges,
 *               cap = 2(M-1)(N-1), n_tri)
 *   pl_laplacian(pts -> pts_out, kernel_lap, lambda, iters_lap)
 *   pl_tri_normals(pts_out -> normals before filtering, centroids)
 *   pl_bilateral(-> normals, kernel_bil, sigma_length, sigma_angle,
 *                iters_bil, tri_map -> normals_T)
 *   pl_group_assign(pts_out, M N, triangles, normals_T, n_tri,
 *                   cap = 2(M-1)(N-1), dominant, n_dominant, l_max,
 *                   ang_min -> groups)       (only if groups != NULL)
 * All pointers are device pointers owned by the caller, 16-byte aligned,
 * with the sizes of the single-frame calls (triangles [2(M-1)(N-1)][3],
 * halfedges [6(M-1)(N-1)], normals / normals_T in the batch's dtype);
 * tri_valid and halfedges may be NULL.  No output may overlap any input or
 * any other output of the batch.
 *
 * pl_batch_workspace  bytes of workspace the batch needs (0 if the frame
 *                     list is invalid); depends on the tuning table.
 * pl_batch_create     validates the frames, builds the plan in `ws` (which
 *                     must stay allocated and untouched until
 *                     pl_batch_destroy) and uploads its tables; synchronises
 *                     `stream` once.  The frames' buffers are bound to the
 *                     plan: later runs read and write the same addresses.
 * pl_batch_run        enqueues one pass of the whole pipeline on `stream`
 *                     over the frames i with active[i] != 0, where `active`
 *                     is a DEVICE array of n bytes read when the run
 *                     executes (NULL = every frame).  Frames left out keep
 *                     their previous outputs.  Device-only work: no
 *                     allocation, no synchronisation, legal under capture.
 * pl_batch_capture    records pl_batch_run(active) into a HIP graph owned by
 *                     the plan (replacing the previous such graph);
 *                     pl_batch_replay launches it on `stream`.  The graph
 *                     reads the mask's contents at replay time, so one graph
 *                     serves any subset of the plan's frames.
 * pl_batch_capture_bounded  the same for replays in which at most
 *                     `max_active` (>= 1) frames are active: every launch is
 *                     sized for the max_active frames with the most tiles in
 *                     its stage, so a step over few frames does not dispatch
 *                     the idle frames' workgroups.  The plan keeps one graph
 *                     per bound (capturing a bound again replaces it; bounds
 *                     above the frame count mean all frames).
 * pl_batch_replay_bounded   launches the graph with the smallest captured
 *                     bound >= n_active (PL_ERR_ARG if there is none).  The
 *                     caller guarantees that at most n_active frames are
 *                     active in the mask: tiles past a launch's workgroups
 *                     would go unprocessed.
 * pl_batch_destroy    releases the host-side plan (and its graph).
 * Runs of one plan must not overlap in time (they share the queue counters
 * and scratch in `ws`).
 */
typedef struct {
    const float *pts;          /* [M][N][3] input points                     */
    int32_t M, N;
    int32_t kernel_lap, iters_lap;
    float lambda;
    int32_t kernel_bil, iters_bil;
    float sigma_length, sigma_angle;
    float *pts_out;            /* [M][N][3] smoothed points                  */
    void *normals;             /* T_FC layout, filtered normals              */
    float *centroids;          /* T_FC layout                                */
    uint8_t *tri_valid;        /* optional [2(M-1)(N-1)]                     */
    int32_t *tri_map;          /* [2(M-1)(N-1)]                              */
    int32_t *triangles;        /* [2(M-1)(N-1)][3]                           */
    int32_t *halfedges;        /* optional [6(M-1)(N-1)]                     */
    int32_t *n_tri;            /* device scalar                              */
    void *normals_T;           /* [2(M-1)(N-1)][3]                           */
    /* Optional group assignment (pl_group_assign on this frame's smoothed
       points, T and normals_T): groups NULL leaves it out.                 */
    const float *dominant;     /* [n_dominant][3]; may be NULL if none        */
    int32_t n_dominant;        /* 0..254                                     */
    float l_max, ang_min;      /* l_max >= 0, ang_min not NaN                */
    uint8_t *groups;           /* [2(M-1)(N-1)]: rows < |T| receive labels   */
} pl_frame;

typedef struct pl_batch_s *pl_batch;

size_t pl_batch_workspace(const pl_frame *frames, int32_t n, pl_dtype ndt);
pl_status pl_batch_create(const pl_frame *frames, int32_t n, pl_dtype ndt, void *ws,
                          size_t ws_bytes, hipStream_t stream, pl_batch *out);
pl_status pl_batch_run(pl_batch batch, const uint8_t *active, hipStream_t stream);
pl_status pl_batch_capture(pl_batch batch, const uint8_t *active, hipStream_t stream);
pl_status pl_batch_replay(pl_batch batch, hipStream_t stream);
pl_status pl_batch_capture_bounded(pl_batch batch, const uint8_t *active, int32_t max_active,
                                   hipStream_t stream);
pl_status pl_batch_replay_bounded(pl_batch batch, int32_t n_active, hipStream_t stream);

/*
 * The whole path on ONE frame in as few kernel launches as its dependencies
 * allow: mesh (Sec. 4.2, Alg. 1 and Alg. 2), Laplacian (Sec. 2.3 Eqs. 1-2,
 * Sec. 5.1), centroids and normals, bilateral filter and the gather onto T
 * (Eqs. 3-6, Sec. 5.2), and the group labels of Alg. 4 (Sec. 7.1) when
 * frame->groups is set.  The outputs are exactly those of the single-frame
 * calls listed for the batched path below (pl_mesh_opc, pl_laplacian,
 * pl_tri_normals, pl_bilateral with the gather, pl_group_assign), bit for
 * bit; frame->normals receives the FILTERED normals (T_FC layout) and the
 * unfiltered normals are not stored.  The mesh's validity pass runs in the
 * same launch as the Laplacian's first pass, the mesh emit in the launch
 * after it (whose gather, if it is the last bilateral pass, ranks the
 * triangles in T from the validity codes instead of reading T_map), and the
 * first bilateral pass computes the normals and centroids itself: one
 * launch per filter pass (a 480 x 640 frame with the committed tuning: 3
 * launches instead of 6; a 120 x 160 frame: 2).
 *
 * frame      HOST pointer to one pl_frame (the layout is documented with the
 *            batched path below); its buffers are device memory owned by
 *            the caller, 16-byte aligned, sized as listed there.
 * ndt        storage type of the normals.
 * ws         pl_smooth_frame_workspace(frame, ndt) bytes of device memory
 *            (codes and counts of the mesh, ping-pong buffers when a filter
 *            takes more than one sweep); must not overlap the frame's
 *            buffers.  pl_smooth_frame_workspace returns 0 for an invalid
 *            frame.
 * Errors are those of pl_batch_create for a one-frame list, plus
 * PL_ERR_WORKSPACE.  Device-only work on `stream`: no allocation, no
 * synchronisation, legal under graph capture.
 */
size_t pl_smooth_frame_workspace(const pl_frame *frame, pl_dtype ndt);
pl_status pl_smooth_frame(const pl_frame *frame, pl_dtype ndt, void *ws, size_t ws_bytes,
                          hipStream_t stream);

/*
 * Measurement form of pl_smooth_frame, for profilers and benchmarks: the
 * same work on `stream`, with events[0] recorded before the first launch and
 * events[k] after launch k (as many as n_events allows; the events are
 * created by the caller, hipEventCreate), and kinds[k-1] (HOST array of
 * n_kinds entries, may be NULL) describing launch k: PL_LAUNCH_* bits of the
 * work it carries and, in bits 8..15, the number of filter sweeps it fuses.
 * *n_launches (HOST, may be NULL) receives the number of launches.  A frame
 * meshed by whole rows reports pl_mesh_opc's two launches as one count and
 * one emit launch.  Recording events costs the stream a few microseconds
 * each, so the per-launch durations are upper bounds.
 * Errors: those of pl_smooth_frame; PL_ERR_ARG for a negative count or a
 * positive count with a NULL array.
 */
enum {
    PL_LAUNCH_LAPLACIAN = 1,     /* Laplacian sweeps over point tiles       */
    PL_LAUNCH_BILATERAL = 2,     /* bilateral sweeps over quad tiles        */
    PL_LAUNCH_NORMALS = 4,       /* centroids and normals from the points  */
    PL_LAUNCH_GATHER = 8,        /* filtered normals gathered onto T       */
    PL_LAUNCH_MESH_COUNT = 16,   /* validity codes and counts (a1)         */
    PL_LAUNCH_MESH_EMIT = 32,    /* T_map, T, HE (a2, a3)                  */
    PL_LAUNCH_GROUPS = 64        /* group assignment (Alg. 4)              */
};
pl_status pl_smooth_frame_events(const pl_frame *frame, pl_dtype ndt, void *ws, size_t ws_bytes,
                                 hipEvent_t *events, int32_t n_events, int32_t *kinds,
                                 int32_t n_kinds, int32_t *n_launches, hipStream_t stream);

/*
 * One-shot form for callers that run a frame list once: pl_batch_create,
 * pl_batch_run over all frames, pl_batch_destroy.  `ws` holds
 * pl_batch_workspace(frames, n, ndt) bytes and must stay allocated and
 * untouched until the enqueued run has completed on `stream`.  Synchronises
 * `stream` once (the plan's table upload), like pl_batch_create.
 */
pl_status pl_smooth_batch(const pl_frame *frames, int32_t n, pl_dtype ndt, void *ws,
                          size_t ws_bytes, hipStream_t stream);
void pl_batch_destroy(pl_batch batch);

#ifdef __cplusplus
}
#endif

#endif /* PL_H */
