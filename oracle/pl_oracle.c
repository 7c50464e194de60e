/*
 * FP64 CPU oracle for organized-point-cloud meshing and smoothing
 * (Polylidar3D, Castagno & Atkins, arXiv 2007.12065).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header or
 * constant with the HIP library, and the HIP library never calls it.
 *
 * Every floating-point step runs in double precision on double inputs (the
 * caller promotes the float32 frame), except in group assignment and in the
 * Gaussian accumulator's integration, whose comparisons decide an integer
 * label or cell and are taken in float32 (see there).  Loops follow the paper's definitions
 * directly; the only parallelism is an OpenMP loop over independent outputs,
 * so results do not depend on the thread count.
 *
 * Readings of points the paper leaves open are marked "Reading:" below.
 *
 * Parity unpinned: oracle_vertex_update.  The paper names the vertex update
 * of the method it cites but gives no formula for it; the routine restates
 * that published update, and its pins (closed forms, invariants) check the
 * restatement, not a result printed in the paper.  Every other routine is
 * pinned to values or properties the paper and the mathematics fix.
 *
 * Grid conventions (Sec. 3, Sec. 4.2): points p[u][v], u = row in [0, M),
 * v = column in [0, N), flat index i = u*N + v, 3 doubles per point.  Quad
 * (u, v) with u < M-1, v < N-1 holds the corners
 *     p1 = (u, v), p2 = (u, v+1), p3 = (u+1, v+1), p4 = (u+1, v)
 * Reading: the paper leaves GetPointIndices undefined; this is the labelling
 * under which the twin links of Alg. 2 (Right/Top/Left/Bottom) are true
 * twins and the triangles wind counter-clockwise as displayed, with the cut
 * along p1-p3.  The first triangle (k = 0) is (p3, p2, p1), the second
 * (k = 1) is (p1, p4, p3), and the global id of t_{u,v,k} is
 * GID = 2 (u (N-1) + v) + k.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_EXPORT __attribute__((visibility("default")))

static int point_valid(const double *p)
{
    /* A point is valid iff none of its coordinates is NaN (Sec. 4.2). */
    return !(isnan(p[0]) || isnan(p[1]) || isnan(p[2]));
}

static void quad_corners(int u, int v, int N, int64_t c[5])
{
    /* c[1..4] = flat indices of p1..p4 of quad (u, v); c[0] unused. */
    c[0] = -1;
    c[1] = (int64_t)u * N + v;
    c[2] = (int64_t)u * N + v + 1;
    c[3] = (int64_t)(u + 1) * N + v + 1;
    c[4] = (int64_t)(u + 1) * N + v;
}

/* Vertex indices of t_{u,v,k} in Alg. 1's order. */
static void tri_vertices(int u, int v, int k, int N, int64_t out[3])
{
    int64_t c[5];
    quad_corners(u, v, N, c);
    if (k == 0) { out[0] = c[3]; out[1] = c[2]; out[2] = c[1]; }
    else        { out[0] = c[1]; out[1] = c[4]; out[2] = c[3]; }
}

/* A triangle of T_FC is valid iff its three vertices are (Sec. 4.2). */
static int gid_valid(const double *pts, int64_t g, int Nq, int N)
{
    const int64_t q = g / 2;
    const int u = (int)(q / Nq), v = (int)(q % Nq);
    int64_t vert[3];
    tri_vertices(u, v, (int)(g % 2), N, vert);
    return point_valid(pts + 3 * vert[0]) && point_valid(pts + 3 * vert[1]) &&
           point_valid(pts + 3 * vert[2]);
}

/*
 * T and T_map, Sec. 4.2 (computed by Alg. 1): T lists the valid triangles of
 * T_FC in increasing GID, each as its three point indices in the order
 * above, and T_map sends a GID to its position in T (-1 if not valid).
 * Written as that definition: validity per GID, then the rank of each valid
 * GID among the valid GIDs before it, then T filled at those ranks.
 * pts:       [M*N*3] doubles.
 * tri_map:   [2(M-1)(N-1)] out.
 * triangles: [3 * 2(M-1)(N-1)] out (the first |T| rows are set).
 * Returns |T|.
 */
OR_EXPORT int64_t oracle_mesh_triangles(const double *pts, int M, int N,
                                        int32_t *tri_map, int32_t *triangles)
{
    const int Mq = M - 1, Nq = N - 1;
    const int64_t n_gid = 2LL * Mq * Nq;
    int64_t rank = 0;
    for (int64_t g = 0; g < n_gid; ++g)
        tri_map[g] = gid_valid(pts, g, Nq, N) ? (int32_t)rank++ : -1;
    for (int64_t g = 0; g < n_gid; ++g) {
        if (tri_map[g] < 0) continue;
        const int64_t q = g / 2;
        int64_t vert[3];
        tri_vertices((int)(q / Nq), (int)(q % Nq), (int)(g % 2), N, vert);
        for (int j = 0; j < 3; ++j) triangles[3LL * tri_map[g] + j] = (int32_t)vert[j];
    }
    return rank;
}

/* Half-edge records keyed by their ordered point pair (a, b), for the twin
 * search by reversed pairs (Sec. 4.3). */
typedef struct {
    uint64_t key;
    int64_t id;
} he_rec;

static uint64_t he_key(int32_t a, int32_t b) { return ((uint64_t)(uint32_t)a << 32) | (uint32_t)b; }

static int he_cmp(const void *x, const void *y)
{
    const he_rec *p = (const he_rec *)x, *q = (const he_rec *)y;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return p->id < q->id ? -1 : (p->id > q->id);
}

/* Lowest half-edge id keyed `key` in the sorted records, or -1. */
static int64_t he_first(const he_rec *r, int64_t n, uint64_t key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (r[mid].key < key) lo = mid + 1; else hi = mid;
    }
    return (lo < n && r[lo].key == key) ? r[lo].id : -1;
}

/*
 * Twins of the half-edges of a triangle list by their definition (Sec. 3,
 * Sec. 4.3): half-edge 3t + j runs from vertex j to vertex (j+1) mod 3 of
 * triangle t, and its twin is a half-edge running the other way between the
 * same two points.  Where a point pair carries more than one half-edge
 * (meshes that are not two-manifold), the paper's option 1 keeps the first
 * pair found: h = (a, b) is paired only if no lower id is also (a, b), and
 * then with the lowest id running (b, a).  Half-edges from a point to itself
 * are never paired.  he: [3 n_tri] out, -1 where there is no twin.
 */
static void twins_by_point_pairs(const int32_t *tris, int64_t n_tri, int32_t *he)
{
    he_rec *r = (he_rec *)malloc(sizeof(he_rec) * (size_t)(3 * n_tri + 1));
    int64_t n = 0;
    for (int64_t t = 0; t < n_tri; ++t)
        for (int j = 0; j < 3; ++j) {
            const int32_t a = tris[3 * t + j], b = tris[3 * t + (j + 1) % 3];
            if (a != b) {
                r[n].key = he_key(a, b);
                r[n].id = 3 * t + j;
                ++n;
            }
        }
    qsort(r, (size_t)n, sizeof(he_rec), he_cmp);
    for (int64_t h = 0; h < 3 * n_tri; ++h) he[h] = -1;
    for (int64_t k = 0; k < n; ++k) {
        if (k > 0 && r[k - 1].key == r[k].key) continue;     /* not the first of its key */
        const int32_t a = (int32_t)(r[k].key >> 32), b = (int32_t)(r[k].key & 0xffffffffu);
        he[r[k].id] = (int32_t)he_first(r, n, he_key(b, a));
    }
    free(r);
}

/*
 * HE of the organized mesh, Sec. 4.2 (computed there by Alg. 2): the twin of
 * every half-edge of T.  Taken from the definition -- the half-edge running
 * the other way between the same two points -- over T recovered from T_map
 * (an organized mesh is two-manifold, so every point pair carries at most one
 * half-edge each way).  Reading: a half-edge on the grid border or next to a
 * missing triangle has no twin (-1).
 * he: [3 n_tri] out.
 */
OR_EXPORT void oracle_mesh_halfedges(const int32_t *tri_map, int M, int N,
                                     int64_t n_tri, int32_t *he)
{
    const int Mq = M - 1, Nq = N - 1;
    int32_t *tris = (int32_t *)malloc(sizeof(int32_t) * (size_t)(3 * n_tri + 1));
    for (int64_t g = 0; g < 2LL * Mq * Nq; ++g) {
        const int32_t t = tri_map[g];
        if (t < 0 || t >= n_tri) continue;
        const int64_t q = g / 2;
        int64_t vert[3];
        tri_vertices((int)(q / Nq), (int)(q % Nq), (int)(g % 2), N, vert);
        for (int j = 0; j < 3; ++j) tris[3LL * t + j] = (int32_t)vert[j];
    }
    twins_by_point_pairs(tris, n_tri, he);
    free(tris);
}

/*
 * Laplacian filter on the organized cloud: Eqs. (1)-(2) of Sec. 2.3 applied
 * with the image-space neighbourhood of Sec. 5.1.
 *
 * Reading of Eq. (1): the printed "v_i . (lambda/W) sum w_j (v_i - v_j)" has
 * a vector product that cannot be meant; the update used is
 *     v_o = v_i - (lambda / W) sum_j w_j (v_i - v_j),   w_j = 1/||v_i - v_j||,
 * i.e. v_i moves a fraction lambda toward the inverse-distance-weighted mean
 * of its neighbours (lambda in [0, 1] adjusts smoothing).
 * Neighbours of pixel (u, v): every (u+du, v+dv) with |du|, |dv| <= K/2,
 * (du, dv) != (0, 0), that is valid.  Readings: a NaN neighbour is skipped; a
 * neighbour at distance 0 is skipped (its weight would be infinite); a pixel
 * with no usable neighbour keeps its value; an invalid pixel is copied.
 * Pixels within K/2 of the image border are not filtered (Sec. 5.1).
 * Iterations are Jacobi: each one reads only the previous iteration's values.
 * in/out: [M*N*3]; they may not alias.
 */
OR_EXPORT void oracle_laplacian(const double *in, double *out, int M, int N,
                                int K, double lambda, int iterations,
                                int nthreads)
{
    const int64_t P = (int64_t)M * N;
    const int r = K / 2;
    double *prev = (double *)malloc(sizeof(double) * 3 * P);
    memcpy(prev, in, sizeof(double) * 3 * P);
    memcpy(out, in, sizeof(double) * 3 * P);
    for (int it = 0; it < iterations; ++it) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int u = 0; u < M; ++u) {
            for (int v = 0; v < N; ++v) {
                const double *vi = prev + 3 * ((int64_t)u * N + v);
                double *vo = out + 3 * ((int64_t)u * N + v);
                vo[0] = vi[0]; vo[1] = vi[1]; vo[2] = vi[2];
                if (!point_valid(vi)) continue;
                if (u < r || u >= M - r || v < r || v >= N - r) continue;
                double W = 0.0, S[3] = {0.0, 0.0, 0.0};
                for (int du = -r; du <= r; ++du) {
                    for (int dv = -r; dv <= r; ++dv) {
                        if (du == 0 && dv == 0) continue;
                        const double *vj = prev + 3 * ((int64_t)(u + du) * N + (v + dv));
                        if (!point_valid(vj)) continue;
                        const double dx = vi[0] - vj[0];
                        const double dy = vi[1] - vj[1];
                        const double dz = vi[2] - vj[2];
                        const double d = sqrt(dx * dx + dy * dy + dz * dz);
                        if (!(d > 0.0)) continue;
                        const double w = 1.0 / d;
                        W += w;
                        S[0] += w * dx; S[1] += w * dy; S[2] += w * dz;
                    }
                }
                if (W > 0.0) {
                    vo[0] = vi[0] - lambda / W * S[0];
                    vo[1] = vi[1] - lambda / W * S[1];
                    vo[2] = vi[2] - lambda / W * S[2];
                }
            }
        }
        memcpy(prev, out, sizeof(double) * 3 * P);
    }
    free(prev);
}

/*
 * Triangle centroids and normals over the implicit full mesh T_FC (Sec. 5.2),
 * laid out in GID order: normals/centroids [2(M-1)(N-1)][3].
 * For t_{u,v,k} with vertices (a, b, c) in Alg. 1's order:
 *     centroid = (a + b + c) / 3,   normal = (b - a) x (c - a) / ||.||
 * Any NaN vertex makes both NaN (Sec. 5.2).  Reading: the paper prints no
 * normal formula; this orientation agrees with the counter-clockwise winding
 * of Sec. 4.2 and points toward a camera looking down +z.  A degenerate
 * triangle (zero cross product) gets a NaN normal.
 */
OR_EXPORT void oracle_tri_normals(const double *pts, int M, int N,
                                  double *normals, double *centroids,
                                  int nthreads)
{
    const int Mq = M - 1, Nq = N - 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int u = 0; u < Mq; ++u) {
        for (int v = 0; v < Nq; ++v) {
            for (int k = 0; k < 2; ++k) {
                const int64_t g = 2LL * ((int64_t)u * Nq + v) + k;
                int64_t idx[3];
                tri_vertices(u, v, k, N, idx);
                const double *a = pts + 3 * idx[0];
                const double *b = pts + 3 * idx[1];
                const double *c = pts + 3 * idx[2];
                double *n = normals + 3 * g;
                double *ce = centroids + 3 * g;
                if (!point_valid(a) || !point_valid(b) || !point_valid(c)) {
                    n[0] = n[1] = n[2] = NAN;
                    ce[0] = ce[1] = ce[2] = NAN;
                    continue;
                }
                for (int d = 0; d < 3; ++d) ce[d] = (a[d] + b[d] + c[d]) / 3.0;
                const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
                const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
                const double x[3] = {e1[1] * e2[2] - e1[2] * e2[1],
                                     e1[2] * e2[0] - e1[0] * e2[2],
                                     e1[0] * e2[1] - e1[1] * e2[0]};
                const double len = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
                if (!(len > 0.0)) {
                    n[0] = n[1] = n[2] = NAN;
                    continue;
                }
                n[0] = x[0] / len; n[1] = x[1] / len; n[2] = x[2] / len;
            }
        }
    }
}

static int vec_ok(const double *p)
{
    return !(isnan(p[0]) || isnan(p[1]) || isnan(p[2]));
}

/*
 * Bilateral normal filter on the organized mesh: Eqs. (3)-(6) of Sec. 2.3 on
 * the neighbourhood of Sec. 5.2.
 *
 * Neighbour set (Reading): the quad is the unit of work and the K x K window
 * is over quads.  The neighbours of t_{u,v,k} are both triangles of each of
 * the K*K - 1 other quads (u+du, v+dv), |du|, |dv| <= K/2, (du, dv) != 0, that
 * lie on the grid and have neither a NaN centroid nor a NaN normal.  At
 * K = 3 that is at most 16 neighbours, the count the paper gives.  The
 * triangle itself and its partner in the same quad are not neighbours.
 *
 * Weights (Eqs. 4-5): w_j = exp(-||c_i - c_j||^2 / (2 sl^2))
 *                         * exp(-||n_i - n_j||^2 / (2 sa^2)).
 * Reading of Eq. (6): the weighted mean is renormalised to unit length, so
 * the constant K cancels and any common positive factor of the weights does
 * too.  The sum is therefore formed with every exponent shifted by the
 * smallest one in the neighbourhood, which is the same value in exact
 * arithmetic and keeps the largest term at exp(0) = 1 instead of letting all
 * terms underflow.  A triangle with no neighbour, or whose weighted sum is
 * the zero vector, keeps its normal.  A triangle whose own normal or
 * centroid has a NaN is copied unchanged.  Centroids never change (vertices
 * are not updated, Sec. 5.2); iterations are Jacobi on the normals.
 *
 * normals_in/normals_out/centroids: [2(M-1)(N-1)][3] in GID order.
 */
OR_EXPORT void oracle_bilateral(const double *normals_in, const double *centroids,
                                int M, int N, int K, double sigma_length,
                                double sigma_angle, int iterations,
                                double *normals_out, int nthreads)
{
    const int Mq = M - 1, Nq = N - 1;
    const int64_t T = 2LL * Mq * Nq;
    const int r = K / 2;
    const int max_nb = 2 * (K * K - 1);
    double *prev = (double *)malloc(sizeof(double) * 3 * T);
    memcpy(prev, normals_in, sizeof(double) * 3 * T);
    memcpy(normals_out, normals_in, sizeof(double) * 3 * T);
    const double cl = 1.0 / (2.0 * sigma_length * sigma_length);
    const double ca = 1.0 / (2.0 * sigma_angle * sigma_angle);
    for (int it = 0; it < iterations; ++it) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int u = 0; u < Mq; ++u) {
            double *e = (double *)malloc(sizeof(double) * max_nb);
            int64_t *nb = (int64_t *)malloc(sizeof(int64_t) * max_nb);
            for (int v = 0; v < Nq; ++v) {
                for (int k = 0; k < 2; ++k) {
                    const int64_t i = 2LL * ((int64_t)u * Nq + v) + k;
                    const double *ni = prev + 3 * i;
                    const double *ci = centroids + 3 * i;
                    double *no = normals_out + 3 * i;
                    no[0] = ni[0]; no[1] = ni[1]; no[2] = ni[2];
                    if (!vec_ok(ni) || !vec_ok(ci)) continue;
                    int cnt = 0;
                    for (int du = -r; du <= r; ++du) {
                        for (int dv = -r; dv <= r; ++dv) {
                            if (du == 0 && dv == 0) continue;
                            const int uu = u + du, vv = v + dv;
                            if (uu < 0 || uu >= Mq || vv < 0 || vv >= Nq) continue;
                            for (int kk = 0; kk < 2; ++kk) {
                                const int64_t j = 2LL * ((int64_t)uu * Nq + vv) + kk;
                                const double *nj = prev + 3 * j;
                                const double *cj = centroids + 3 * j;
                                if (!vec_ok(nj) || !vec_ok(cj)) continue;
                                double dc2 = 0.0, dn2 = 0.0;
                                for (int d = 0; d < 3; ++d) {
                                    const double a = ci[d] - cj[d];
                                    const double b = ni[d] - nj[d];
                                    dc2 += a * a;
                                    dn2 += b * b;
                                }
                                e[cnt] = dc2 * cl + dn2 * ca;
                                nb[cnt] = j;
                                ++cnt;
                            }
                        }
                    }
                    if (cnt == 0) continue;
                    double emin = e[0];
                    for (int q = 1; q < cnt; ++q) if (e[q] < emin) emin = e[q];
                    double s[3] = {0.0, 0.0, 0.0};
                    for (int q = 0; q < cnt; ++q) {
                        const double w = exp(-(e[q] - emin));
                        const double *nj = prev + 3 * nb[q];
                        s[0] += w * nj[0]; s[1] += w * nj[1]; s[2] += w * nj[2];
                    }
                    const double len = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
                    if (!(len > 0.0)) continue;
                    no[0] = s[0] / len; no[1] = s[1] / len; no[2] = s[2] / len;
                }
            }
            free(e);
            free(nb);
        }
        memcpy(prev, normals_out, sizeof(double) * 3 * T);
    }
    free(prev);
}

/*
 * Smoothed normals of the final mesh T (Sec. 5.2): the filter runs on T_FC
 * and T_map picks out the triangles that exist.  normals_T[T_map[g]] =
 * normals[g] for every g with T_map[g] != -1.
 */
OR_EXPORT void oracle_gather(const double *normals, const int32_t *tri_map,
                             int M, int N, double *normals_T)
{
    const int64_t T = 2LL * (M - 1) * (N - 1);
    for (int64_t g = 0; g < T; ++g) {
        const int32_t t = tri_map[g];
        if (t < 0) continue;
        normals_T[3LL * t + 0] = normals[3 * g + 0];
        normals_T[3LL * t + 1] = normals[3 * g + 1];
        normals_T[3LL * t + 2] = normals[3 * g + 2];
    }
}

/*
 * Group assignment (Sec. 7.1, Alg. 4): label every triangle t of T with the
 * index j of the dominant plane normal most similar to its normal, or the
 * sentinel 255 when one of its edges is longer than l_max or the best
 * similarity falls short of ang_min.
 *
 * Reading: the points are the mesh vertices after smoothing and the normals
 * the filtered normals of T (the half-edge mesh the planar segmentation
 * receives).  Every label starts at 255; a triangle whose normal is NaN
 * matches no dominant normal and keeps it; with no dominant normal every
 * label is 255; among equal similarities the first wins (the strict
 * comparison of Alg. 4).
 * Reading (precision): these comparisons decide an integer, so they are taken
 * in float32 on the float32 data, as the GPU takes them, with each sum of
 * products written as fused multiply-adds in this order:
 *     |a - b|^2 = fma(dx, dx, fma(dy, dy, dz * dz)),  d = a - b
 *     n . n_j   = fma(nx, njx, fma(ny, njy, nz * njz))
 * and the edge test keeps a triangle iff each squared edge is <= l_max * l_max
 * (for exact reals, max |e| > l_max iff some |e|^2 > l_max^2); an edge with
 * a NaN coordinate passes no such test, so a triangle with an invalid vertex
 * gets 255, as does one with a vertex index outside [0, n_pts).
 */
static float sq_dist_f(const float *a, const float *b)
{
    const float dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

OR_EXPORT void oracle_group_assign(const float *pts, int64_t n_pts, const int32_t *tris,
                                   int64_t n_tri, const float *normals,
                                   const float *dominant, int l, float l_max,
                                   float ang_min, uint8_t *groups)
{
    const float lmax2 = l_max * l_max;
    for (int64_t t = 0; t < n_tri; ++t) {
        groups[t] = 255;
        const int32_t *v = tris + 3 * t;
        if (v[0] < 0 || v[1] < 0 || v[2] < 0 || v[0] >= n_pts || v[1] >= n_pts || v[2] >= n_pts)
            continue;
        const float *a = pts + 3LL * v[0], *b = pts + 3LL * v[1], *c = pts + 3LL * v[2];
        if (!(sq_dist_f(a, b) <= lmax2 && sq_dist_f(b, c) <= lmax2 && sq_dist_f(c, a) <= lmax2))
            continue;                               /* an edge longer than l_max */
        const float *n = normals + 3 * t;
        float best = -1.0f;
        int g = 255;
        for (int j = 0; j < l; ++j) {
            const float *d = dominant + 3 * j;
            const float sim = fmaf(n[0], d[0], fmaf(n[1], d[1], n[2] * d[2]));
            if (sim > best) {
                g = j;
                best = sim;
            }
        }
        if (best < ang_min) g = 255;
        groups[t] = (uint8_t)g;
    }
}

/*
 * Gaussian accumulator (Sec. 6.1): the refined icosahedron of Sec. 6.1.1 and
 * the integration of unit normals into its cells (Alg. 3).
 *
 * Level 0 is the regular icosahedron with vertices on the unit sphere; each
 * refinement splits every triangle into four through its edge midpoints and
 * pushes the new vertices out onto the sphere.  Level L has 10 * 4^L + 2
 * vertices and 20 * 4^L triangles (Table 1).  Each triangle is a cell of the
 * histogram; its surface normal is the unit normal of the triangle's plane,
 * pointing out of the sphere.
 * Reading: the cell normal is the plane normal (b - a) x (c - a), normalised;
 * the minimum angle between edge-adjacent cell normals reproduces Table 1's
 * separations at every level (a test checks it).
 *
 * Integration: the paper's search (space-filling-curve index, windowed
 * binary search, local neighbour search) is a fast way to find the cell
 * whose surface normal is closest to the input normal; the oracle takes that
 * definition directly, by brute force over all cells.
 * Reading (precision): the choice of cell decides an integer, so it is made
 * in float32 on float32 cell normals, with the squared distance written as
 *     d = c - n,  |d|^2 = fma(dx, dx, fma(dy, dy, dz * dz))
 * and the first cell with the smallest value winning (strict <).  A normal
 * with a NaN or infinite coordinate lands in no cell (index -1, not counted).
 * Sampling: rows 0, stride, 2 stride, ... of the normal list are integrated
 * (the paper integrates a sample of the mesh normals).
 */
static const double ICO_T = 1.6180339887498948482; /* golden ratio */

/* Base icosahedron: the 12 points (0, +-1, +-t) and their cyclic
 * permutations, and its 20 faces wound counter-clockwise seen from outside. */
static const double ico_base_v[12][3] = {
    {-1, ICO_T, 0}, {1, ICO_T, 0}, {-1, -ICO_T, 0}, {1, -ICO_T, 0},
    {0, -1, ICO_T}, {0, 1, ICO_T}, {0, -1, -ICO_T}, {0, 1, -ICO_T},
    {ICO_T, 0, -1}, {ICO_T, 0, 1}, {-ICO_T, 0, -1}, {-ICO_T, 0, 1}};
static const int ico_base_f[20][3] = {
    {0, 11, 5}, {0, 5, 1}, {0, 1, 7}, {0, 7, 10}, {0, 10, 11},
    {1, 5, 9}, {5, 11, 4}, {11, 10, 2}, {10, 7, 6}, {7, 1, 8},
    {3, 9, 4}, {3, 4, 2}, {3, 2, 6}, {3, 6, 8}, {3, 8, 9},
    {4, 9, 5}, {2, 4, 11}, {6, 2, 10}, {8, 6, 7}, {9, 8, 1}};

static void unit3(double *v)
{
    const double r = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= r; v[1] /= r; v[2] /= r;
}

OR_EXPORT int oracle_ga_sizes(int level, int64_t *n_vertices, int64_t *n_faces)
{
    if (level < 0 || level > 7) return -1;
    int64_t f = 20;
    for (int l = 0; l < level; ++l) f *= 4;
    *n_faces = f;
    *n_vertices = f / 2 + 2;
    return 0;
}

/* Midpoint vertex of edge (a, b), created once per edge: an open-addressed
 * table keyed by the ordered pair. */
typedef struct {
    int64_t *key;
    int32_t *val;
    int64_t cap;
} edge_map;

static int32_t edge_mid(edge_map *m, double *V, int32_t *nv, int32_t a, int32_t b)
{
    const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
    const int64_t k = ((int64_t)lo << 32) | (uint32_t)hi;
    uint64_t h = (uint64_t)k * 0x9E3779B97F4A7C15ull;
    int64_t i = (int64_t)(h % (uint64_t)m->cap);
    while (m->key[i] != -1 && m->key[i] != k) i = (i + 1) % m->cap;
    if (m->key[i] == k) return m->val[i];
    const int32_t id = (*nv)++;
    for (int c = 0; c < 3; ++c) V[3 * id + c] = 0.5 * (V[3 * lo + c] + V[3 * hi + c]);
    unit3(V + 3 * id);
    m->key[i] = k;
    m->val[i] = id;
    return id;
}

/* Refined icosahedron of `level`: vertices [V][3] (double, unit length),
 * faces [F][3] (counter-clockwise from outside) and cell normals [F][3]
 * rounded to float32.  Returns 0, or -1 for a level outside [0, 7]. */
OR_EXPORT int oracle_ga_icosahedron(int level, double *V, int32_t *F, float *cells)
{
    int64_t nv_all, nf_all;
    if (oracle_ga_sizes(level, &nv_all, &nf_all)) return -1;
    int32_t nv = 12;
    int64_t nf = 20;
    for (int i = 0; i < 12; ++i) {
        for (int c = 0; c < 3; ++c) V[3 * i + c] = ico_base_v[i][c];
        unit3(V + 3 * i);
    }
    for (int i = 0; i < 20; ++i)
        for (int c = 0; c < 3; ++c) F[3 * i + c] = ico_base_f[i][c];
    int32_t *G = (int32_t *)malloc(sizeof(int32_t) * 3 * (size_t)nf_all);
    for (int l = 0; l < level; ++l) {
        edge_map m;
        m.cap = 4 * nf + 7;
        m.key = (int64_t *)malloc(sizeof(int64_t) * (size_t)m.cap);
        m.val = (int32_t *)malloc(sizeof(int32_t) * (size_t)m.cap);
        for (int64_t i = 0; i < m.cap; ++i) m.key[i] = -1;
        for (int64_t f = 0; f < nf; ++f) {
            const int32_t a = F[3 * f], b = F[3 * f + 1], c = F[3 * f + 2];
            const int32_t ab = edge_mid(&m, V, &nv, a, b);
            const int32_t bc = edge_mid(&m, V, &nv, b, c);
            const int32_t ca = edge_mid(&m, V, &nv, c, a);
            const int32_t sub[4][3] = {{a, ab, ca}, {b, bc, ab}, {c, ca, bc}, {ab, bc, ca}};
            for (int s = 0; s < 4; ++s)
                for (int k = 0; k < 3; ++k) G[3 * (4 * f + s) + k] = sub[s][k];
        }
        free(m.key);
        free(m.val);
        nf *= 4;
        memcpy(F, G, sizeof(int32_t) * 3 * (size_t)nf);
    }
    free(G);
    for (int64_t f = 0; f < nf; ++f) {
        const double *a = V + 3 * F[3 * f], *b = V + 3 * F[3 * f + 1], *c = V + 3 * F[3 * f + 2];
        double e1[3], e2[3], n[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = b[k] - a[k];
            e2[k] = c[k] - a[k];
        }
        n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        n[2] = e1[0] * e2[1] - e1[1] * e2[0];
        unit3(n);
        for (int k = 0; k < 3; ++k) cells[3 * f + k] = (float)n[k];
    }
    return nv == nv_all ? 0 : -2;
}

/* Alg. 3 by its definition: nearest cell normal (float32 squared distance,
 * first minimum) for rows 0, stride, 2 stride, ... of `normals`; writes the
 * cell of the j-th integrated row to cell_out[j] (or -1) and adds one to
 * counts[cell] for each row that lands in a cell. */
OR_EXPORT void oracle_ga_integrate(const float *cells, int n_cells, const float *normals,
                                   int64_t n, int stride, int32_t *cell_out, uint32_t *counts)
{
    int64_t j = 0;
    for (int64_t t = 0; t < n; t += stride, ++j) {
        const float *p = normals + 3 * t;
        float best = INFINITY;
        int32_t arg = -1;
        for (int c = 0; c < n_cells; ++c) {
            const float dx = cells[3 * c] - p[0], dy = cells[3 * c + 1] - p[1],
                        dz = cells[3 * c + 2] - p[2];
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
            if (d2 < best) {
                best = d2;
                arg = c;
            }
        }
        cell_out[j] = arg;
        if (arg >= 0) counts[arg] += 1;
    }
}

/*
 * Half-edges of a user-provided mesh (Sec. 4.3): every half-edge is keyed by
 * its ordered point pair (a, b) and its twin is the half-edge keyed (b, a).
 * Half-edge 3t + j of triangle t runs from vertex j to vertex (j+1) mod 3.
 *
 * Edges shared by more than two triangles (the second manifold condition
 * of Sec. 4.3) take the paper's option 1, keep the first pair found:
 * Reading: "first" is the lowest half-edge index.  A half-edge gets a twin
 * only if it is the first with its key (a, b); its twin is then the first
 * half-edge keyed (b, a), if any.  Every other half-edge, and every
 * half-edge with a == b, gets -1.  The twins are then a symmetric pairing.
 *
 * Written as a sort of (key, index) pairs followed by binary searches: the
 * first half-edge of a key is the head of its run (twins_by_point_pairs).
 */
OR_EXPORT void oracle_user_halfedges(const int32_t *tris, int64_t n_tri, int32_t *he)
{
    twins_by_point_pairs(tris, n_tri, he);
}

/*
 * Vertex update after normal filtering: the second stage of the bilateral
 * mesh denoising the paper cites for Eqs. (3)-(6) (Sun et al., 2007), which
 * Polylidar3D itself skips (Sec. 5.2).  The paper does not print it; this is
 * the published update restated: each sweep moves every vertex x_i by the
 * mean, over the triangles f incident to it, of the correction that puts x_i
 * on the plane through f's centroid c_f with f's filtered normal n_f:
 *     x_i <- x_i + (1 / |F_i|) sum_{f in F_i} n_f (n_f . (c_f - x_i)).
 * Reading: F_i are the triangles of T_FC that contain vertex i, whose three
 * vertices are valid and whose filtered normal has no NaN; centroids are
 * recomputed from the current vertices every sweep and every vertex is
 * updated from the previous sweep's positions (Jacobi); a vertex with no
 * such triangle, and an invalid (NaN) point, is copied unchanged.
 * Parity unpinned against the paper itself (it gives no formula): the tests
 * pin this restatement by closed forms and invariants.
 */
OR_EXPORT void oracle_vertex_update(const double *pts, int M, int N, const double *normals,
                                    int iterations, double *out, int nthreads)
{
    const size_t P = (size_t)M * N;
    double *cur = (double *)malloc(sizeof(double) * 3 * P);
    memcpy(cur, pts, sizeof(double) * 3 * P);
    memcpy(out, pts, sizeof(double) * 3 * P);
    for (int it = 0; it < iterations; ++it) {
#pragma omp parallel for num_threads(nthreads) schedule(static)
        for (int r = 0; r < M; ++r) {
            for (int c = 0; c < N; ++c) {
                const int64_t i = (int64_t)r * N + c;
                const double *x = cur + 3 * i;
                double *o = out + 3 * i;
                o[0] = x[0]; o[1] = x[1]; o[2] = x[2];
                if (!point_valid(x)) continue;
                double acc[3] = {0.0, 0.0, 0.0};
                int count = 0;
                for (int u = r - 1; u <= r; ++u)
                    for (int v = c - 1; v <= c; ++v) {
                        if (u < 0 || v < 0 || u >= M - 1 || v >= N - 1) continue;
                        for (int k = 0; k < 2; ++k) {
                            int64_t idx[3];
                            tri_vertices(u, v, k, N, idx);
                            if (idx[0] != i && idx[1] != i && idx[2] != i) continue;
                            const double *a = cur + 3 * idx[0], *b = cur + 3 * idx[1],
                                         *d = cur + 3 * idx[2];
                            const double *n = normals + 3 * (2LL * ((int64_t)u * (N - 1) + v) + k);
                            if (!point_valid(a) || !point_valid(b) || !point_valid(d) || !vec_ok(n))
                                continue;
                            double proj = 0.0;
                            for (int q = 0; q < 3; ++q)
                                proj += n[q] * ((a[q] + b[q] + d[q]) / 3.0 - x[q]);
                            for (int q = 0; q < 3; ++q) acc[q] += n[q] * proj;
                            ++count;
                        }
                    }
                if (count)
                    for (int q = 0; q < 3; ++q) o[q] = x[q] + acc[q] / count;
            }
        }
        memcpy(cur, out, sizeof(double) * 3 * P);
    }
    free(cur);
}
