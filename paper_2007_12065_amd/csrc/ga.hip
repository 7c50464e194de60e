// Gaussian accumulator (Sec. 6.1): the refined icosahedron's cells and the
// integration of normals into them (Alg. 3).
//
// Integration finds, for every sampled normal, the cell whose surface normal
// is nearest (squared Euclidean distance in float32, first minimum) and adds
// one to that cell's count.  The paper reaches that cell on the CPU through a
// space-filling-curve index, a windowed binary search and a 12-neighbour
// check.  Here the search is a table lookup built once per accumulator: the
// sphere is cut into 6 G x G bins (the faces of a cube, gnomonic
// projection); each bin lists, in increasing cell order, every cell that can
// be nearest for some direction in the bin (a conservative angular bound,
// padded for the float32 rounding of the bin index and of the distances).
// A normal then costs one bin computation and the distances to its bin's
// few candidates (stored with their cell normals, so a search is two
// dependent table loads), and the chosen cell is exactly the brute-force
// one.
// A normal with a NaN or infinite coordinate lands in no cell (so does the
// brute force: every distance is NaN or infinite); finite normals whose
// length is outside [0.5, 2] are searched over all cells, which keeps the
// result the brute-force one for every input.
//
// Counts accumulate in an LDS histogram per workgroup (every cell's count,
// 4 bytes each).  A scene's normals crowd into a few cells, and atomic adds
// to one address serialise (about 30 ns each), so workgroups flush their
// non-zero cells into one of kGaReplicas copies of the histogram in the
// accumulator's workspace (copy = workgroup index mod kGaReplicas, which
// also keeps each copy on one XCD), and a second launch folds the copies
// into the caller's counts and clears them.  Sums of integers do not depend
// on the order of the adds.
#include "ga.h"
#include "tuning.h"

#include <algorithm>
#include <cfloat>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

namespace pl {

namespace {

constexpr int kGaBlock = 512;
constexpr int kGaBatch = 6;                // candidate loads issued together
#ifndef PL_GA_MAX_GRID
#define PL_GA_MAX_GRID 768
#endif
constexpr int kGaMaxGrid = PL_GA_MAX_GRID;  // workgroups of one integration launch
constexpr int kGaReplicas = 16;             // histogram copies the workgroups flush into

// Bin of a direction with |n|^2 in [0.25, 4]: the cube face of its largest
// component (+x, -x, +y, -y, +z, -z), then the two other components over
// the largest one's magnitude, each in [-1, 1], cut into G intervals.
__device__ __forceinline__ int ga_bin(float x, float y, float z, int G) {
    const float ax = fabsf(x), ay = fabsf(y), az = fabsf(z);
    int f;
    float m, u, v;
    if (ax >= ay && ax >= az) {
        f = x >= 0.0f ? 0 : 1; m = ax; u = y; v = z;
    } else if (ay >= az) {
        f = y >= 0.0f ? 2 : 3; m = ay; u = z; v = x;
    } else {
        f = z >= 0.0f ? 4 : 5; m = az; u = x; v = y;
    }
    // the hardware reciprocal (1 ulp) instead of two IEEE divisions: the bins
    // are padded by far more than the rounding of the coordinates
    const float hg = 0.5f * (float)G, im = __builtin_amdgcn_rcpf(m);
    const int iu = min(max((int)floorf(fmaf(u * im, hg, hg)), 0), G - 1);
    const int iv = min(max((int)floorf(fmaf(v * im, hg, hg)), 0), G - 1);
    return (f * G + iv) * G + iu;
}

__device__ __forceinline__ float ga_d2(const float *__restrict__ c, float x, float y, float z) {
    const float dx = c[0] - x, dy = c[1] - y, dz = c[2] - z;
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Brute force over all cells (normals whose length is outside [0.5, 2]).
__device__ __noinline__ int ga_nearest_all(float x, float y, float z,
                                           const float *__restrict__ cells, int n_cells) {
    float best = __builtin_inff();
    int arg = -1;
    for (int c = 0; c < n_cells; ++c) {
        const float d2 = ga_d2(cells + 3 * c, x, y, z);
        if (d2 < best) {
            best = d2;
            arg = c;
        }
    }
    return arg;
}

// One integrated row per thread and pass: the row's normal, then its bin's
// candidate range, then every candidate of the range at once (kGaBatch loads
// issued before the first is used; the built tables hold at most 6 per bin,
// longer ranges of a caller's cell set take further batches).  A wave thus
// waits for three dependent loads per row instead of one per candidate of
// its longest range.
template <typename NT>
__global__ __launch_bounds__(kGaBlock) void k_ga_integrate(
    const NT *__restrict__ normals, const int32_t *__restrict__ n_dev, int cap, int stride,
    const float *__restrict__ cells, int n_cells, const int *__restrict__ bin_start,
    const float4 *__restrict__ bin_cells, int G, uint32_t *__restrict__ replicas,
    int32_t *__restrict__ cell_out) {
    extern __shared__ uint32_t hist[];
    const int n = min(max(*n_dev, 0), cap);
    const int rows = n == 0 ? 0 : (n - 1) / stride + 1;
    const int span = (int)gridDim.x * kGaBlock;
    const int first = (int)blockIdx.x * kGaBlock;
    if (first >= rows) return;                       // the whole workgroup has no row
    for (int i = threadIdx.x; i < n_cells; i += kGaBlock) hist[i] = 0u;
    __syncthreads();
    for (int j = first + (int)threadIdx.x; j < rows; j += span) {
        const size_t t = (size_t)j * (size_t)stride;
        const float x = ld_f(normals + 3 * t), y = ld_f(normals + 3 * t + 1),
                    z = ld_f(normals + 3 * t + 2);
        const float s2 = fmaf(x, x, fmaf(y, y, z * z));
        // a NaN or infinite coordinate lands in no cell (every distance is NaN
        // or infinite); only finite normals of odd length search all
        const bool none = !(fabsf(x) <= FLT_MAX && fabsf(y) <= FLT_MAX && fabsf(z) <= FLT_MAX);
        const bool all = !none && !(s2 >= 0.25f && s2 <= 4.0f);
        const int b = (all || none) ? 0 : ga_bin(x, y, z, G);
        const int lo = bin_start[b];
        const int len = (all || none) ? 0 : bin_start[b + 1] - lo;
        float best = __builtin_inff();
        int arg = -1;
        for (int k0 = 0; k0 < len; k0 += kGaBatch) {
            float4 e[kGaBatch];
#pragma unroll
            for (int k = 0; k < kGaBatch; ++k)
                e[k] = k0 + k < len ? bin_cells[lo + k0 + k] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int k = 0; k < kGaBatch; ++k) {
                if (k0 + k < len) {
                    // a candidate is its cell's normal with the cell index in w
                    const float dx = e[k].x - x, dy = e[k].y - y, dz = e[k].z - z;
                    const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
                    if (d2 < best) {
                        best = d2;
                        arg = (int)__float_as_uint(e[k].w);
                    }
                }
            }
        }
        const int c = all ? ga_nearest_all(x, y, z, cells, n_cells) : arg;
        if (cell_out) cell_out[j] = c;
        if (c >= 0) atomicAdd(&hist[c], 1u);
    }
    __syncthreads();
    uint32_t *copy = replicas + (size_t)(blockIdx.x % kGaReplicas) * n_cells;
    for (int i = threadIdx.x; i < n_cells; i += kGaBlock) {
        const uint32_t v = hist[i];
        if (v) atomicAdd(&copy[i], v);
    }
}

// counts[i] += sum of the copies' cell i; the copies return to zero.
__global__ __launch_bounds__(kGaBlock) void k_ga_fold(uint32_t *__restrict__ replicas,
                                                      int n_cells, uint32_t *__restrict__ counts) {
    const int i = (int)blockIdx.x * kGaBlock + (int)threadIdx.x;
    if (i >= n_cells) return;
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < kGaReplicas; ++r) {
        uint32_t *p = replicas + (size_t)r * n_cells + i;
        sum += *p;
        *p = 0u;
    }
    if (sum) atomicAdd(&counts[i], sum);
}

// ---------------------------------------------------------------------------
// Host side: the icosahedron and the bin tables.
// ---------------------------------------------------------------------------

struct V3 {
    double x, y, z;
};
V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
V3 unit(V3 a) { return (1.0 / std::sqrt(dot(a, a))) * a; }

// Level-`level` icosphere: the 12 vertices (0, +-1, +-g) and their cyclic
// permutations (g the golden ratio) on the unit sphere, the 20 faces found
// as the triples of mutually nearest vertices, wound outward; then `level`
// rounds of splitting every face in four through its edge midpoints pushed
// onto the sphere.  Returns the cells' plane normals, float32 [F][3].
std::vector<float> icosphere_cells(int level) {
    const double g = (1.0 + std::sqrt(5.0)) / 2.0;
    std::vector<V3> V;
    for (int s1 : {-1, 1})
        for (int s2 : {-1, 1}) {
            V.push_back(unit({0.0, (double)s1, s2 * g}));
            V.push_back(unit({(double)s1, s2 * g, 0.0}));
            V.push_back(unit({s2 * g, 0.0, (double)s1}));
        }
    double edge2 = 1e9;
    for (size_t i = 0; i < V.size(); ++i)
        for (size_t j = i + 1; j < V.size(); ++j) edge2 = std::min(edge2, dot(V[i] - V[j], V[i] - V[j]));
    auto adjacent = [&](int i, int j) { return dot(V[i] - V[j], V[i] - V[j]) < edge2 * 1.001; };
    std::vector<std::array<int, 3>> F;
    for (int i = 0; i < 12; ++i)
        for (int j = i + 1; j < 12; ++j)
            for (int k = j + 1; k < 12; ++k)
                if (adjacent(i, j) && adjacent(j, k) && adjacent(i, k)) {
                    const bool out = dot(cross(V[j] - V[i], V[k] - V[i]), V[i] + V[j] + V[k]) > 0;
                    F.push_back(out ? std::array<int, 3>{i, j, k} : std::array<int, 3>{i, k, j});
                }
    for (int l = 0; l < level; ++l) {
        std::unordered_map<uint64_t, int> mid;
        auto midpoint = [&](int a, int b) {
            const uint64_t key = ((uint64_t)std::min(a, b) << 32) | (uint32_t)std::max(a, b);
            auto it = mid.find(key);
            if (it != mid.end()) return it->second;
            V.push_back(unit(0.5 * (V[std::min(a, b)] + V[std::max(a, b)])));
            mid.emplace(key, (int)V.size() - 1);
            return (int)V.size() - 1;
        };
        std::vector<std::array<int, 3>> G;
        G.reserve(F.size() * 4);
        for (const auto &f : F) {
            const int ab = midpoint(f[0], f[1]), bc = midpoint(f[1], f[2]), ca = midpoint(f[2], f[0]);
            G.push_back({ab, bc, ca});
            G.push_back({f[0], ab, ca});
            G.push_back({ab, f[1], bc});
            G.push_back({ca, bc, f[2]});
        }
        F.swap(G);
    }
    std::vector<float> cells(3 * F.size());
    for (size_t i = 0; i < F.size(); ++i) {
        const V3 n = unit(cross(V[F[i][1]] - V[F[i][0]], V[F[i][2]] - V[F[i][0]]));
        cells[3 * i] = (float)n.x;
        cells[3 * i + 1] = (float)n.y;
        cells[3 * i + 2] = (float)n.z;
    }
    return cells;
}

// Direction of cube-face coordinates (u, v) on face f (see ga_bin).
V3 face_dir(int f, double u, double v) {
    const double s = (f & 1) ? -1.0 : 1.0;
    switch (f >> 1) {
    case 0: return unit({s, u, v});
    case 1: return unit({v, s, u});
    default: return unit({u, v, s});
    }
}

struct BinRegion {
    V3 center;
    double radius;                 // angle from the centre to the farthest corner
};

// Bin (f, iv, iu) of a G x G face grid, padded by `pad` in (u, v).
BinRegion bin_region(int f, int iu, int iv, int G, double pad) {
    const double u0 = -1.0 + 2.0 * iu / G - pad, u1 = -1.0 + 2.0 * (iu + 1) / G + pad;
    const double v0 = -1.0 + 2.0 * iv / G - pad, v1 = -1.0 + 2.0 * (iv + 1) / G + pad;
    BinRegion r;
    r.center = face_dir(f, 0.5 * (u0 + u1), 0.5 * (v0 + v1));
    r.radius = 0.0;
    for (double u : {u0, u1})
        for (double v : {v0, v1})
            r.radius = std::max(r.radius, std::acos(std::min(1.0, dot(r.center, face_dir(f, u, v)))));
    return r;
}

// Cells that can be nearest for some direction within angle `R` of centre
// `c`.  With t_i the angle from c to cell i, a direction d of the region is
// within t_j + R of the cell j closest to c, so its nearest cell is within
// H = min_j t_j + R of d, and cell i is at least t_i - R from d: only cells
// with t_i - R <= H can be nearest.  Cells with t_i - R <= H + margin are
// kept: every other cell is farther from every direction of the region than
// its nearest cell by more than `margin`, which float32 distances resolve.
void candidates(const std::vector<V3> &cn, const std::vector<int> &pool, V3 c, double R,
                double margin, std::vector<int> &out) {
    // t_i - R <= min t + R + margin  <=>  cos t_i >= cos(min t + 2R + margin)
    double best_dot = -2.0;
    std::vector<double> d(pool.size());
    for (size_t k = 0; k < pool.size(); ++k) {
        d[k] = dot(c, cn[pool[k]]);
        best_dot = std::max(best_dot, d[k]);
    }
    const double reach = std::acos(std::max(-1.0, std::min(1.0, best_dot))) + 2.0 * R + margin;
    const double floor_dot = reach >= 3.14159265358979 ? -2.0 : std::cos(reach);
    out.clear();
    for (size_t k = 0; k < pool.size(); ++k)
        if (d[k] >= floor_dot) out.push_back(pool[k]);
}

struct GaTables {
    int n_cells = 0, G = 0;
    std::vector<float> cells;
    std::vector<int32_t> bin_start;
    std::vector<float> bin_cells;     // per candidate: x, y, z, cell index (bits)
    size_t off_cells = 0, off_start = 0, off_list = 0, off_replicas = 0, bytes = 0;
};

constexpr double kPad = 1e-5;      // (u, v) padding: float32 rounding of the bin index
constexpr double kMargin = 1e-3;   // radians: float32 rounding of the distances

std::unique_ptr<GaTables> build_tables(const float *cells, int n_cells, int G) {
    auto T = std::make_unique<GaTables>();
    T->n_cells = n_cells;
    T->G = G;
    T->cells.assign(cells, cells + 3 * (size_t)n_cells);
    std::vector<V3> cn(n_cells);
    for (int i = 0; i < n_cells; ++i)
        cn[i] = unit({cells[3 * i], cells[3 * i + 1], cells[3 * i + 2]});
    std::vector<int> all(n_cells);
    for (int i = 0; i < n_cells; ++i) all[i] = i;
    // coarse bins first (a superset for every fine bin inside), then fine bins
    const int C = std::max(1, G / 8), per = G / C;
    double r_fine = 0.0;
    for (int f = 0; f < 6; ++f)
        for (int iv = 0; iv < G; ++iv)
            for (int iu = 0; iu < G; ++iu) r_fine = std::max(r_fine, bin_region(f, iu, iv, G, kPad).radius);
    T->bin_start.assign(6 * (size_t)G * G + 1, 0);
    std::vector<int> coarse, fine;
    std::vector<std::vector<uint16_t>> lists(6 * (size_t)G * G);
    for (int f = 0; f < 6; ++f)
        for (int cv = 0; cv < C; ++cv)
            for (int cu = 0; cu < C; ++cu) {
                // the coarse region spans `per` fine bins each way
                const double u0 = -1.0 + 2.0 * cu * per / G - kPad, u1 = -1.0 + 2.0 * (cu + 1) * per / G + kPad;
                const double v0 = -1.0 + 2.0 * cv * per / G - kPad, v1 = -1.0 + 2.0 * (cv + 1) * per / G + kPad;
                const V3 cc = face_dir(f, 0.5 * (u0 + u1), 0.5 * (v0 + v1));
                double rc = 0.0;
                for (double u : {u0, u1})
                    for (double v : {v0, v1})
                        rc = std::max(rc, std::acos(std::min(1.0, dot(cc, face_dir(f, u, v)))));
                // a superset of every fine bin's candidates: with b a fine
                // centre (within rc of cc) and r <= r_fine its radius, a fine
                // candidate has t_i(b) <= min t(b) + 2r + margin, hence
                // t_i(cc) <= min t(cc) + 2 rc + 2 r_fine + margin, which the
                // bound below with R = rc + r_fine admits
                candidates(cn, all, cc, rc + r_fine, kMargin, coarse);
                for (int iv = cv * per; iv < (cv + 1) * per; ++iv)
                    for (int iu = cu * per; iu < (cu + 1) * per; ++iu) {
                        const BinRegion b = bin_region(f, iu, iv, G, kPad);
                        candidates(cn, coarse, b.center, b.radius, kMargin, fine);
                        std::sort(fine.begin(), fine.end());
                        auto &L = lists[((size_t)f * G + iv) * G + iu];
                        L.assign(fine.begin(), fine.end());
                    }
            }
    size_t total = 0;
    for (size_t b = 0; b < lists.size(); ++b) {
        T->bin_start[b] = (int32_t)total;
        total += lists[b].size();
    }
    T->bin_start[lists.size()] = (int32_t)total;
    T->bin_cells.reserve(4 * total);
    for (auto &L : lists)
        for (uint16_t c : L) {
            uint32_t bits = c;
            float w;
            std::memcpy(&w, &bits, 4);
            T->bin_cells.insert(T->bin_cells.end(), {cells[3 * c], cells[3 * c + 1], cells[3 * c + 2], w});
        }
    T->off_cells = 0;
    T->off_start = align_up(12 * (size_t)n_cells, 256);
    T->off_list = T->off_start + align_up(4 * T->bin_start.size(), 256);
    T->off_replicas = T->off_list + align_up(16 * std::max<size_t>(total, 1), 256);
    T->bytes = T->off_replicas + align_up(4 * (size_t)kGaReplicas * n_cells, 256);
    return T;
}

int grid_for_level(int level) { return std::min(256, 8 << level); }

std::mutex g_ga_mu;
std::map<int, std::unique_ptr<GaTables>> g_ga_levels;   // built once per level

const GaTables *level_tables(int level) {
    std::lock_guard<std::mutex> lk(g_ga_mu);
    auto it = g_ga_levels.find(level);
    if (it != g_ga_levels.end()) return it->second.get();
    const std::vector<float> cells = icosphere_cells(level);
    auto T = build_tables(cells.data(), (int)(cells.size() / 3), grid_for_level(level));
    const GaTables *p = T.get();
    g_ga_levels.emplace(level, std::move(T));
    return p;
}

}  // namespace

}  // namespace pl

struct pl_ga_s {
    std::unique_ptr<pl::GaTables> own;      // tables of caller-given cells
    const pl::GaTables *tab = nullptr;
    uint8_t *ws = nullptr;
    size_t lds = 0;
};

namespace pl {

size_t ga_level_workspace(int level) { return level_tables(level)->bytes; }

size_t ga_cells_workspace(const float *cells, int n_cells) {
    return build_tables(cells, n_cells, 64)->bytes;
}

namespace {

pl_status ga_upload(pl_ga_s *g, hipStream_t s) {
    const GaTables &T = *g->tab;
    std::vector<uint8_t> img(T.bytes, 0);      // the histogram copies start at zero
    std::memcpy(img.data() + T.off_cells, T.cells.data(), 4 * T.cells.size());
    std::memcpy(img.data() + T.off_start, T.bin_start.data(), 4 * T.bin_start.size());
    std::memcpy(img.data() + T.off_list, T.bin_cells.data(), 4 * T.bin_cells.size());
    if (pl_status st = hip_check(hipMemcpyAsync(g->ws, img.data(), T.bytes, hipMemcpyHostToDevice, s),
                                 "hipMemcpyAsync"))
        return st;
    if (pl_status st = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize")) return st;
    g->lds = 4 * (size_t)T.n_cells;
    for (const void *k : {(const void *)k_ga_integrate<float>, (const void *)k_ga_integrate<__half>})
        if (pl_status st = allow_lds(k, g->lds)) return st;
    return PL_OK;
}

}  // namespace

pl_status ga_create_level(int level, void *ws, hipStream_t s, pl_ga_s **out) {
    auto g = std::unique_ptr<pl_ga_s>(new (std::nothrow) pl_ga_s());
    if (!g) {
        set_error("out of host memory");
        return PL_ERR_ARG;
    }
    g->tab = level_tables(level);
    g->ws = static_cast<uint8_t *>(ws);
    if (pl_status st = ga_upload(g.get(), s)) return st;
    *out = g.release();
    return PL_OK;
}

pl_status ga_create_cells(const float *cells, int n_cells, void *ws, hipStream_t s, pl_ga_s **out) {
    auto g = std::unique_ptr<pl_ga_s>(new (std::nothrow) pl_ga_s());
    if (!g) {
        set_error("out of host memory");
        return PL_ERR_ARG;
    }
    g->own = build_tables(cells, n_cells, 64);
    g->tab = g->own.get();
    g->ws = static_cast<uint8_t *>(ws);
    if (pl_status st = ga_upload(g.get(), s)) return st;
    *out = g.release();
    return PL_OK;
}

size_t ga_bytes(const pl_ga_s *g) { return g->tab->bytes; }
int ga_cell_count(const pl_ga_s *g) { return g->tab->n_cells; }
const float *ga_cells(const pl_ga_s *g) {
    return reinterpret_cast<const float *>(g->ws + g->tab->off_cells);
}

pl_status ga_integrate(const pl_ga_s *g, const void *normals, pl_dtype ndt, const int32_t *n_dev,
                       int cap, int stride, uint32_t *counts, int32_t *cell_out, hipStream_t s) {
    if (cap == 0) return PL_OK;
    const GaTables &T = *g->tab;
    const long rows = ((long)cap + stride - 1) / stride;
    const float *cells = reinterpret_cast<const float *>(g->ws + T.off_cells);
    const int *start = reinterpret_cast<const int *>(g->ws + T.off_start);
    const float4 *list = reinterpret_cast<const float4 *>(g->ws + T.off_list);
    uint32_t *reps = reinterpret_cast<uint32_t *>(g->ws + T.off_replicas);
    // one row per thread and pass, at most kGaMaxGrid workgroups (past that,
    // threads loop: fewer histograms to clear and flush)
    const int grid = (int)std::min<long>(kGaMaxGrid, (rows + kGaBlock - 1) / kGaBlock);
    const size_t lds = g->lds;
    if (ndt == PL_F32)
        k_ga_integrate<float><<<grid, kGaBlock, lds, s>>>(static_cast<const float *>(normals), n_dev,
                                                          cap, stride, cells, T.n_cells, start, list,
                                                          T.G, reps, cell_out);
    else
        k_ga_integrate<__half><<<grid, kGaBlock, lds, s>>>(static_cast<const __half *>(normals), n_dev,
                                                           cap, stride, cells, T.n_cells, start, list,
                                                           T.G, reps, cell_out);
    if (pl_status st = hip_check(hipGetLastError(), "k_ga_integrate")) return st;
    k_ga_fold<<<(T.n_cells + kGaBlock - 1) / kGaBlock, kGaBlock, 0, s>>>(reps, T.n_cells, counts);
    return hip_check(hipGetLastError(), "k_ga_fold");
}

void ga_destroy(pl_ga_s *g) { delete g; }

}  // namespace pl
