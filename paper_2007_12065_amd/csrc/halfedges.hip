// Half-edges of a user-provided mesh (Sec. 4.3) through a device hash table.
//
// Every half-edge (a, b) of T (3t + j runs from vertex j to vertex j+1 mod 3
// of triangle t) is keyed by its ordered point pair; its twin is the
// half-edge keyed (b, a).  Edges shared by more than two triangles keep the
// first pair (the paper's option 1): a half-edge is paired only if it has
// the lowest index among the half-edges with its key, and then with the
// lowest-index half-edge keyed (b, a).  Half-edges from a point to itself
// are never paired.
//
// The table is keyed by the undirected edge (lo, hi), lo < hi, and each slot
// holds two values: the first half-edge running lo -> hi and the first
// running hi -> lo.  Three launches:
//   k_he_clear    every slot of the table empty (a kernel, so the sequence
//                 can be captured into a graph)
//   k_he_insert   one thread per triangle: each half-edge claims its edge's
//                 slot (64-bit compare-and-swap, linear probing) and lowers
//                 its direction's value to its index (atomic min), so every
//                 slot ends with the first index of each direction whatever
//                 the order of the threads
//   k_he_lookup   one thread per triangle: a half-edge that is the first of
//                 its direction takes the other direction's value
// The table has at least twice as many slots as half-edges (load <= 1/2),
// so every probe sequence meets its key or an empty slot.
//
// Probing reads a slot before it tries an atomic on it: only an empty slot
// or the edge's own key is worth a compare-and-swap.
#include "he.h"

#include <algorithm>
#include <climits>

namespace pl {

namespace {

constexpr int kHeBlock = 256;
constexpr unsigned long long kEmpty = ~0ull;   // (-1, -1): lo == hi, never inserted

__device__ __forceinline__ unsigned long long he_key(int lo, int hi) {
    return ((unsigned long long)(unsigned)lo << 32) | (unsigned)hi;
}

// The 64-bit finaliser of MurmurHash3 (Appleby): every input bit reaches
// every output bit.
__device__ __forceinline__ unsigned long long he_mix(unsigned long long k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

__device__ __forceinline__ size_t he_slot(int lo, int hi, size_t mask) {
    return (size_t)he_mix(he_key(lo, hi)) & mask;
}

size_t table_slots(int cap) {
    size_t s = 256;
    while (s < 6 * (size_t)cap) s <<= 1;
    return s;
}

__global__ __launch_bounds__(kHeBlock) void k_he_clear(unsigned long long *__restrict__ keys,
                                                       int2 *__restrict__ vals, size_t slots) {
    for (size_t i = (size_t)blockIdx.x * kHeBlock + threadIdx.x; i < slots;
         i += (size_t)gridDim.x * kHeBlock) {
        keys[i] = kEmpty;
        vals[i] = make_int2(INT_MAX, INT_MAX);
    }
}

__global__ __launch_bounds__(kHeBlock) void k_he_insert(const int32_t *__restrict__ tris,
                                                        const int32_t *__restrict__ n_tri,
                                                        int cap,
                                                        unsigned long long *__restrict__ keys,
                                                        int2 *__restrict__ vals, size_t mask) {
    const int n = min(max(*n_tri, 0), cap);
    const int t = (int)blockIdx.x * kHeBlock + (int)threadIdx.x;
    if (t >= n) return;
    const int v[3] = {tris[3 * (size_t)t], tris[3 * (size_t)t + 1], tris[3 * (size_t)t + 2]};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int a = v[j], b = v[(j + 1) % 3];
        if (a == b) continue;
        const int lo = min(a, b), hi = max(a, b);
        const unsigned long long key = he_key(lo, hi);
        size_t slot = he_slot(lo, hi, mask);
        for (;;) {
            // a plain read first: only an empty slot or the key itself is
            // worth an atomic
            const unsigned long long seen = __hip_atomic_load(&keys[slot], __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long prev =
                seen == kEmpty ? atomicCAS(&keys[slot], kEmpty, key) : seen;
            if (prev == kEmpty || prev == key) {
                int *dir = a < b ? &vals[slot].x : &vals[slot].y;
                atomicMin(dir, 3 * t + j);
                break;
            }
            slot = (slot + 1) & mask;
        }
    }
}

__global__ __launch_bounds__(kHeBlock) void k_he_lookup(const int32_t *__restrict__ tris,
                                                        const int32_t *__restrict__ n_tri,
                                                        int cap,
                                                        const unsigned long long *__restrict__ keys,
                                                        const int2 *__restrict__ vals, size_t mask,
                                                        int32_t *__restrict__ he) {
    const int n = min(max(*n_tri, 0), cap);
    const int t = (int)blockIdx.x * kHeBlock + (int)threadIdx.x;
    if (t >= n) return;
    const int v[3] = {tris[3 * (size_t)t], tris[3 * (size_t)t + 1], tris[3 * (size_t)t + 2]};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int a = v[j], b = v[(j + 1) % 3];
        int twin = -1;
        if (a != b) {
            const int lo = min(a, b), hi = max(a, b);
            const unsigned long long key = he_key(lo, hi);
            size_t slot = he_slot(lo, hi, mask);
            while (keys[slot] != key) slot = (slot + 1) & mask;   // inserted above: present
            const int2 f = vals[slot];
            const int own = a < b ? f.x : f.y, other = a < b ? f.y : f.x;
            if (own == 3 * t + j && other != INT_MAX) twin = other;
        }
        he[3 * (size_t)t + j] = twin;
    }
}

}  // namespace

size_t user_halfedges_workspace(int cap) {
    const size_t s = table_slots(cap);
    return align_up(8 * s, 256) + align_up(8 * s, 256);
}

pl_status launch_user_halfedges(const int32_t *tris, const int32_t *n_tri, int cap, int32_t *he,
                                void *ws, hipStream_t s) {
    if (cap == 0) return PL_OK;
    const size_t slots = table_slots(cap);
    auto *keys = static_cast<unsigned long long *>(ws);
    auto *vals = reinterpret_cast<int2 *>(static_cast<uint8_t *>(ws) + align_up(8 * slots, 256));
    const int clear_grid = (int)std::min<size_t>(4096, (slots + kHeBlock - 1) / kHeBlock);
    k_he_clear<<<clear_grid, kHeBlock, 0, s>>>(keys, vals, slots);
    if (pl_status st = hip_check(hipGetLastError(), "k_he_clear")) return st;
    const int grid = (cap + kHeBlock - 1) / kHeBlock;
    k_he_insert<<<grid, kHeBlock, 0, s>>>(tris, n_tri, cap, keys, vals, slots - 1);
    if (pl_status st = hip_check(hipGetLastError(), "k_he_insert")) return st;
    k_he_lookup<<<grid, kHeBlock, 0, s>>>(tris, n_tri, cap, keys, vals, slots - 1, he);
    return hip_check(hipGetLastError(), "k_he_lookup");
}

}  // namespace pl
