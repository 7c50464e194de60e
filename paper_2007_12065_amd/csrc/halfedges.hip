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
// The table is keyed by the undirected edge (lo, hi), lo < hi; a slot (16
// bytes, one cache line holds eight) keeps the key and two values: the
// first half-edge running lo -> hi and the first running hi -> lo.  Three
// launches:
//   k_he_clear    every slot of the table empty (a kernel, so the sequence
//                 can be captured into a graph)
//   k_he_insert   one thread per half-edge: it claims its edge's
//                 slot (64-bit compare-and-swap, linear probing), lowers its
//                 direction's value to its index (atomic min, in the same
//                 line as the key), so every slot ends with the first index
//                 of each direction whatever the order of the threads, and
//                 records the slot it found
//   k_he_lookup   one thread per half-edge: a half-edge that is the first of
//                 its direction takes the other direction's value from its
//                 recorded slot (one read, no probing)
// The table has 4 cap slots (rounded up to 64), at least 4/3 as many as
// half-edges (load <= 3/4), so every probe sequence meets its key or an
// empty slot.  Hash values are reduced to a slot by a 64 x 64-bit high
// product, which needs no power-of-two size.  Triangles are dealt to
// workgroups in contiguous runs per XCD, so the two triangles of an edge in
// an organized mesh, a row apart, usually run under the same L2.
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

struct alignas(16) HeSlot {
    unsigned long long key;
    int fwd, bwd;                    // first half-edge lo -> hi, hi -> lo
};

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

// hash in [0, 2^64) scaled to [0, slots)
__device__ __forceinline__ unsigned long long he_slot(unsigned long long key,
                                                      unsigned long long slots) {
    return __umul64hi(he_mix(key), slots);
}

size_t table_slots(int cap) {
    const size_t s = (4 * (size_t)cap + 63) / 64 * 64;
    return s < 256 ? 256 : s;
}

__global__ __launch_bounds__(kHeBlock) void k_he_clear(HeSlot *__restrict__ tab, size_t slots) {
    for (size_t i = (size_t)blockIdx.x * kHeBlock + threadIdx.x; i < slots;
         i += (size_t)gridDim.x * kHeBlock) {
        HeSlot e;
        e.key = kEmpty;
        e.fwd = INT_MAX;
        e.bwd = INT_MAX;
        tab[i] = e;
    }
}

__global__ __launch_bounds__(kHeBlock) void k_he_insert(const int32_t *__restrict__ tris,
                                                        const int32_t *__restrict__ n_tri,
                                                        int cap, HeSlot *__restrict__ tab,
                                                        unsigned long long slots,
                                                        int32_t *__restrict__ hslot) {
    // one thread per half-edge: the three of a triangle run side by side
    const int n = 3 * min(max(*n_tri, 0), cap);
    const int h = xcd_remap((int)blockIdx.x, (int)gridDim.x) * kHeBlock + (int)threadIdx.x;
    if (h >= n) return;
    const int t = h / 3, j = h - 3 * t;
    const int a = tris[h], b = tris[3 * t + (j == 2 ? 0 : j + 1)];
    int found = -1;
    if (a != b) {
        const int lo = min(a, b), hi = max(a, b);
        const unsigned long long key = he_key(lo, hi);
        unsigned long long slot = he_slot(key, slots);
        for (;;) {
            // a plain read first: only an empty slot or the key itself is
            // worth an atomic
            const unsigned long long seen = __hip_atomic_load(&tab[slot].key, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
            const unsigned long long prev =
                seen == kEmpty ? atomicCAS(&tab[slot].key, kEmpty, key) : seen;
            if (prev == kEmpty || prev == key) {
                atomicMin(a < b ? &tab[slot].fwd : &tab[slot].bwd, h);
                found = (int)slot;
                break;
            }
            slot = slot + 1 == slots ? 0 : slot + 1;
        }
    }
    hslot[h] = found;
}

__global__ __launch_bounds__(kHeBlock) void k_he_lookup(const int32_t *__restrict__ tris,
                                                        const int32_t *__restrict__ n_tri,
                                                        int cap, const HeSlot *__restrict__ tab,
                                                        const int32_t *__restrict__ hslot,
                                                        int32_t *__restrict__ he) {
    const int n = 3 * min(max(*n_tri, 0), cap);
    const int h = xcd_remap((int)blockIdx.x, (int)gridDim.x) * kHeBlock + (int)threadIdx.x;
    if (h >= n) return;
    const int sl = hslot[h];
    int twin = -1;
    if (sl >= 0) {
        const int t = h / 3, j = h - 3 * t;
        const int a = tris[h], b = tris[3 * t + (j == 2 ? 0 : j + 1)];
        const int2 f = *reinterpret_cast<const int2 *>(&tab[sl].fwd);
        const int own = a < b ? f.x : f.y, other = a < b ? f.y : f.x;
        if (own == h && other != INT_MAX) twin = other;
    }
    he[h] = twin;
}

}  // namespace

size_t user_halfedges_workspace(int cap) {
    return align_up(sizeof(HeSlot) * table_slots(cap), 256) + align_up(12 * (size_t)cap, 256);
}

pl_status launch_user_halfedges(const int32_t *tris, const int32_t *n_tri, int cap, int32_t *he,
                                void *ws, hipStream_t s) {
    if (cap == 0) return PL_OK;
    const size_t slots = table_slots(cap);
    auto *tab = static_cast<HeSlot *>(ws);
    auto *hslot = reinterpret_cast<int32_t *>(static_cast<uint8_t *>(ws) +
                                              align_up(sizeof(HeSlot) * slots, 256));
    const int clear_grid = (int)std::min<size_t>(4096, (slots + kHeBlock - 1) / kHeBlock);
    k_he_clear<<<clear_grid, kHeBlock, 0, s>>>(tab, slots);
    if (pl_status st = hip_check(hipGetLastError(), "k_he_clear")) return st;
    const int grid = (int)((3 * (size_t)cap + kHeBlock - 1) / kHeBlock);
    k_he_insert<<<grid, kHeBlock, 0, s>>>(tris, n_tri, cap, tab, slots, hslot);
    if (pl_status st = hip_check(hipGetLastError(), "k_he_insert")) return st;
    k_he_lookup<<<grid, kHeBlock, 0, s>>>(tris, n_tri, cap, tab, hslot, he);
    return hip_check(hipGetLastError(), "k_he_lookup");
}

}  // namespace pl
