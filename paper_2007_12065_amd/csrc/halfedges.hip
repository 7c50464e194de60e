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
// Both ways below key an edge by its undirected point pair (lo, hi), lo < hi,
// and keep per key the first half-edge of each direction (lo -> hi and
// hi -> lo); a half-edge that is the first of its direction then takes the
// other direction's first, if any.  Minima are order-free, so the output is
// deterministic whatever the order of the threads.
//
// Partitioned (up to kHeMaxBuckets buckets, 5.6 M triangles): the keys are
// dealt to buckets by hash and every bucket is solved in the LDS of one
// workgroup, so the common case has no atomics on global memory.
//   k_he_count     per chunk of kHeChunk half-edges: how many fall in each
//                  bucket (LDS histogram), one row per chunk
//   k_he_offsets   per bucket, over the chunks: where each chunk's entries
//                  start in the bucket's region (a scan), and the total
//   k_he_scatter   every half-edge's key and index into its bucket's region
//                  (kHeRegion entries), staged in LDS in bucket order first
//                  so that each chunk writes one contiguous run per bucket;
//                  entries past a full region go to an overflow list, which
//                  only the buckets that overflowed read
//   k_he_solve     one workgroup per bucket: an LDS hash table of the
//                  bucket's keys (compare-and-swap on the key, atomic min of
//                  each direction's first index), then each entry looks its
//                  key up and writes its twin
//   k_he_fallback  one workgroup that returns at once unless a bucket held
//                  more distinct keys than its LDS table (only inputs built
//                  against the hash can): then it redoes the whole mesh
//                  with the global table below, which overlays the regions
// Buckets: the power of two nearest above 3 cap / kHeBucketMean; a
// bucket's keys are the top bits of the hash, its LDS slot the low bits.
//
// Global table (larger meshes): a slot (16 bytes, one cache line holds
// eight) keeps the key and both first indices.  Three launches:
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
#include "tuning.h"

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

// ---------------------------------------------------------------------------
// Partitioned way
// ---------------------------------------------------------------------------

constexpr int kHeChunk = 4096;            // half-edges per row of the histogram
constexpr int kHeBucketMean = 2048;       // mean entries per bucket at n = 3 cap, at most
constexpr int kHeRegion = 3072;           // entries a bucket's region holds
constexpr int kHeLdsSlots = 4096;         // LDS table of a bucket (64 KB)
constexpr int kHeMaxBuckets = 8192;       // LDS histogram of a chunk (32 KB)
constexpr int kHeScanBuckets = 16;        // buckets per offsets workgroup
constexpr int kHeScanParts = 64;          // parts splitting the chunks of a bucket
constexpr int kHeScanBlock = kHeScanBuckets * kHeScanParts;

int bucket_bits(int cap) {
    const long long want = (3LL * cap + kHeBucketMean - 1) / kHeBucketMean;
    int lg = 0;
    while ((1LL << lg) < want) ++lg;
    return lg;
}

// the half-edge h of T: from tris[h] to the next vertex of its triangle
__device__ __forceinline__ void he_ends(const int32_t *__restrict__ tris, int h, int &a, int &b) {
    const int t = h / 3, j = h - 3 * t;
    a = tris[h];
    b = tris[3 * t + (j == 2 ? 0 : j + 1)];
}

__device__ __forceinline__ int he_bucket(unsigned long long mix, int lg) {
    return lg == 0 ? 0 : (int)(mix >> (64 - lg));
}

__global__ __launch_bounds__(kHeBlock) void k_he_count(const int32_t *__restrict__ tris,
                                                       const int32_t *__restrict__ n_tri, int cap,
                                                       int lg, int32_t *__restrict__ hist_out) {
    extern __shared__ int hist[];
    const int nb = 1 << lg;
    const int n = 3 * min(max(*n_tri, 0), cap);
    for (int i = threadIdx.x; i < nb; i += kHeBlock) hist[i] = 0;
    __syncthreads();
    const int base = (int)blockIdx.x * kHeChunk;
#pragma unroll 4
    for (int i = 0; i < kHeChunk / kHeBlock; ++i) {
        const int h = base + i * kHeBlock + (int)threadIdx.x;
        if (h >= n) break;
        int a, b;
        he_ends(tris, h, a, b);
        if (a != b) atomicAdd(&hist[he_bucket(he_mix(he_key(min(a, b), max(a, b))), lg)], 1);
    }
    __syncthreads();
    int32_t *row = hist_out + (size_t)blockIdx.x * nb;
    for (int i = threadIdx.x; i < nb; i += kHeBlock) row[i] = hist[i];
}

// 16 buckets per workgroup of 1024 threads: lane l of wave w takes bucket
// l mod 16 and part 4 w + l / 16 of the chunks (kHeScanParts parts); each
// part sums its chunks, the parts are scanned in LDS, then each part writes
// its chunks' starts.  Also clears the control words.
__global__ __launch_bounds__(kHeScanBlock) void k_he_offsets(
    const int32_t *__restrict__ hist, int chunks, int lg, int32_t *__restrict__ start,
    int32_t *__restrict__ total, int32_t *__restrict__ ctl) {
    __shared__ int part_sum[kHeScanParts][kHeScanBuckets];
    const int nb = 1 << lg;
    const int col = (int)threadIdx.x % kHeScanBuckets, part = (int)threadIdx.x / kHeScanBuckets;
    const int b = (int)blockIdx.x * kHeScanBuckets + col;
    if (blockIdx.x == 0 && threadIdx.x < 2) ctl[threadIdx.x] = 0;
    const int per = (chunks + kHeScanParts - 1) / kHeScanParts;
    const int c0 = part * per, c1 = min(c0 + per, chunks);
    int sum = 0;
    if (b < nb) {
#pragma unroll 4
        for (int c = c0; c < c1; ++c) sum += hist[(size_t)c * nb + b];
    }
    part_sum[part][col] = sum;
    __syncthreads();
    int run = 0, all = 0;
    for (int k = 0; k < kHeScanParts; ++k) {
        const int v = part_sum[k][col];
        run += k < part ? v : 0;
        all += v;
    }
    if (b >= nb) return;
    if (part == 0) total[b] = all;
    for (int c = c0; c < c1; ++c) {
        const int v = hist[(size_t)c * nb + b];
        start[(size_t)c * nb + b] = run;
        run += v;
    }
}

// Entry of a half-edge: its key and h | 2^31 when it runs hi -> lo.  The
// chunk's entries are first placed in LDS in bucket order (the chunk's
// counts, scanned), then written out: the chunk's entries of one bucket are
// one contiguous run of the bucket's region, written by consecutive lanes.
// LDS: the chunk's keys and entries (12 kHeChunk bytes), then its bucket
// starts and cursors (2 x 4 nb bytes).
__device__ __forceinline__ int block_exclusive_scan(int x, int *tmp) {
    const int lane = (int)threadIdx.x & (kWave - 1), w = (int)threadIdx.x / kWave;
    const int incl = wave_inclusive_scan(x);
    if (lane == kWave - 1) tmp[w] = incl;
    __syncthreads();
    int before = 0;
    for (int k = 0; k < w; ++k) before += tmp[k];
    return before + incl - x;
}

__global__ __launch_bounds__(kHeBlock) void k_he_scatter(
    const int32_t *__restrict__ tris, const int32_t *__restrict__ n_tri, int cap, int lg,
    const int32_t *__restrict__ hist, const int32_t *__restrict__ start,
    unsigned long long *__restrict__ keys, int32_t *__restrict__ hds, int32_t *__restrict__ ctl,
    unsigned long long *__restrict__ okeys, int32_t *__restrict__ ohds, int32_t *__restrict__ he) {
    extern __shared__ unsigned long long lds_u64[];
    __shared__ int tmp[kHeBlock / kWave];
    const int nb = 1 << lg;
    unsigned long long *skey = lds_u64;                                  // [kHeChunk]
    int *shd = reinterpret_cast<int *>(skey + kHeChunk);                 // [kHeChunk]
    int *lstart = shd + kHeChunk;                                        // [nb]
    int *lcur = lstart + nb;                                             // [nb]
    const int n = 3 * min(max(*n_tri, 0), cap);
    const int base = (int)blockIdx.x * kHeChunk;
    if (base >= n) return;
    const int32_t *crow = hist + (size_t)blockIdx.x * nb;
    const int32_t *srow = start + (size_t)blockIdx.x * nb;
    // the chunk's starts per bucket: each thread scans `per` consecutive
    // counts (nb < kHeBlock: one or none)
    const int per = (nb + kHeBlock - 1) / kHeBlock;
    const int b0 = (int)threadIdx.x * per;
    int own = 0;
    for (int k = 0; k < per && b0 + k < nb; ++k) own += crow[b0 + k];
    int run = block_exclusive_scan(own, tmp);
    for (int k = 0; k < per && b0 + k < nb; ++k) {
        lstart[b0 + k] = run;
        lcur[b0 + k] = run;
        run += crow[b0 + k];
    }
    __syncthreads();
#pragma unroll 4
    for (int i = 0; i < kHeChunk / kHeBlock; ++i) {
        const int h = base + i * kHeBlock + (int)threadIdx.x;
        if (h >= n) break;
        int a, b;
        he_ends(tris, h, a, b);
        if (a == b) {
            he[h] = -1;                  // from a point to itself: never paired
            continue;
        }
        const unsigned long long key = he_key(min(a, b), max(a, b));
        const int lp = atomicAdd(&lcur[he_bucket(he_mix(key), lg)], 1);
        skey[lp] = key;
        shd[lp] = a < b ? h : (h | INT_MIN);
    }
    __syncthreads();
    const int m = lcur[nb - 1];                  // entries staged: the last bucket's end
    for (int i = threadIdx.x; i < m; i += kHeBlock) {
        const unsigned long long key = skey[i];
        const int bk = he_bucket(he_mix(key), lg);
        const int pos = srow[bk] + (i - lstart[bk]);
        if (pos < kHeRegion) {
            keys[(size_t)bk * kHeRegion + pos] = key;
            hds[(size_t)bk * kHeRegion + pos] = shd[i];
        } else {
            const int o = atomicAdd(&ctl[0], 1);
            okeys[o] = key;
            ohds[o] = shd[i];
        }
    }
}

struct HeLdsTable {
    unsigned long long key[kHeLdsSlots];
    int2 first[kHeLdsSlots];             // first half-edge lo -> hi, hi -> lo
};

// Claims the key's slot and lowers its direction's first index; false when
// the table is full.
__device__ __forceinline__ bool he_lds_insert(HeLdsTable &t, unsigned long long key, int hd) {
    int slot = (int)(he_mix(key) & (kHeLdsSlots - 1));
    for (int p = 0; p < kHeLdsSlots; ++p) {
        const unsigned long long prev = atomicCAS(&t.key[slot], kEmpty, key);
        if (prev == kEmpty || prev == key) {
            atomicMin(hd < 0 ? &t.first[slot].y : &t.first[slot].x, hd & INT_MAX);
            return true;
        }
        slot = (slot + 1) & (kHeLdsSlots - 1);
    }
    return false;
}

// The twin of entry hd; false if its key is not in the table (it always is
// once every insert succeeded: the probe is bounded all the same).
__device__ __forceinline__ bool he_lds_twin(const HeLdsTable &t, unsigned long long key, int hd,
                                            int &twin) {
    int slot = (int)(he_mix(key) & (kHeLdsSlots - 1));
    for (int p = 0; p < kHeLdsSlots; ++p) {
        if (t.key[slot] == key) {
            const int2 f = t.first[slot];
            const int h = hd & INT_MAX;
            const int own = hd < 0 ? f.y : f.x, other = hd < 0 ? f.x : f.y;
            twin = own == h && other != INT_MAX ? other : -1;
            return true;
        }
        slot = (slot + 1) & (kHeLdsSlots - 1);
    }
    return false;
}

// The global-table way in one workgroup (the fallback).  The table is
// cleared, filled and read by this workgroup alone, all through atomics
// (which meet in L2).
__device__ void he_global_one_group(const int32_t *__restrict__ tris, int n, HeSlot *tab,
                                    unsigned long long slots, int32_t *__restrict__ he) {
    for (size_t i = threadIdx.x; i < slots; i += kHeBlock) {
        __hip_atomic_store(&tab[i].key, kEmpty, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&tab[i].fwd, INT_MAX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&tab[i].bwd, INT_MAX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    for (int h = threadIdx.x; h < n; h += kHeBlock) {
        int a, b;
        he_ends(tris, h, a, b);
        if (a == b) continue;
        const unsigned long long key = he_key(min(a, b), max(a, b));
        unsigned long long slot = he_slot(key, slots);
        for (unsigned long long p = 0; p < slots; ++p) {     // a free slot is always left
            const unsigned long long prev = atomicCAS(&tab[slot].key, kEmpty, key);
            if (prev == kEmpty || prev == key) {
                atomicMin(a < b ? &tab[slot].fwd : &tab[slot].bwd, h);
                break;
            }
            slot = slot + 1 == slots ? 0 : slot + 1;
        }
    }
    __syncthreads();
    for (int h = threadIdx.x; h < n; h += kHeBlock) {
        int a, b;
        he_ends(tris, h, a, b);
        int twin = -1;
        if (a != b) {
            const unsigned long long key = he_key(min(a, b), max(a, b));
            unsigned long long slot = he_slot(key, slots);
            for (unsigned long long p = 0; p < slots; ++p) {     // found at once or soon
                if (__hip_atomic_load(&tab[slot].key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == key) {
                    const int f = __hip_atomic_load(&tab[slot].fwd, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
                    const int g = __hip_atomic_load(&tab[slot].bwd, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
                    const int own = a < b ? f : g, other = a < b ? g : f;
                    if (own == h && other != INT_MAX) twin = other;
                    break;
                }
                slot = slot + 1 == slots ? 0 : slot + 1;
            }
        }
        he[h] = twin;
    }
}

// ctl: [0] overflow entries, [1] some bucket's table was full.
__global__ __launch_bounds__(kHeBlock) void k_he_solve(
    const unsigned long long *__restrict__ keys, const int32_t *__restrict__ hds,
    const int32_t *__restrict__ total, int32_t *ctl,
    const unsigned long long *__restrict__ okeys, const int32_t *__restrict__ ohds, int lg,
    int32_t *__restrict__ he) {
    __shared__ HeLdsTable t;
    const int bk = (int)blockIdx.x;
    for (int i = threadIdx.x; i < kHeLdsSlots; i += kHeBlock) {
        t.key[i] = kEmpty;
        t.first[i] = make_int2(INT_MAX, INT_MAX);
    }
    __syncthreads();
    const int tot = total[bk], m = min(tot, kHeRegion);
    // a bucket that overflowed also takes its entries from the overflow list
    const int no = tot > kHeRegion ? ctl[0] : 0;
    const unsigned long long *rk = keys + (size_t)bk * kHeRegion;
    const int32_t *rh = hds + (size_t)bk * kHeRegion;
    for (int i = threadIdx.x; i < m + no; i += kHeBlock) {
        const unsigned long long key = i < m ? rk[i] : okeys[i - m];
        if (i >= m && he_bucket(he_mix(key), lg) != bk) continue;
        if (!he_lds_insert(t, key, i < m ? rh[i] : ohds[i - m]))    // table full
            __hip_atomic_store(&ctl[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    // once any bucket's table was full the fallback redoes the whole mesh
    if (__hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
        for (int i = threadIdx.x; i < m + no; i += kHeBlock) {
            const unsigned long long key = i < m ? rk[i] : okeys[i - m];
            if (i >= m && he_bucket(he_mix(key), lg) != bk) continue;
            const int hd = i < m ? rh[i] : ohds[i - m];
            int twin;
            if (he_lds_twin(t, key, hd, twin))
                he[hd & INT_MAX] = twin;
            else
                __hip_atomic_store(&ctl[1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// One workgroup after the buckets: returns at once unless some bucket's
// table was full, and then redoes the whole mesh with the global table
// (the launch boundary orders it after every bucket's writes).
__global__ __launch_bounds__(kHeBlock) void k_he_fallback(const int32_t *__restrict__ tris,
                                                          const int32_t *__restrict__ n_tri,
                                                          int cap, const int32_t *__restrict__ ctl,
                                                          HeSlot *tab, unsigned long long slots,
                                                          int32_t *__restrict__ he) {
    if (ctl[1] == 0) return;
    he_global_one_group(tris, 3 * min(max(*n_tri, 0), cap), tab, slots, he);
}

// Workspace of the partitioned way: the histogram rows and their starts,
// the bucket totals, two control words, then the regions and the overflow
// list, which the fallback's global table overlays.
struct HeParts {
    int lg, nb, chunks;
    size_t hist, start, total, ctl, keys, hds, okeys, ohds, end;
};

HeParts he_parts(int cap) {
    HeParts p{};
    p.lg = bucket_bits(cap);
    p.nb = 1 << p.lg;
    p.chunks = (int)((3 * (size_t)cap + kHeChunk - 1) / kHeChunk);
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o += align_up(bytes, 256); return at; };
    p.hist = take(4 * (size_t)p.chunks * p.nb);
    p.start = take(4 * (size_t)p.chunks * p.nb);
    p.total = take(4 * (size_t)p.nb);
    p.ctl = take(8);
    const size_t region = (size_t)p.nb * kHeRegion;
    const size_t lists = align_up(8 * region, 256) + align_up(4 * region, 256) +
                         align_up(24 * (size_t)cap, 256) + align_up(12 * (size_t)cap, 256);
    p.keys = o;
    p.hds = p.keys + align_up(8 * region, 256);
    p.okeys = p.hds + align_up(4 * region, 256);
    p.ohds = p.okeys + align_up(24 * (size_t)cap, 256);
    const size_t table = sizeof(HeSlot) * table_slots(cap);
    p.end = o + std::max(lists, align_up(table, 256));
    return p;
}

bool partitioned(int cap) { return (1LL << bucket_bits(cap)) <= kHeMaxBuckets; }

}  // namespace

size_t user_halfedges_workspace(int cap) {
    if (partitioned(cap)) return he_parts(cap).end;
    return align_up(sizeof(HeSlot) * table_slots(cap), 256) + align_up(12 * (size_t)cap, 256);
}

pl_status launch_user_halfedges(const int32_t *tris, const int32_t *n_tri, int cap, int32_t *he,
                                void *ws, hipStream_t s) {
    if (cap == 0) return PL_OK;
    auto *w = static_cast<uint8_t *>(ws);
    if (partitioned(cap)) {
        const HeParts p = he_parts(cap);
        auto *hist = reinterpret_cast<int32_t *>(w + p.hist);
        auto *start = reinterpret_cast<int32_t *>(w + p.start);
        auto *total = reinterpret_cast<int32_t *>(w + p.total);
        auto *ctl = reinterpret_cast<int32_t *>(w + p.ctl);
        auto *keys = reinterpret_cast<unsigned long long *>(w + p.keys);
        auto *hds = reinterpret_cast<int32_t *>(w + p.hds);
        auto *okeys = reinterpret_cast<unsigned long long *>(w + p.okeys);
        auto *ohds = reinterpret_cast<int32_t *>(w + p.ohds);
        const size_t hist_lds = 4 * (size_t)p.nb;
        k_he_count<<<p.chunks, kHeBlock, hist_lds, s>>>(tris, n_tri, cap, p.lg, hist);
        if (pl_status st = hip_check(hipGetLastError(), "k_he_count")) return st;
        k_he_offsets<<<(p.nb + kHeScanBuckets - 1) / kHeScanBuckets, kHeScanBlock, 0, s>>>(
            hist, p.chunks, p.lg, start, total, ctl);
        if (pl_status st = hip_check(hipGetLastError(), "k_he_offsets")) return st;
        const size_t scatter_lds = 12 * (size_t)kHeChunk + 8 * (size_t)p.nb;
        if (pl_status st = allow_lds((const void *)k_he_scatter, scatter_lds)) return st;
        k_he_scatter<<<p.chunks, kHeBlock, scatter_lds, s>>>(tris, n_tri, cap, p.lg, hist, start,
                                                             keys, hds, ctl, okeys, ohds, he);
        if (pl_status st = hip_check(hipGetLastError(), "k_he_scatter")) return st;
        k_he_solve<<<p.nb, kHeBlock, 0, s>>>(keys, hds, total, ctl, okeys, ohds, p.lg, he);
        if (pl_status st = hip_check(hipGetLastError(), "k_he_solve")) return st;
        k_he_fallback<<<1, kHeBlock, 0, s>>>(tris, n_tri, cap, ctl,
                                             reinterpret_cast<HeSlot *>(w + p.keys),
                                             table_slots(cap), he);
        return hip_check(hipGetLastError(), "k_he_fallback");
    }
    const size_t slots = table_slots(cap);
    auto *tab = static_cast<HeSlot *>(ws);
    auto *hslot = reinterpret_cast<int32_t *>(w + align_up(sizeof(HeSlot) * slots, 256));
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
