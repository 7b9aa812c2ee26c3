// HIP kernels of the Free Join executor for gfx950 (wave64).
//
//  * selection push-down:   filter_lt                       (Section 2.1)
//  * COLT force:            force_* pipeline, used both for the root build
//                           and for lazy forcing of inner sub-tries
//                           (Section 4.2, figure "colt-impl", force())
//  * cover choice:          cover_choose / cover_fill        (Section 4.4)
//  * probe / intersect:     probe                           (Section 3.3 figure
//                           "fj-algo", vectorized as in Section 4.3)
//  * output:                emit_count / emit_rows          (bag multiplicities)
//  * scans:                 exclusive prefix sums used for load balancing
//
// No kernel here is a dense contraction, so nothing uses MFMA; every kernel is
// bound by HBM or L2/MALL traffic and written for coalesced streams, wave64
// ballots and one atomic per wave.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "fj_dev.h"
#include "fj_launch.h"

namespace fj {

typedef unsigned long long u64;

constexpr uint32_t kClaim = 0x80000000u;

// ----------------------------------------------------------------- hashing
// MurmurHash3 finalizers (Appleby): full avalanche for 32- and 64-bit keys.
__device__ __forceinline__ uint32_t mix32(uint32_t h) {
    h ^= h >> 16; h *= 0x85ebca6bu; h ^= h >> 13; h *= 0xc2b2ae35u; h ^= h >> 16;
    return h;
}
__device__ __forceinline__ u64 mix64(u64 k) {
    k ^= k >> 33; k *= 0xff51afd7ed558ccdull; k ^= k >> 33; k *= 0xc4ceb9fe1a85ec53ull; k ^= k >> 33;
    return k;
}

struct Key {
    uint32_t h;                  // handle (start position) of the probed trie
    uint32_t span;               // per-trie maps: the trie's offset count (its map has 2 span slots)
    int32_t v[FJ_MAX_COLS];
};

// Below the root each forced trie has a map of its own, as in the paper's
// COLT, where every trie node is a hash map: the trie starting at position p
// with n offsets (so at most n keys) owns the 2n slots from 2p, a disjoint
// range since tries of one level own disjoint position ranges.  All lookups
// of one trie, which the threads of one binding make together, touch only
// its own few cache lines instead of lines spread over the level's table.
// The start within the range takes the hash's top 32 bits times the range
// size (a multiply-shift range reduction, no division).
__device__ __forceinline__ u64 local_pick(u64 h, uint32_t n) { return ((h >> 32) * (u64)n) >> 32; }

// Probing walks forward slot by slot from the start of a 32-byte bucket:
// four KM_K32 slots (keys first, then values), or two 16-byte slots, so one
// 16-byte key load (KM_K32) or one pair of them usually settles a lookup.
// Insert and find use the same sequence.
constexpr int kBucketBytes = 32;
template <typename SlotT> __device__ __forceinline__ u64 bucket_start(u64 h, u64 mask) {
    return (h & mask) & ~(u64)(kBucketBytes / sizeof(SlotT) - 1);
}
__device__ __forceinline__ u64 k32_bucket(uint32_t h, u64 mask) { return (h & mask) & ~(u64)(kK32Bucket - 1); }

// A KM_K32 key's membership-filter bits (two, from its hash's top ten bits;
// the bucket takes the low bits) and filter word (its home bucket, shifted).
__device__ __forceinline__ uint32_t bloom_bits(uint32_t h) { return (1u << (h >> 27)) | (1u << ((h >> 22) & 31u)); }
__device__ __forceinline__ uint32_t bloom_word(uint32_t h, u64 mask, uint32_t shift) {
    return (uint32_t)(k32_bucket(h, mask) >> (2 + shift));
}

__device__ __forceinline__ u64 pack64(const LevelDev &L, const Key &k) {
    // root with two key columns: (v0, v1); below the root: (handle, v0)
    return L.nk == 2 ? ((u64)(uint32_t)k.v[0] << 32) | (uint32_t)k.v[1]
                     : ((u64)k.h << 32) | (uint32_t)k.v[0];
}

__device__ __forceinline__ u64 rep_hash(const Key &k, int nk) {
    u64 x = mix64(((u64)k.h << 32) ^ 0x9E3779B97F4A7C15ull);
    for (int j = 0; j < nk; j++) x = mix64(x ^ (u64)(uint32_t)k.v[j]);
    return x;
}

__device__ __forceinline__ bool rep_equal(const LevelDev &L, const int32_t *const *cols, uint32_t row,
                                          const Key &k) {
    for (int j = 0; j < L.nk; j++)
        if (cols[L.kcol[j]][row] != k.v[j]) return false;
    return true;
}

// get(): the slot of key k in level L's map, or ~0 when absent.  Every hit
// compares the full key.  Tables are immutable while probes run.
__device__ __forceinline__ u64 table_find(const LevelDev &L, const int32_t *const *cols, const Key &k) {
    const u64 mask = L.mask;
    if (L.mode == KM_K32) {
        const uint32_t *T = (const uint32_t *)L.table;
        uint32_t key = (uint32_t)k.v[0];
        if (key == kEmpty32) return T[k32_key_word(mask + 1)] ? mask + 1 : ~0ull;
        // a bucket's four keys in one 16-byte load, then the next bucket
        u64 b = k32_bucket(mix32(key), mask);
        for (u64 n = 0; n <= k32_part_mask(mask); n += kK32Bucket) {
            const uint4 q = *(const uint4 *)(T + k32_key_word(b));
            const uint32_t ks[kK32Bucket] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int s = 0; s < kK32Bucket; s++) {
                if (ks[s] == key) return b + s;
                if (ks[s] == kEmpty32) return ~0ull;
            }
            b = k32_next(b, mask);
        }
    } else if (L.mode == KM_K64) {
        const Slot64 *T = (const Slot64 *)L.table;
        u64 key = pack64(L, k);
        if (L.local) {
            // the trie's own buckets: span pairs of slots from 2h
            if (k.span == 0) return ~0ull;
            const u64 base = 2 * (u64)k.h, end = base + 2 * (u64)k.span;
            u64 b = base + 2 * local_pick(mix64(key), k.span);
            for (uint32_t n = 0; n < k.span; n++) {
                const u64 c0 = T[b].key, c1 = T[b + 1].key;
                if (c0 == key) return b;
                if (c0 == kEmpty64) return ~0ull;
                if (c1 == key) return b + 1;
                if (c1 == kEmpty64) return ~0ull;
                b += 2;
                if (b == end) b = base;
            }
            return L.nslots;
        }
        if (key == kEmpty64) return T[mask + 1].key ? mask + 1 : ~0ull;
        // a bucket's two slots in one 32-byte read, then the next bucket
        u64 b = bucket_start<Slot64>(mix64(key), mask);
        for (u64 n = 0; n <= mask; n += 2) {
            const u64 c0 = T[b].key, c1 = T[b + 1].key;
            if (c0 == key) return b;
            if (c0 == kEmpty64) return ~0ull;
            if (c1 == key) return b + 1;
            if (c1 == kEmpty64) return ~0ull;
            b = (b + 2) & mask;
        }
    } else {
        const SlotRep *T = (const SlotRep *)L.table;
        const u64 hh = rep_hash(k, L.nk);
        const u64 base = L.local ? 2 * (u64)k.h : 0, m = L.local ? 2 * (u64)k.span : mask + 1;
        if (m == 0) return ~0ull;
        u64 i = L.local ? local_pick(hh, 2 * k.span) : bucket_start<SlotRep>(hh, mask);
        for (u64 n = 0; n < m; n++) {
            u64 c = T[base + i].hr;
            if (c == kEmpty64) return ~0ull;
            if ((uint32_t)c == k.h && (uint32_t)(c >> 32) < L.nrows &&
                rep_equal(L, cols, (uint32_t)(c >> 32), k)) return base + i;
            if (++i == m) i = 0;
        }
    }
    return L.nslots;  // no empty slot: the map is corrupt (callers check the index)
}

__device__ __forceinline__ uint32_t slot_val(const LevelDev &L, u64 i) {
    if (L.mode == KM_K32) return ((const uint32_t *)L.table)[k32_key_word(i) + 4];
    if (L.mode == KM_K64) return ((const Slot64 *)L.table)[i].val;
    return ((const SlotRep *)L.table)[i].val;
}

__device__ __forceinline__ void set_slot_val(const LevelDev &L, u64 i, uint32_t v) {
    if (L.mode == KM_K32) ((uint32_t *)L.table)[k32_key_word(i) + 4] = v;
    else if (L.mode == KM_K64) ((Slot64 *)L.table)[i].val = v;
    else ((SlotRep *)L.table)[i].val = v;
}

__device__ __forceinline__ uint32_t *slot_val_ptr(const LevelDev &L, u64 i) {
    if (L.mode == KM_K32) return (uint32_t *)L.table + k32_key_word(i) + 4;
    if (L.mode == KM_K64) return &((Slot64 *)L.table)[i].val;
    return &((SlotRep *)L.table)[i].val;
}

// Insert-or-find for force(); `row` is the representative row for KM_REP.
__device__ __forceinline__ u64 table_insert(const LevelDev &L, const int32_t *const *cols, const Key &k,
                                            uint32_t row, bool &claimed) {
    const u64 mask = L.mask;
    claimed = false;
    if (L.mode == KM_K32) {
        uint32_t *T = (uint32_t *)L.table;
        uint32_t key = (uint32_t)k.v[0];
        if (key == kEmpty32) {
            claimed = atomicCAS(&T[k32_key_word(mask + 1)], 0u, 1u) == 0u;
            return mask + 1;
        }
        // read a bucket's keys (one 16-byte load), then compare-and-swap
        // only the first slot seen empty; the read may be stale, but slots
        // only ever go from empty to a key and the swap returns the true
        // occupant, so a lost race just moves on in slot order
        u64 b = k32_bucket(mix32(key), mask);
        for (u64 n = 0; n <= k32_part_mask(mask); n += kK32Bucket) {
            const uint4 q = *(const uint4 *)(T + k32_key_word(b));
            const uint32_t ks[kK32Bucket] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int s = 0; s < kK32Bucket; s++) {
                uint32_t c = ks[s];
                if (c == kEmpty32) {
                    c = atomicCAS(&T[k32_key_word(b + s)], kEmpty32, key);
                    if (c == kEmpty32) { claimed = true; return b + s; }
                }
                if (c == key) return b + s;
            }
            b = k32_next(b, mask);
        }
    } else if (L.mode == KM_K64) {
        Slot64 *T = (Slot64 *)L.table;
        u64 key = pack64(L, k);
        // as for KM_K32: read the bucket's two keys, swap the first empty one
        if (L.local) {
            if (k.span == 0) return L.nslots;
            const u64 base = 2 * (u64)k.h, end = base + 2 * (u64)k.span;
            u64 b = base + 2 * local_pick(mix64(key), k.span);
            for (uint32_t n = 0; n < k.span; n++) {
                const u64 ks[2] = {T[b].key, T[b + 1].key};
#pragma unroll
                for (int s = 0; s < 2; s++) {
                    u64 c = ks[s];
                    if (c == kEmpty64) {
                        c = atomicCAS(&T[b + s].key, kEmpty64, key);
                        if (c == kEmpty64) { claimed = true; return b + s; }
                    }
                    if (c == key) return b + s;
                }
                b += 2;
                if (b == end) b = base;
            }
            return L.nslots;
        }
        if (key == kEmpty64) {
            claimed = atomicCAS(&T[mask + 1].key, 0ull, 1ull) == 0ull;
            return mask + 1;
        }
        u64 b = bucket_start<Slot64>(mix64(key), mask);
        for (u64 n = 0; n <= mask; n += 2) {
            const u64 ks[2] = {T[b].key, T[b + 1].key};
#pragma unroll
            for (int s = 0; s < 2; s++) {
                u64 c = ks[s];
                if (c == kEmpty64) {
                    c = atomicCAS(&T[b + s].key, kEmpty64, key);
                    if (c == kEmpty64) { claimed = true; return b + s; }
                }
                if (c == key) return b + s;
            }
            b = (b + 2) & mask;
        }
    } else {
        SlotRep *T = (SlotRep *)L.table;
        u64 mine = ((u64)row << 32) | k.h;
        const u64 hh = rep_hash(k, L.nk);
        const u64 base = L.local ? 2 * (u64)k.h : 0, m = L.local ? 2 * (u64)k.span : mask + 1;
        if (m == 0) return L.nslots;
        u64 i = L.local ? local_pick(hh, 2 * k.span) : bucket_start<SlotRep>(hh, mask);
        for (u64 n = 0; n < m; n++) {
            u64 c = T[base + i].hr;   // may be stale-empty; the CAS settles it
            if (c == kEmpty64) {
                u64 old = atomicCAS(&T[base + i].hr, kEmpty64, mine);
                if (old == kEmpty64) { claimed = true; return base + i; }
                c = old;
            }
            if ((uint32_t)c == k.h && (uint32_t)(c >> 32) < L.nrows &&
                rep_equal(L, cols, (uint32_t)(c >> 32), k)) return base + i;
            if (++i == m) i = 0;
        }
    }
    return L.nslots;  // the map is full: callers check the index
}

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ u64 wave_sum_u64(u64 v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Wave-aggregated reservation: returns this lane's slot for `pred` lanes.
// Block-wide forms (every thread of the block calls them; blocks of at most
// 1024 threads; lds holds 17 words): one atomic per block instead of one per
// wave.
__device__ __forceinline__ void block_add_count(u64 v, StatusDev *st, u64 *lds) {
    v = wave_sum_u64(v);
    const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (__lane_id() == 0) lds[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 t = 0;
        for (int w = 0; w < nw; w++) t += lds[w];
        if (t) atomicAdd(&st->count_part[(blockIdx.x % kCountParts) * kPartStride], t);
    }
    __syncthreads();
}

__device__ __forceinline__ u64 block_reserve(bool pred, u64 *counter, u64 *lds) {
    const u64 mask = __ballot(pred);
    const int lane = __lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0) lds[wid] = (u64)__popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        u64 off = 0;
        for (int w = 0; w < nw; w++) {
            const u64 t = lds[w];
            lds[w] = off;
            off += t;
        }
        lds[16] = off ? atomicAdd(counter, off) : 0ull;
    }
    __syncthreads();
    const u64 base = lds[16] + lds[wid] + (u64)__popcll(mask & ((1ull << lane) - 1ull));
    __syncthreads();
    return base;
}

__device__ __forceinline__ u64 wave_reserve(bool pred, u64 *counter) {
    const u64 mask = __ballot(pred);
    const int lane = __lane_id();
    const int n = __popcll(mask);
    u64 base = 0;
    const int leader = n ? (__ffsll((long long)mask) - 1) : 0;
    if (n && lane == leader) base = atomicAdd(counter, (u64)n);
    base = __shfl(base, leader, 64);
    return base + __popcll(mask & ((1ull << lane) - 1ull));
}

__device__ __forceinline__ uint32_t upper_entry(const u64 *starts, uint32_t lo, uint32_t hi, u64 g) {
    // largest e in [lo, hi) with starts[e] <= g (starts non-decreasing, starts[lo] <= g)
    while (hi - lo > 1) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (starts[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t upper_entry32(const uint32_t *starts, uint32_t lo, uint32_t hi, uint32_t g) {
    while (hi - lo > 1) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (starts[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ fills
template <typename T>
__global__ void k_fill(T *p, u64 n, T v) {
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    u64 stride = (u64)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// Fill a list of regions with periodic 32-bit patterns (table slots, zeroed
// state arrays) in one launch; also set the root handle and the one-handle
// force queue of the root.
__global__ void k_fill_list(const FillList *__restrict__ fl, LevelDev root, uint32_t nroot, uint32_t *pre) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    const u64 tid = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    for (int k = 0; k < fl->n; k++) {
        const FillRegion &r = fl->r[k];
        const u64 m = (u64)r.period - 1;   // periods are 1, 2, 4 or 8
        for (u64 i = tid; i < r.nwords; i += stride) r.p[i] = r.pat[i & m];
    }
    if (tid == 0 && root.len) {
        root.len[0] = nroot;
        root.st[0] = 0;
        if (root.fq) root.fq[0] = 0;
        if (pre) { pre[0] = 0; pre[1] = nroot; }
    }
}

// ------------------------------------------------------------------ scans
// Exclusive scan of n values (u32 or u64) in three phases: per-block sums,
// a single-block scan of the sums, and a per-block rescan with offsets.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *lds, T &total) {
    // v: per-thread value; returns exclusive prefix over the block
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T x = v;
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) { T t = lds[w]; lds[w] = run; run += t; }
        lds[16] = run;
    }
    __syncthreads();
    T r = lds[wid] + x - v;
    total = lds[16];
    __syncthreads();
    return r;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const T *in, u64 n, T *bsum) {
    __shared__ T lds[17];
    u64 base = (u64)blockIdx.x * kScanTile + (u64)threadIdx.x * kScanItems;
    T s = 0;
    for (int j = 0; j < kScanItems; j++) if (base + j < n) s += in[base + j];
    T tot;
    block_excl_scan<T>(s, lds, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_scan_blocks(T *bsum, u64 nb, T *total_out, T *out_last) {
    __shared__ T lds[17];
    T carry = 0;
    for (u64 c = 0; c < nb; c += kScanThreads) {
        u64 i = c + threadIdx.x;
        T v = i < nb ? bsum[i] : 0;
        T tot;
        T ex = block_excl_scan<T>(v, lds, tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        if (total_out) *total_out = carry;
        if (out_last) *out_last = carry;
    }
}

// The block-sum scan of an emit's per-binding row counts, which also places
// the emit in the output: its first row follows the rows written so far and
// its row count is cut to the output's capacity.
__global__ void __launch_bounds__(kScanThreads) k_scan_blocks_emit(u64 *bsum, u64 nb, u64 *out_last,
                                                                   StatusDev *st, u64 cap) {
    __shared__ u64 lds[17];
    u64 carry = 0;
    for (u64 c = 0; c < nb; c += kScanThreads) {
        u64 i = c + threadIdx.x;
        u64 v = i < nb ? bsum[i] : 0;
        u64 tot;
        u64 ex = block_excl_scan<u64>(v, lds, tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        *out_last = carry;
        st->total = carry;
        const u64 base = st->written;
        const u64 rows = base < cap ? (carry < cap - base ? carry : cap - base) : 0;
        st->emit_base = base;
        st->emit_rows = rows;
        st->written = base + rows;
    }
}

template <typename T>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const T *in, T *out, u64 n, const T *bsum) {
    __shared__ T lds[17];
    u64 base = (u64)blockIdx.x * kScanTile + (u64)threadIdx.x * kScanItems;
    T v[kScanItems];
    T s = 0;
    for (int j = 0; j < kScanItems; j++) { v[j] = (base + j < n) ? in[base + j] : 0; s += v[j]; }
    T tot;
    T ex = block_excl_scan<T>(s, lds, tot) + bsum[blockIdx.x];
    for (int j = 0; j < kScanItems; j++) {
        if (base + j < n) out[base + j] = ex;
        ex += v[j];
    }
}

template <typename T>
__global__ void k_scan_total(T *out, u64 n, const T *total) {
    if (threadIdx.x == 0 && blockIdx.x == 0) out[n] = *total;
}

// ----------------------------------------------------------------- filter
// sigma_{col < bound}: row offsets of passing rows, in row order.  Three
// launches without atomics: per-block pass counts, a scan of the counts, and
// a rescan that writes each block's rows at its offset.  Each thread reads
// four consecutive rows with one 16-byte load.
constexpr int kFilterRows = 4;
constexpr int kFilterBlock = 256 * kFilterRows;

// Bit r: row first + r passes (ROWS consecutive rows, a multiple of four,
// read with 16-byte loads when the column is 16-byte aligned).
template <int ROWS>
__device__ __forceinline__ uint32_t filter_bits_n(const int32_t *col, u64 n, int32_t bound, u64 first, bool vec) {
    static_assert(ROWS % 4 == 0 && ROWS <= 32, "whole 16-byte loads, one bit a row");
    uint32_t bits = 0;
    if (vec && first + ROWS <= n) {
        int4 x[ROWS / 4];
#pragma unroll
        for (int q = 0; q < ROWS / 4; q++) x[q] = *(const int4 *)(col + first + 4 * q);
#pragma unroll
        for (int q = 0; q < ROWS / 4; q++)
            bits |= ((uint32_t)(x[q].x < bound) | ((uint32_t)(x[q].y < bound) << 1) |
                     ((uint32_t)(x[q].z < bound) << 2) | ((uint32_t)(x[q].w < bound) << 3)) << (4 * q);
    } else {
        for (int r = 0; r < ROWS; r++)
            if (first + r < n && col[first + r] < bound) bits |= 1u << r;
    }
    return bits;
}
__device__ __forceinline__ uint32_t filter_bits(const int32_t *col, u64 n, int32_t bound, u64 first, bool vec) {
    return filter_bits_n<kFilterRows>(col, n, bound, first, vec);
}

__global__ void __launch_bounds__(256) k_filter_count(const int32_t *__restrict__ col, u64 n, int32_t bound, int vec,
                                                      uint32_t *bsum) {
    __shared__ uint32_t lds[17];
    const u64 first = ((u64)blockIdx.x * 256 + threadIdx.x) * kFilterRows;
    const uint32_t bits = filter_bits(col, n, bound, first, vec);
    uint32_t tot;
    block_excl_scan<uint32_t>((uint32_t)__popc(bits), lds, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_filter_write(const int32_t *__restrict__ col, u64 n, int32_t bound, int vec,
                                                      const uint32_t *bsum, uint32_t *__restrict__ out) {
    __shared__ uint32_t lds[17];
    const u64 first = ((u64)blockIdx.x * 256 + threadIdx.x) * kFilterRows;
    const uint32_t bits = filter_bits(col, n, bound, first, vec);
    uint32_t tot;
    uint32_t pos = bsum[blockIdx.x] + block_excl_scan<uint32_t>((uint32_t)__popc(bits), lds, tot);
    for (int r = 0; r < kFilterRows; r++)
        if (bits & (1u << r)) out[pos++] = (uint32_t)(first + r);
}

// Many selections in two launches: block b of a grouped launch belongs to
// selection i with bpre[i] <= b < bpre[i + 1] and is its block b - bpre[i].
// The first launch counts each block's kept rows; in the second, each block
// sums the counts of its selection's earlier blocks (a few hundred
// contiguous words) for its place, and writes its rows in order.  A thread
// takes sixteen consecutive rows, so that a million-row selection is a
// few hundred blocks, all resident at once.
constexpr int kFilterGroupRows = 16;
constexpr int kFilterGroupBlock = 256 * kFilterGroupRows;
struct FilterGroup {
    int n;
    const int32_t *col[FJ_MAX_ATOMS];
    unsigned long long rows[FJ_MAX_ATOMS];
    int32_t bound[FJ_MAX_ATOMS];
    int vec[FJ_MAX_ATOMS];
    uint32_t *out[FJ_MAX_ATOMS];
    uint32_t *bsum[FJ_MAX_ATOMS];
    uint32_t *total[FJ_MAX_ATOMS];
    uint32_t bpre[FJ_MAX_ATOMS + 1];
};

__device__ __forceinline__ int filter_member(const FilterGroup &g, uint32_t b) {
    int i = 0;
    while (i + 1 < g.n && g.bpre[i + 1] <= b) i++;
    return i;
}

__global__ void __launch_bounds__(256) k_filter_count_group(FilterGroup g) {
    __shared__ uint32_t lds[17];
    const int i = filter_member(g, blockIdx.x);
    const uint32_t b = blockIdx.x - g.bpre[i];
    const u64 first = ((u64)b * 256 + threadIdx.x) * kFilterGroupRows;
    const uint32_t bits = filter_bits_n<kFilterGroupRows>(g.col[i], g.rows[i], g.bound[i], first, g.vec[i]);
    uint32_t tot;
    block_excl_scan<uint32_t>((uint32_t)__popc(bits), lds, tot);
    if (threadIdx.x == 0) g.bsum[i][b] = tot;
}

__global__ void __launch_bounds__(256) k_filter_write_group(FilterGroup g) {
    __shared__ uint32_t lds[17];
    const int i = filter_member(g, blockIdx.x);
    const uint32_t b = blockIdx.x - g.bpre[i];
    const uint32_t *bsum = g.bsum[i];
    uint32_t part = 0;
    for (uint32_t k = threadIdx.x; k < b; k += 256) part += bsum[k];
    uint32_t base;
    block_excl_scan<uint32_t>(part, lds, base);
    const u64 first = ((u64)b * 256 + threadIdx.x) * kFilterGroupRows;
    const uint32_t bits = filter_bits_n<kFilterGroupRows>(g.col[i], g.rows[i], g.bound[i], first, g.vec[i]);
    uint32_t tot;
    uint32_t pos = base + block_excl_scan<uint32_t>((uint32_t)__popc(bits), lds, tot);
    if (threadIdx.x == 0 && b + 1 == g.bpre[i + 1] - g.bpre[i]) *g.total[i] = base + tot;
    uint32_t *out = g.out[i];
    for (uint32_t m = bits; m; m &= m - 1) out[pos++] = (uint32_t)(first + __builtin_ctz(m));
}

// ------------------------------------------------------------------ checks
// Every indexed access of the join kernels is checked against the size of
// the array it touches.  A failed check records the source line in the status
// block and the access is skipped, so corrupt state becomes an error status on
// the host instead of a memory fault.
__device__ __noinline__ void fj_bad(StatusDev *st, int line) {
    atomicCAS(&st->err_line, 0u, (uint32_t)line);
    atomicAdd(&st->err_count, 1u);
}
#define CK(cond) ((cond) ? true : (fj_bad(status, __LINE__), false))

// ------------------------------------------------------------------ force
// force() of every handle in a queue (atom a, level l): regroup each
// handle's offsets by the level's key into child segments of level l + 1
// occupying the handle's own position range, and fill the level's map with
// (handle, key) -> child start.


// Locate work item w: queue entry j, handle p, index i in it, base row.
__device__ __forceinline__ bool force_item(const ForceArgs &a, uint32_t w, uint32_t &j, uint32_t &p,
                                           uint32_t &i, uint32_t &row) {
    StatusDev *status = a.status;
    j = a.nh == 1 ? 0u : upper_entry32(a.pre, 0, a.nh, w);
    if (!CK(j < a.nh)) return false;
    p = a.fq[j];
    i = w - a.pre[j];
    if (!CK((u64)p + i < a.L.npos && w < a.wcap)) return false;
    row = a.L.offs ? a.L.offs[p + i] : p + i;
    return CK(row < a.L.nrows);
}

__global__ void __launch_bounds__(256) k_fq_lens(LevelDev L, const uint32_t *fq, uint32_t nh, uint32_t *lens,
                                                 StatusDev *status) {
    uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nh) return;
    uint32_t p = fq[j];
    lens[j] = CK(p < L.npos) ? L.len[p] : 0u;
}

// Pass 1: insert each offset's key (handle, key values) and count the
// offsets per key in the slot's value word; the inserting item is marked.
// Called by every active lane of a wave (wave-wide rounds below).
__device__ __forceinline__ void force_insert_item(const ForceArgs &a, uint32_t w) {
    StatusDev *status = a.status;
    uint32_t j, p, i, row;
    bool todo = force_item(a, w, j, p, i, row);
    if (!todo) a.wslot[w] = 0;
    if (todo && a.L.mode == KM_ZERO) {     // one key: the first offset claims it
        a.wslot[w] = i == 0 ? kClaim : 0u;
        todo = false;
    }
    Key k;
    k.h = p;
    k.span = 0;
    k.v[0] = k.v[1] = 0;
    if (todo) {
        for (int c = 0; c < a.L.nk; c++) k.v[c] = a.cols[a.L.kcol[c]][row];
        if (a.L.local) k.span = a.L.len[p];
    }
    // Up to two rounds: the lanes holding the same key (same map, handle and
    // key of at most two columns) as the wave's first remaining lane insert
    // it once and add their number at once, which keeps a heavy key under
    // skew from serializing many atomics on one slot.
    const int lane = __lane_id();
    for (int round = 0; round < 2; round++) {
        const u64 act = __ballot(todo);
        if (act == 0) break;
        const int leader = __ffsll((long long)act) - 1;
        const u64 tb = (u64)(uintptr_t)a.L.table;
        const u64 ltb = __shfl(tb, leader, 64);
        const uint32_t lh = __shfl(k.h, leader, 64);
        const int32_t l0 = __shfl(k.v[0], leader, 64), l1 = __shfl(k.v[1], leader, 64);
        const bool same = todo && a.L.mode != KM_REP && tb == ltb && k.h == lh && k.v[0] == l0 &&
                          (a.L.nk < 2 || k.v[1] == l1);
        const u64 grp = __ballot(same);
        const int m = __popcll(grp);
        if (m < 2) break;
        uint32_t ws = 0;
        int good = 0;
        if (lane == leader) {
            bool claimed;
            const u64 sl = table_insert(a.L, a.cols, k, row, claimed);
            if (CK(sl < a.L.nslots && sl < kClaim)) {
                atomicAdd(slot_val_ptr(a.L, sl), (uint32_t)(claimed ? m - 1 : m));
                ws = (uint32_t)sl | (claimed ? kClaim : 0u);
                good = 1;
            }
        }
        ws = __shfl(ws, leader, 64);
        good = __shfl(good, leader, 64);
        if (same) {
            a.wslot[w] = !good ? 0u : (lane == leader ? ws : (ws & ~kClaim));
            todo = false;
        }
    }
    if (!todo) return;
    bool claimed;
    const u64 sl = table_insert(a.L, a.cols, k, row, claimed);
    if (!CK(sl < a.L.nslots && sl < kClaim)) { a.wslot[w] = 0; return; }
    // the slot's value counts the offsets after the first: unique keys cost
    // one CAS and no counter update
    if (!claimed) atomicAdd(slot_val_ptr(a.L, sl), 1u);
    a.wslot[w] = (uint32_t)sl | (claimed ? kClaim : 0u);
}

__global__ void __launch_bounds__(256) k_force_insert(ForceArgs a) {
    uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < a.W) force_insert_item(a, w);
}

// Pass 2: each key's (1, offset count) at its inserting item; a scan of
// these pairs gives every key its rank among its handle's keys (high half)
// and the start of its child segment (low half).
__device__ __forceinline__ void force_pack_item(const ForceArgs &a, uint32_t w) {
    const uint32_t ws = a.wslot[w];
    u64 v = 0;
    if (ws & kClaim) {
        uint32_t cnt;
        if (a.L.mode == KM_ZERO) {
            const uint32_t j = a.nh == 1 ? 0u : upper_entry32(a.pre, 0, a.nh, w);
            cnt = a.pre[j + 1] - a.pre[j];
        } else {
            cnt = *slot_val_ptr(a.L, ws & ~kClaim) + 1u;
        }
        v = (1ull << 32) | cnt;
    }
    a.cntv[w] = v;
}

__global__ void __launch_bounds__(256) k_force_pack(ForceArgs a) {
    uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < a.W) force_pack_item(a, w);
}

// Pass 3: keys publish their child segment: key list entry, child length,
// scatter cursor, and the map value becomes the child's start.  The first
// item of each handle records its key count (the forced state).
__device__ __forceinline__ void force_children_item(const ForceArgs &a, uint32_t w) {
    StatusDev *status = a.status;
    uint32_t j, p, i, row;
    if (!force_item(a, w, j, p, i, row)) return;
    const u64 base = a.ex[a.pre[j]];
    if (i == 0) {
        const uint32_t nkeys = (uint32_t)(a.ex[a.pre[j + 1]] >> 32) - (uint32_t)(base >> 32);
        a.L.rank_ctr[p] = nkeys;
        a.L.st[p] = nkeys + 1;
    }
    const uint32_t ws = a.wslot[w];
    if (!(ws & kClaim)) return;
    const uint32_t rank = (uint32_t)(a.ex[w] >> 32) - (uint32_t)(base >> 32);
    const uint32_t s = p + ((uint32_t)a.ex[w] - (uint32_t)base);
    const uint32_t cnt = (uint32_t)a.cntv[w];
    if (!CK((u64)p + rank < a.L.npos && s < a.C.npos && cnt > 0)) return;
    a.L.kl[p + rank] = s;
    if (a.L.kk) {
        a.L.kk[p + rank] = a.cols[a.L.kcol[0]][row];
        a.L.kn[p + rank] = cnt;
    }
    a.C.len[s] = cnt;
    a.L.cnt[s] = cnt;
    if (a.L.mode != KM_ZERO) *slot_val_ptr(a.L, ws & ~kClaim) = s;
    // 16-byte slots also carry the child's length: a lookup that reaches an
    // offset vector reads its multiplicity from the slot it found
    if (a.L.mode == KM_K64) ((Slot64 *)a.L.table)[ws & ~kClaim].pad = cnt;
}

__global__ void __launch_bounds__(256) k_force_children(ForceArgs a) {
    uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < a.W) force_children_item(a, w);
}

// Pass 4: every offset moves into its key's child segment.  The cursor
// counts down to zero, leaving the counter array clean for the next force.
// Called by every active lane of a wave (wave-wide rounds below).
__device__ __forceinline__ void force_scatter_item(const ForceArgs &a, uint32_t w) {
    StatusDev *status = a.status;
    uint32_t j, p, i, row;
    bool todo = force_item(a, w, j, p, i, row);
    uint32_t s = 0;
    if (todo) {
        const uint32_t ws = a.wslot[w];
        s = a.L.mode == KM_ZERO ? p : *slot_val_ptr(a.L, ws & ~kClaim);
        todo = CK(s >= p && s < a.C.npos);
    }
    // Up to two rounds: the lanes moving into the same child segment as the
    // wave's first remaining lane take consecutive positions with one
    // subtraction from its cursor.
    const int lane = __lane_id();
    for (int round = 0; round < 2; round++) {
        const u64 act = __ballot(todo);
        if (act == 0) break;
        const int leader = __ffsll((long long)act) - 1;
        const u64 cp = (u64)(uintptr_t)a.L.cnt;
        const u64 lcp = __shfl(cp, leader, 64);
        const uint32_t ls = __shfl(s, leader, 64);
        const bool same = todo && cp == lcp && s == ls;
        const u64 grp = __ballot(same);
        const int m = __popcll(grp);
        if (m < 2) break;
        uint32_t old = 0;
        if (lane == leader) old = atomicSub(&a.L.cnt[s], (uint32_t)m);
        old = __shfl(old, leader, 64);
        if (same) {
            todo = false;
            const uint32_t r = (uint32_t)__popcll(grp & ((1ull << lane) - 1ull));
            const uint32_t pos = s + old - 1u - r;
            if (CK(old >= (uint32_t)m && pos >= s && pos < p + a.L.len[p])) {
                a.C.offs[pos] = row;
                if (a.C.kv) a.C.kv[pos] = a.cols[a.C.kcol[0]][row];
            }
        }
    }
    if (!todo) return;
    const uint32_t pos = s + atomicSub(&a.L.cnt[s], 1u) - 1u;
    if (!CK(pos >= s && pos < p + a.L.len[p])) return;
    a.C.offs[pos] = row;
    if (a.C.kv) a.C.kv[pos] = a.cols[a.C.kcol[0]][row];
}

__global__ void __launch_bounds__(256) k_force_scatter(ForceArgs a) {
    uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w < a.W) force_scatter_item(a, w);
}

// ------------------------------------------------------- grouped root builds
// The root builds of many COLTs in one launch per phase: work item g of the
// group belongs to the COLT k with wpre[k] <= g < wpre[k + 1] and is that
// COLT's item g - wpre[k].  Each COLT's descriptor points at its own slice of
// the group's scratch, so one scan over the concatenated per-item pairs gives
// every COLT its ranks and child starts.

__device__ __forceinline__ int group_member(const u64 *__restrict__ wpre, int n, u64 g) {
    int lo = 0, hi = n;   // wpre[lo] <= g < wpre[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (wpre[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <int PHASE>
__device__ __forceinline__ void group_item(const ForceArgs &a, uint32_t w) {
    if (PHASE == 0) force_insert_item(a, w);
    else if (PHASE == 1) force_pack_item(a, w);
    else if (PHASE == 2) force_children_item(a, w);
    else force_scatter_item(a, w);
}

template <int PHASE>
__global__ void __launch_bounds__(256) k_group_force(const ForceArgs *__restrict__ descs, const u64 *__restrict__ wpre,
                                                     int n, u64 wtot) {
    // the block's first member by one search; lanes step on at boundaries
    const u64 gb = (u64)blockIdx.x * 256;
    if (gb >= wtot) return;
    const int kb = group_member(wpre, n, gb);
    const u64 g = gb + threadIdx.x;
    if (g >= wtot) return;
    int k = kb;
    while (k + 1 < n && wpre[k + 1] <= g) k++;
    const uint32_t w = (uint32_t)(g - wpre[k]);
    if (__all(k == kb)) {
        // the whole wave works for one member: its descriptor at a uniform address
        const ForceArgs &a = descs[kb];
        if (w < a.W) group_item<PHASE>(a, w);
    } else {
        const ForceArgs &a = descs[k];
        if (w < a.W) group_item<PHASE>(a, w);
    }
}

// One block per FillBlock: a chunk of one region set to its periodic
// pattern (period 1, 2 or 4 words), in 16-byte stores from a 16-byte
// aligned chunk start.
__device__ __forceinline__ void group_root_words(const GroupRoot &g);

// Blocks [0, nfill): one FillBlock each; the blocks after them: the COLTs'
// root words (which no fill region covers), 256 COLTs per block.
__global__ void __launch_bounds__(256) k_group_fill(const FillBlock *__restrict__ fb, uint32_t nfill,
                                                    const GroupRoot *__restrict__ roots, int n) {
    if (blockIdx.x >= nfill) {
        const int k = (int)(blockIdx.x - nfill) * 256 + threadIdx.x;
        if (k < n) group_root_words(roots[k]);
        return;
    }
    const FillBlock &b = fb[blockIdx.x];
    const u64 m = (u64)b.period - 1;   // 1, 2, 4 or 8 words; b.start % 8 == 0
    uint32_t *p = b.p + b.start;
    const u64 n4 = b.n >> 2;
    const uint4 v0 = make_uint4(b.pat[0], b.pat[1 & m], b.pat[2 & m], b.pat[3 & m]);
    const uint4 v1 = make_uint4(b.pat[4 & m], b.pat[5 & m], b.pat[6 & m], b.pat[7 & m]);
    for (u64 i = threadIdx.x; i < n4; i += 256) ((uint4 *)p)[i] = (i & 1) ? v1 : v0;
    for (u64 i = (n4 << 2) + threadIdx.x; i < b.n; i += 256) p[i] = b.pat[i & m];
}

// Per COLT: the root handle spans every root row; a built root with no rows
// is forced with no keys; the root's force queue holds the root handle.
__device__ __forceinline__ void group_root_words(const GroupRoot &g) {
    g.len[0] = g.nroot;
    g.st[0] = (g.built && g.nroot == 0) ? 1u : 0u;
    if (g.fq) g.fq[0] = 0;
    if (g.pre) { g.pre[0] = 0; g.pre[1] = g.nroot; }
}

// ------------------------------------------- grouped root builds by range
// A KM_K32 root map is probed within ranges of kK32Part slots (k32_next), so
// the keys of one range can all be placed by one workgroup.  A first pass
// cuts each member's items into slices, one per block, and writes each slice
// grouped by range, with the range offsets of every slice in a small matrix
// (no global atomics, no scan); then one workgroup per range gathers its
// items (one segment of each slice), builds the range in LDS and writes it
// out whole: table words, child segments and offsets, with plain stores; a
// last pass numbers the keys across ranges.  The map needs no clearing
// beforehand and no per-key device atomics, which on this GPU are performed
// past the L2 and are slow.

// The member of place block b, and of range P (host-written tables).
__device__ __forceinline__ int part_member_of_block(const PartArgs &a, uint32_t b) { return (int)a.mob[b]; }
__device__ __forceinline__ int part_member_of_part(const PartArgs &a, uint32_t P) { return (int)a.mop[P]; }

// The range of a root key: its bucket's range, or the last range for the
// key equal to the empty marker (kept in the reserved slot).
__device__ __forceinline__ uint32_t key_part(const LevelDev &L, uint32_t key, uint32_t np, uint32_t plog) {
    if (key == kEmpty32) return np - 1;
    return (uint32_t)(k32_bucket(mix32(key), L.mask) >> plog);
}

// Sum of in[lo, hi) by the whole block (every thread gets it).
__device__ __forceinline__ uint32_t block_sum_u32(const uint32_t *in, uint32_t lo, uint32_t hi, uint32_t *red) {
    uint32_t v = 0;
    for (uint32_t i = lo + threadIdx.x; i < hi; i += blockDim.x) v += in[i];
    uint32_t tot;
    block_excl_scan<uint32_t>(v, red, tot);
    return tot;
}

// A chunk of a place block's items (kPlaceChunk, four a thread): row, root
// key, child key and range; part = 0xFFFFFFFF for an item past the slice or
// failing a check.
struct PlaceItems {
    uint32_t row[kPlaceChunk / 256], key[kPlaceChunk / 256], kv[kPlaceChunk / 256], part[kPlaceChunk / 256];
};

__device__ __forceinline__ void place_gather(const ForceArgs &f, const PartMember &m, uint32_t c, uint32_t w1,
                                             const int32_t *kc, const int32_t *kvc, PlaceItems &it,
                                             StatusDev *status) {
    constexpr int R = (int)(kPlaceChunk / 256);
    bool ok[R];
    // the gathers of all the thread's items in flight together
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t w = c + r * 256 + threadIdx.x;
        ok[r] = w < w1;
        it.row[r] = ok[r] ? (f.L.offs ? f.L.offs[w] : w) : 0u;
        ok[r] = ok[r] && CK(it.row[r] < f.L.nrows);
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        it.key[r] = ok[r] ? (uint32_t)kc[it.row[r]] : 0u;
        it.kv[r] = (ok[r] && kvc) ? (uint32_t)kvc[it.row[r]] : 0u;
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t part = ok[r] ? key_part(f.L, it.key[r], m.np, m.plog) : 0xFFFFFFFFu;
        it.part[r] = (ok[r] && CK(part < m.np)) ? part : 0xFFFFFFFFu;
    }
}

// Pass 1: block b of a member takes its items [b ipb, (b + 1) ipb), counts
// them per range in LDS, writes the slice's range offsets to column b of
// the member's offset matrix (row p: the slice's items in ranges before p,
// row np: all of them) and the items themselves into the slice's own
// positions, grouped by range.  A slice of one chunk keeps its items in
// registers; a longer one reads them again for the writes.
// Blocks after the place blocks: the group's root words, 256 COLTs a block
// (when no fill launch precedes the pass).
__global__ void __launch_bounds__(256) k_part_place(PartArgs a) {
    __shared__ uint32_t hist[kMaxParts + 1];   // counts, then offsets (then write cursors)
    __shared__ uint32_t red[17];
    if (blockIdx.x >= a.nblocks) {
        const int k = (int)(blockIdx.x - a.nblocks) * 256 + threadIdx.x;
        if (k < a.nroots) group_root_words(a.roots[k]);
        return;
    }
    StatusDev *status = a.status;
    const int k = part_member_of_block(a, blockIdx.x);
    const PartMember &m = a.mem[k];
    const ForceArgs &f = a.descs[m.desc];
    const uint32_t np = m.np;
    const uint32_t b = blockIdx.x - m.block_base;
    const uint32_t w0 = b * m.ipb;                                 // < W: b < nb = ceil(W / ipb)
    const uint32_t w1 = (uint32_t)min((u64)w0 + m.ipb, (u64)m.W);
    for (uint32_t p = threadIdx.x; p < np; p += 256) hist[p] = 0;
    __syncthreads();
    const int32_t *kc = f.cols[f.L.kcol[0]];
    const int32_t *kvc = f.C.kv ? f.cols[f.C.kcol[0]] : nullptr;
    constexpr int R = (int)(kPlaceChunk / 256);
    const bool one = w1 - w0 <= kPlaceChunk;
    PlaceItems it;
    uint32_t loc[R];
    for (uint32_t c = w0; c < w1; c += kPlaceChunk) {
        place_gather(f, m, c, w1, kc, kvc, it, status);
#pragma unroll
        for (int r = 0; r < R; r++)
            if (it.part[r] < np) loc[r] = atomicAdd(&hist[it.part[r]], 1u);
    }
    __syncthreads();
    // exclusive scan of the counts, in place: each thread its own run of ranges
    {
        const uint32_t per = (np + 255) / 256;
        const uint32_t lo = min(threadIdx.x * per, np), hi = min(lo + per, np);
        uint32_t v = 0;
        for (uint32_t p = lo; p < hi; p++) v += hist[p];
        uint32_t tot;
        uint32_t ex = block_excl_scan<uint32_t>(v, red, tot);
        for (uint32_t p = lo; p < hi; p++) {
            const uint32_t c = hist[p];
            hist[p] = ex;
            ex += c;
        }
        if (threadIdx.x == 0) hist[np] = tot;
    }
    __syncthreads();
    uint32_t *O = a.poff + m.off_base;
    for (uint32_t p = threadIdx.x; p <= np; p += 256) O[(u64)p * m.nb + b] = hist[p];
    const uint32_t slice = m.item_base + w0;                       // its first position in the item arrays
    const bool has_kv = kvc != nullptr;
    if (one) {
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (it.part[r] >= np) continue;
            const uint32_t pos = slice + hist[it.part[r]] + loc[r];
            if (!CK(pos < m.item_base + w1 && pos < a.items)) continue;
            a.prow[pos] = it.row[r];
            a.pkey[pos] = it.key[r];
            if (has_kv) a.pkv[pos] = it.kv[r];
        }
        return;
    }
    __syncthreads();   // the offsets are read out; they become the write cursors
    for (uint32_t c = w0; c < w1; c += kPlaceChunk) {
        place_gather(f, m, c, w1, kc, kvc, it, status);
#pragma unroll
        for (int r = 0; r < R; r++) {
            if (it.part[r] >= np) continue;
            const uint32_t pos = slice + atomicAdd(&hist[it.part[r]], 1u);
            if (!CK(pos < m.item_base + w1 && pos < a.items)) continue;
            a.prow[pos] = it.row[r];
            a.pkey[pos] = it.key[r];
            if (has_kv) a.pkv[pos] = it.kv[r];
        }
    }
}

// Find (or, inserting, claim) key's slot in an LDS range of n slots
// (n a power of two, at least a bucket): the walk of k32_next within it.
__device__ __forceinline__ uint32_t lds_slot(uint32_t *keys, uint32_t n, uint32_t start, uint32_t key, bool insert) {
    uint32_t b = start;
    for (uint32_t i = 0; i < n; i++) {
        const uint32_t c = keys[b];
        if (c == key) return b;
        if (c == kEmpty32) {
            if (!insert) return 0xFFFFFFFFu;
            const uint32_t old = atomicCAS(&keys[b], kEmpty32, key);
            if (old == kEmpty32 || old == key) return b;
        }
        b = (b + 1) & (n - 1);
    }
    return 0xFFFFFFFFu;   // the range is full
}

// Lanes of a wave holding the same LDS slot as the wave's first remaining
// lane add their number to its counter with one atomic (up to two rounds,
// so that a heavy key under skew does not serialize a wave on one LDS
// word).  A lane so served gets todo = false and, in old, the counter's
// value before the group's addition plus its rank in the group; lanes left
// with todo make their own atomic.
__device__ __forceinline__ bool wave_slot_add(bool &todo, uint32_t s, uint32_t *ctr, uint32_t &old) {
    const int lane = __lane_id();
    for (int round = 0; round < 2; round++) {
        const u64 act = __ballot(todo);
        if (act == 0) return false;
        const int leader = __ffsll((long long)act) - 1;
        const uint32_t ls = __shfl(s, leader, 64);
        const bool same = todo && s == ls;
        const u64 grp = __ballot(same);
        const int m = __popcll(grp);
        if (m < 2) return false;
        uint32_t b = 0;
        if (lane == leader) b = atomicAdd(&ctr[ls], (uint32_t)m);
        b = __shfl(b, leader, 64);
        if (same) {
            todo = false;
            old = b + (uint32_t)__popcll(grp & ((1ull << lane) - 1ull));
            return true;
        }
    }
    return false;
}

// The item arrays' position of item j of a range whose items are segments
// of the place slices: segment t holds the range's items [sst[t], sst[t+1])
// from position ssrc[t] on (the last t with sst[t] <= j; empty segments
// share their start with the next one).
__device__ __forceinline__ uint32_t range_item_pos(const uint32_t *sst, const uint32_t *ssrc, uint32_t nb,
                                                   uint32_t j) {
    uint32_t lo = 0, hi = nb;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (sst[mid] <= j) lo = mid; else hi = mid;
    }
    return ssrc[lo] + (j - sst[lo]);
}

// Pass 2: one workgroup per range builds it in LDS: keys and their offset
// counts, child segments laid out in the range's own item positions (the
// empty marker's first), then the range's table words, child lengths,
// offsets (and the keys beside them) and per-slot counts are written.  The
// range's items are one segment of each place slice, found from row lp and
// lp + 1 of the member's offset matrix; the sum of row lp is the member's
// items in the ranges before this one, where its child segments start.
constexpr int kPartBuildThreads = 1024;
__global__ void __launch_bounds__(kPartBuildThreads) k_part_build(PartArgs a) {
    __shared__ uint32_t keys[kK32Part];
    __shared__ uint32_t cnt[kK32Part];
    __shared__ uint32_t fw[kK32Part / kK32Bucket];   // the range's filter words
    __shared__ uint32_t red[17];
    __shared__ uint32_t emp;
    __shared__ uint32_t sst[kMaxPlaceBlocks + 1];   // the range's items: segment starts
    __shared__ uint32_t ssrc[kMaxPlaceBlocks];      // and their first positions in the item arrays
    static_assert(kMaxPlaceBlocks <= kPartBuildThreads, "a thread per place block");
    StatusDev *status = a.status;
    const uint32_t P = blockIdx.x;
    const int k = part_member_of_part(a, P);
    const PartMember &m = a.mem[k];
    const ForceArgs &f = a.descs[m.desc];
    const uint32_t lp = P - m.part_base;
    const uint32_t n = 1u << m.plog;                  // slots of the range
    const u64 s0 = (u64)lp << m.plog;                 // its first slot in the map
    const uint32_t nb = m.nb;
    uint32_t seg = 0, before = 0;
    if (threadIdx.x < nb) {
        const uint32_t *O = a.poff + m.off_base;
        const uint32_t t = threadIdx.x;
        before = O[(u64)lp * nb + t];
        const uint32_t e = O[(u64)(lp + 1) * nb + t];
        seg = CK(e >= before) ? e - before : 0u;
        ssrc[t] = m.item_base + t * m.ipb + before;
    }
    for (uint32_t s = threadIdx.x; s < n; s += kPartBuildThreads) { keys[s] = kEmpty32; cnt[s] = 0; }
    // the filter's words of this range (the host keeps at least one per range)
    const uint32_t fsh = 2 + f.L.bloom_shift;
    const uint32_t nfw = f.L.bloom ? n >> fsh : 0u;
    const uint32_t fw0 = (uint32_t)(s0 >> fsh);
    for (uint32_t w = threadIdx.x; w < nfw; w += kPartBuildThreads) fw[w] = 0;
    if (threadIdx.x == 0) emp = 0;
    uint32_t ni;
    const uint32_t sx = block_excl_scan<uint32_t>(seg, red, ni);
    if (threadIdx.x < nb) sst[threadIdx.x] = sx;
    if (threadIdx.x == 0) sst[nb] = ni;
    uint32_t base;                                    // the range's first position in the member
    block_excl_scan<uint32_t>(before, red, base);
    __syncthreads();
    if (m.clear_cst)                                  // level 1's tries start unforced
        for (uint32_t j = threadIdx.x; j < ni; j += kPartBuildThreads)
            if (CK((u64)base + j < f.C.npos)) f.C.st[base + j] = 0u;
    const bool has_kv = f.C.kv != nullptr;
    // (the loops run whole waves, so that lanes can pool their atomics)
    const uint32_t niw = ((ni + kPartBuildThreads - 1) / kPartBuildThreads) * kPartBuildThreads;
    for (uint32_t j = threadIdx.x; j < niw; j += kPartBuildThreads) {
        const uint32_t i = j < ni ? range_item_pos(sst, ssrc, nb, j) : 0u;
        const bool live = j < ni && CK(i < a.items);
        const uint32_t key = live ? a.pkey[i] : kEmpty32;
        if (live && key == kEmpty32) atomicAdd(&emp, 1u);
        uint32_t s = 0xFFFFFFFFu;
        if (live && key != kEmpty32) {
            s = lds_slot(keys, n, (uint32_t)(k32_bucket(mix32(key), f.L.mask) - s0), key, true);
            CK(s < n);
        }
        bool todo = s < n;
        uint32_t old;
        wave_slot_add(todo, s, cnt, old);
        if (todo) atomicAdd(&cnt[s], 1u);
    }
    __syncthreads();
    // child starts in slot order, the empty marker's child first
    constexpr int SPT = (int)(kK32Part / kPartBuildThreads);   // slots per thread
    uint32_t sum = 0, nk = 0;
#pragma unroll
    for (int j = 0; j < SPT; j++) {
        const uint32_t s = threadIdx.x * SPT + j;
        if (s < n) { sum += cnt[s]; nk += keys[s] != kEmpty32; }
    }
    uint32_t tot;
    uint32_t pre = block_excl_scan<uint32_t>(sum, red, tot) + emp;
    uint32_t ktot;
    block_excl_scan<uint32_t>(nk, red, ktot);
    uint32_t *T = (uint32_t *)f.L.table;
    uint32_t *sc = a.scnt + m.slot_base + s0;
#pragma unroll
    for (int j = 0; j < SPT; j++) {
        const uint32_t s = threadIdx.x * SPT + j;
        if (s >= n) continue;
        const uint32_t c = cnt[s];
        const u64 w = k32_key_word(s0 + s);
        T[w] = keys[s];
        T[w + 4] = c ? base + pre : 0u;
        if (nfw && keys[s] != kEmpty32) {
            const uint32_t h = mix32(keys[s]);
            const uint32_t fi = bloom_word(h, f.L.mask, f.L.bloom_shift) - fw0;
            if (CK(fi < nfw)) atomicOr(&fw[fi], bloom_bits(h));
        }
        sc[s] = c;
        if (c && CK((u64)base + pre < f.C.npos)) f.C.len[base + pre] = c;
        cnt[s] = base + pre;                          // from here on: the slot's scatter cursor
        pre += c;
    }
    const bool last = lp + 1 == m.np;
    if (threadIdx.x == 0) {
        if (last) {
            // the reserved slot: claimed when the empty marker is a key
            const u64 w = k32_key_word(f.L.mask + 1);
            T[w] = emp ? 1u : 0u;
            T[w + 4] = emp ? base : 0u;
            if (emp && CK(base < f.C.npos)) f.C.len[base] = emp;
        }
        a.pdist[P] = ktot + (emp ? 1u : 0u);
        if (!m.keys && lp == 0) f.L.st[0] = 1u;       // a root only probed: forced, its keys not listed
        emp = base;                                   // the empty marker's scatter cursor
    }
    __syncthreads();
    for (uint32_t w = threadIdx.x; w < nfw; w += kPartBuildThreads) f.L.bloom[fw0 + w] = fw[w];
    for (uint32_t j = threadIdx.x; j < niw; j += kPartBuildThreads) {
        const uint32_t i = j < ni ? range_item_pos(sst, ssrc, nb, j) : 0u;
        const bool live = j < ni && i < a.items;       // (a failed check was reported above)
        const uint32_t key = live ? a.pkey[i] : kEmpty32;
        uint32_t pos = 0xFFFFFFFFu;
        if (live && key == kEmpty32) pos = atomicAdd(&emp, 1u);
        uint32_t s = 0xFFFFFFFFu;
        if (live && key != kEmpty32) {
            s = lds_slot(keys, n, (uint32_t)(k32_bucket(mix32(key), f.L.mask) - s0), key, false);
            CK(s < n);
        }
        bool todo = s < n;
        wave_slot_add(todo, s, cnt, pos);
        if (todo) pos = atomicAdd(&cnt[s], 1u);
        if (!live || pos == 0xFFFFFFFFu) continue;
        if (!CK(pos < f.C.npos && pos >= base)) continue;
        f.C.offs[pos] = a.prow[i];
        if (has_kv) f.C.kv[pos] = (int32_t)a.pkv[i];
    }
}

// Pass 3 (after the scan of the distinct counts; roots whose keys are
// listed): the keys of each range take their ranks in slot order (the empty
// marker's first) and are listed in the root's key list; a member's first
// range records its key count.
__global__ void __launch_bounds__(256) k_part_ranks(PartArgs a) {
    __shared__ uint32_t red[17];
    StatusDev *status = a.status;
    const uint32_t P = blockIdx.x;
    const int k = part_member_of_part(a, P);
    const PartMember &m = a.mem[k];
    if (!m.keys) return;   // a root only probed (the build marked it forced)
    const ForceArgs &f = a.descs[m.desc];
    const uint32_t lp = P - m.part_base;
    const uint32_t n = 1u << m.plog;
    const u64 s0 = (u64)lp << m.plog;
    const uint32_t *T = (const uint32_t *)f.L.table;
    const uint32_t *sc = a.scnt + m.slot_base + s0;
    const bool last = lp + 1 == m.np;
    const u64 wr = k32_key_word(f.L.mask + 1);
    const uint32_t has_emp = (last && T[wr]) ? 1u : 0u;
    uint32_t r;
    if (a.inline_scan) {
        // the distinct keys of the member's earlier ranges (and, for its
        // first range, of all of them), summed here
        r = block_sum_u32(a.pdist, m.part_base, P, red);
        if (lp == 0) {
            const uint32_t nk = block_sum_u32(a.pdist, m.part_base, m.part_base + m.np, red);
            if (threadIdx.x == 0) { f.L.st[0] = nk + 1; f.L.rank_ctr[0] = nk; }
        }
    } else {
        r = a.rstart[P] - a.rstart[m.part_base];
        if (threadIdx.x == 0 && lp == 0) {
            const uint32_t nk = a.rstart[m.part_base + m.np] - a.rstart[m.part_base];
            f.L.st[0] = nk + 1;
            f.L.rank_ctr[0] = nk;
        }
    }
    if (has_emp && threadIdx.x == 0 && CK(r < f.L.npos)) {
        const uint32_t c = T[wr + 4];
        f.L.kl[r] = c;
        if (f.L.kk) { f.L.kk[r] = (int32_t)kEmpty32; f.L.kn[r] = f.C.len[c]; }
    }
    r += has_emp;
    constexpr int SPT = (int)(kK32Part / 256);
    uint32_t key[SPT], val[SPT];
    uint32_t nk = 0;
#pragma unroll
    for (int j = 0; j < SPT; j++) {
        const uint32_t s = threadIdx.x * SPT + j;
        const u64 w = k32_key_word(s0 + (s < n ? s : 0));
        key[j] = s < n ? T[w] : kEmpty32;
        val[j] = s < n ? T[w + 4] : 0u;
        nk += key[j] != kEmpty32;
    }
    uint32_t ktot;
    r += block_excl_scan<uint32_t>(nk, red, ktot);
#pragma unroll
    for (int j = 0; j < SPT; j++) {
        const uint32_t s = threadIdx.x * SPT + j;
        if (key[j] == kEmpty32) continue;
        if (CK(r < f.L.npos)) {
            f.L.kl[r] = val[j];
            if (f.L.kk) { f.L.kk[r] = (int32_t)key[j]; f.L.kn[r] = sc[s]; }
        }
        r++;
    }
}

// ----------------------------------------------------------- cover choice
// Per input binding: among the node's pure covers pick the one whose current
// trie has the fewest keys (a forced map's key count, an unforced vector's
// length), first on ties (Section 4.4).  A last-level unforced vector is
// iterated by offset; anything else is iterated by key, forcing it first.

__device__ __forceinline__ uint32_t handle_of(const SubDev &S, const FrontierDev &F, const NodeDev &nd,
                                              uint32_t e) {
    if (S.level == 0) return 0u;
    for (int j = 0; j < nd.nin_h; j++)
        if (nd.in_h_atom[j] == S.atom) return F.hdl[(u64)j * F.cap + e];
    return 0xFFFFFFFFu;
}

__device__ __forceinline__ uint32_t trie_len(const SubDev &S, uint32_t p) {
    return S.level == 0 ? S.root_len : S.L.len[p];
}

__global__ void __launch_bounds__(256) k_cover_choose(const NodeDev *__restrict__ ndp, uint32_t E, uint8_t *cov,
                                                      u64 *cnt, StatusDev *status) {
    const NodeDev &nd = *ndp;
    uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    cov[e] = 0;
    cnt[e] = 0;
    if (!CK(e < nd.in.cap)) return;
    int best = -1;
    uint32_t best_est = 0, best_p = 0, best_st = 0;
    for (int q = 0; q < nd.npure; q++) {
        const SubDev &S = nd.sub[nd.pure[q]];
        uint32_t p = handle_of(S, nd.in, nd, e);
        if (!CK(p < S.L.npos)) return;
        uint32_t st = S.L.st[p];
        uint32_t est = (st != 0 && st != kQueued) ? st - 1 : trie_len(S, p);
        if (best < 0 || est < best_est) { best = q; best_est = est; best_p = p; best_st = st; }
    }
    const SubDev &S = nd.sub[nd.pure[best]];
    bool forced = best_st != 0 && best_st != kQueued;
    uint8_t keys_mode = 0;
    u64 n;
    if (forced) { keys_mode = 1; n = best_st - 1; }
    else if (S.last) { keys_mode = 0; n = trie_len(S, best_p); }
    else {
        // iter() on a vector that is not the last level: force it first
        keys_mode = 1; n = 0;
        if (!CK(S.level > 0)) return;
        if (atomicCAS(&S.L.st[best_p], 0u, kQueued) == 0u) {
            uint32_t pos = atomicAdd(&status->fq_n[S.fq_slot], 1u);
            if (CK(pos < S.L.npos)) S.L.fq[pos] = best_p;
        }
        atomicAdd(&status->pending, 1u);
    }
    cov[e] = (uint8_t)(nd.pure[best] | (keys_mode << 7));
    cnt[e] = n;
    // The first lookup after the cover, in node order, is reached by the
    // binding's first cover tuple whenever the cover is not empty, so its
    // get() is certain: its trie joins the force queue now, with the
    // covers', instead of deferring every tuple that meets it unforced.
    // The forced tries are the ones a tuple-at-a-time run forces.
    if (forced ? n == 0 : trie_len(S, best_p) == 0) return;
    for (int j = 0; j < nd.nsub; j++) {
        if (j == nd.pure[best]) continue;
        const SubDev &P = nd.sub[j];
        if (P.level == 0 && !P.L.fq) break;   // a root built up front
        const uint32_t ph = handle_of(P, nd.in, nd, e);
        if (!CK(ph < P.L.npos)) return;
        if (P.L.st[ph] == 0u && atomicCAS(&P.L.st[ph], 0u, kQueued) == 0u) {
            const uint32_t pos = atomicAdd(&status->fq_n[P.fq_slot], 1u);
            if (CK(pos < P.L.npos)) P.L.fq[pos] = ph;
            atomicAdd(&status->pending, 1u);
        }
        break;
    }
}

__global__ void __launch_bounds__(256) k_cover_fill(const NodeDev *__restrict__ ndp, uint32_t E, const uint8_t *cov,
                                                    u64 *cnt, StatusDev *status) {
    const NodeDev &nd = *ndp;
    uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    uint8_t c = cov[e];
    if (!(c & 0x80)) return;
    const SubDev &S = nd.sub[c & 0x7F];
    uint32_t p = handle_of(S, nd.in, nd, e);
    if (!CK(p < S.L.npos)) { cnt[e] = 0; return; }
    uint32_t st = S.L.st[p];
    if (!CK(st != 0 && st != kQueued)) { cnt[e] = 0; return; }
    cnt[e] = st - 1;
}

// ------------------------------------------------------------------ probe
// One thread per cover tuple of the tile.  The tuple's binding is located by
// binary search over the scanned cover counts, its cover tuple is bound, and
// the node's other subatoms are probed in node order with early exit.  A
// probe that meets an unforced trie queues that trie for forcing (once, by
// state CAS) and defers the tuple; the host forces the queue and re-runs the
// deferred tuples from that lookup on.

struct ProbeArgs {
    const NodeDev *nd;
    const u64 *starts;        // E + 1 scanned cover counts
    const uint8_t *cov;
    uint32_t E;
    u64 t0;                   // first tuple of the tile
    uint32_t n;               // threads' work items
    const uint32_t *din;      // deferred mode: tuple (tile-local) and resume lookup
    const uint8_t *din_j;
    uint32_t *dout;           // deferrals of this launch
    uint8_t *dout_j;
    uint32_t dcap;            // capacity of the deferral lists
    u64 surv_base;            // survivor and deferral counters before this launch
    u64 def_base;
    StatusDev *status;
    int count_stats;
    const uint32_t *chunk_e;  // per block: the binding of its first tuple (+1 sentinel), or null
};

// The binding of the first tuple of every block-sized chunk of a tile (and
// of the tile's last tuple, as a sentinel), so that a probe thread searches
// only between its block's two bounds instead of over every binding.
__global__ void k_chunk_entries(const u64 *__restrict__ starts, uint32_t E, u64 t0, uint32_t n, uint32_t bs,
                                uint32_t nchunks, uint32_t *out) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c > nchunks) return;
    const u64 off = std::min<u64>((u64)c * bs, (u64)n - 1);
    out[c] = E == 1 ? 0u : upper_entry(starts, 0, E, t0 + off);
}

// MV and MA bound the binding's variable slots and atoms (powers of two; the
// host picks the smallest that fits the query, and every index is masked so
// that no plan can index past them).
// Largest e in [lo, hi) with starts[e] <= g, searching a copy of
// starts[lo, hi] held in LDS (sst[k] = starts[lo + k]).
__device__ __forceinline__ uint32_t upper_entry_lds(const u64 *sst, uint32_t lo, uint32_t hi, u64 g) {
    uint32_t a = 0, b = hi - lo;
    while (b - a > 1) {
        const uint32_t mid = a + ((b - a) >> 1);
        if (sst[mid] <= g) a = mid; else b = mid;
    }
    return lo + a;
}

constexpr uint32_t kProbeStartsLds = 1024;   // scanned cover counts a block caches for its search

#ifndef FJ_PROBE_WAVES
#define FJ_PROBE_WAVES 1
#endif
template <int MV, int MA>
__global__ void __launch_bounds__(256, FJ_PROBE_WAVES) k_probe(ProbeArgs a) {
    __shared__ u64 red[17];
    __shared__ u64 sst[kProbeStartsLds];
    // The node's subatom descriptors, copied to LDS once per workgroup: a
    // tuple's cover is its binding's choice, so threads index them by a
    // per-lane number, and from LDS those reads cost no memory round trips.
    __shared__ SubDev ssub[FJ_MAX_ATOMS];
    const NodeDev &nd = *a.nd;
    {
        const uint32_t words = (uint32_t)(min(nd.nsub, FJ_MAX_ATOMS) * sizeof(SubDev) / sizeof(uint32_t));
        const uint32_t *src = (const uint32_t *)nd.sub;
        uint32_t *dst = (uint32_t *)ssub;
        for (uint32_t k = threadIdx.x; k < words; k += blockDim.x) dst[k] = src[k];
    }
    StatusDev *status = a.status;
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    bool survive = false, defer = false;
    uint32_t t = 0;
    int resume = 0, defer_j = 0;
    u64 mult = 1, emitv = 0;
    uint32_t nprobe = 0, nhit = 0;
    int32_t v[MV];
    uint32_t h[MA];
    uint32_t e = 0;
    // a block of a tile's tuples needs only the bindings between its first
    // and last tuple's: their scanned counts go to LDS in one coalesced
    // read, so each thread's search costs no dependent HBM reads
    uint32_t lo = 0, hi = a.E;
    bool in_lds = false, range_ok = true;
    if (!a.din && a.chunk_e) {
        lo = a.chunk_e[blockIdx.x];
        hi = a.chunk_e[blockIdx.x + 1] + 1;
        range_ok = CK(lo < hi && hi <= a.E);
        in_lds = range_ok && hi - lo + 1 <= kProbeStartsLds;   // block-uniform
        if (in_lds)
            for (uint32_t k = threadIdx.x; k <= hi - lo; k += blockDim.x) sst[k] = a.starts[lo + k];
    }
    __syncthreads();
    bool ok = idx < a.n && range_ok;
    if (ok) {
        if (a.din) { t = a.din[idx]; resume = a.din_j[idx]; } else { t = idx; }
        const u64 g = a.t0 + t;
        if (a.E == 1) e = 0;
        else if (in_lds) e = upper_entry_lds(sst, lo, hi, g);
        else e = upper_entry(a.starts, lo, hi, g);
        if (in_lds) ok = CK(e < a.E && e < nd.in.cap && g >= sst[e - lo] && g < sst[e - lo + 1]);
        else ok = CK(e < a.E && e < nd.in.cap && g >= a.starts[e] && g < a.starts[e + 1]);
    }
    if (ok) {
        const u64 i = a.t0 + t - (in_lds ? sst[e - lo] : a.starts[e]);
        const FrontierDev &F = nd.in;
        for (int j = 0; j < nd.nin; j++) v[(j) & (MV - 1)] = F.vals[(u64)j * F.cap + e];
        for (int j = 0; j < nd.nin_h; j++) h[(nd.in_h_atom[j]) & (MA - 1)] = F.hdl[(u64)j * F.cap + e];
        mult = F.mult ? F.mult[e] : 1ull;
        // bind the cover tuple
        const uint8_t cb = a.cov[e];
        const int ci = cb & 0x7F;
        const SubDev &S = ssub[ci & (FJ_MAX_ATOMS - 1)];
        const uint32_t p = S.level == 0 ? 0u : h[(S.atom) & (MA - 1)];
        if (cb & 0x80) {
            ok = CK(p + i < S.L.npos);
            const uint32_t s = ok ? S.L.kl[p + (uint32_t)i] : 0u;
            ok = ok && CK(s < S.C.npos);
            if (ok && S.L.kk && S.nk == 1) {
                // the key list holds the key and its offset count
                v[(S.kslot[0]) & (MV - 1)] = S.L.kk[p + (uint32_t)i];
                if (S.child_leaf) mult *= S.L.kn[p + (uint32_t)i];
                else h[(S.atom) & (MA - 1)] = s;
            } else {
                const uint32_t row = ok ? S.C.offs[s] : 0u;
                ok = ok && CK(row < S.L.nrows);
                if (ok) {
                    for (int c = 0; c < S.nk; c++) v[(S.kslot[c]) & (MV - 1)] = S.cols[S.kcol[c]][row];
                    if (S.child_leaf) mult *= S.C.len[s];
                    else h[(S.atom) & (MA - 1)] = s;
                }
            }
        } else {
            const u64 pos = p + i;
            ok = CK(p < S.L.npos) && CK(pos < S.L.npos && i < trie_len(S, p));
            if (ok && S.L.kv && S.nk == 1) {
                v[(S.kslot[0]) & (MV - 1)] = S.L.kv[pos];   // the key beside the offset
            } else {
                const uint32_t row = ok ? (S.L.offs ? S.L.offs[pos] : (uint32_t)pos) : 0u;
                ok = ok && CK(row < S.L.nrows);
                if (ok)
                    for (int c = 0; c < S.nk; c++) v[(S.kslot[c]) & (MV - 1)] = S.cols[S.kcol[c]][row];
            }
        }
        // lookups in node order
        survive = ok;
        for (int j = 0; j < nd.nsub && survive; j++) {
            if (j == ci) continue;
            const SubDev &P = ssub[j & (FJ_MAX_ATOMS - 1)];
            const uint32_t ph = P.level == 0 ? 0u : h[(P.atom) & (MA - 1)];
            if (!CK(ph < P.L.npos)) { survive = false; break; }
            const uint32_t st = P.L.st[ph];
            if (st == 0 || st == kQueued) {
                // an inner trie, or a root left as its base table by the
                // build phase (a single-level pure cover of this node)
                if (!CK(P.level > 0 || P.L.fq != nullptr)) { survive = false; break; }
                if (st == 0 && atomicCAS(&P.L.st[ph], 0u, kQueued) == 0u) {
                    uint32_t pos = atomicAdd(&status->fq_n[P.fq_slot], 1u);
                    if (CK(pos < P.L.npos)) P.L.fq[pos] = ph;
                }
                defer = true; defer_j = j; survive = false;
                break;
            }
            uint32_t s, clen = 0;
            bool have_len = false;
            if (j >= resume) nprobe++;
            if (P.L.mode == KM_ZERO) {
                // a map with no variables has one key, or none when empty
                if (st - 1 == 0) { survive = false; break; }
                s = P.L.kl[ph];
            } else {
                Key k;
                k.h = ph;
                k.span = P.L.local ? P.L.len[ph] : 0u;
                for (int c = 0; c < P.nk; c++) k.v[c] = v[(P.kslot[c]) & (MV - 1)];
                const u64 slot = table_find(P.L, P.cols, k);
                if (slot == ~0ull) { survive = false; break; }
                if (!CK(slot < P.L.nslots)) { survive = false; break; }
                s = slot_val(P.L, slot);
                if (P.L.mode == KM_K64) {
                    clen = ((const Slot64 *)P.L.table)[slot].pad;   // the line just read
                    have_len = true;
                }
            }
            if (!CK(s < P.C.npos)) { survive = false; break; }
            if (j >= resume) nhit++;
            if (P.child_leaf) mult *= have_len ? clen : P.C.len[s];
            else h[(P.atom) & (MA - 1)] = s;
        }
        if (survive && nd.emit) {
            emitv = mult;
            for (int q = 0; q < nd.ntail; q++) {
                const TailDev &T = nd.tail[q];
                if (T.level == 0) { emitv *= (u64)T.root_len; continue; }
                const uint32_t th = h[(T.atom) & (MA - 1)];
                if (!CK(th < T.L.npos)) { survive = false; emitv = 0; break; }
                emitv *= (u64)T.L.len[th];
            }
        }
    }
    if (a.count_stats) {
        u64 np = wave_sum_u64(nprobe), nh = wave_sum_u64(nhit);
        if (__lane_id() == 0 && (np | nh)) {
            atomicAdd(&a.status->probe[nd.k], np);
            atomicAdd(&a.status->hit[nd.k], nh);
        }
    }
    if (nd.emit) block_add_count(emitv, status, red);
    // deferred tuples
    // the counters only grow; this launch's entries start at its base
    if (__syncthreads_or(defer)) {
        u64 pos = block_reserve(defer, &a.status->deferred, red) - a.def_base;
        if (defer && CK(pos < a.dcap)) { a.dout[pos] = t; a.dout_j[pos] = (uint8_t)defer_j; }
    }
    // survivors to the output frontier
    const bool write = survive && (!nd.emit || nd.materialize);
    if (!__syncthreads_or(write)) return;
    u64 pos = block_reserve(write, &a.status->survivors, red) - a.surv_base;
    if (write && CK(pos < nd.out.cap)) {
        const FrontierDev &O = nd.out;
        for (int j = 0; j < nd.nout; j++) O.vals[(u64)j * O.cap + pos] = v[(nd.out_slot[j]) & (MV - 1)];
        for (int j = 0; j < nd.nout_h; j++) O.hdl[(u64)j * O.cap + pos] = h[(nd.out_h_atom[j]) & (MA - 1)];
        if (O.mult) O.mult[pos] = mult;
    }
}

// ------------------------------------------------------------------- emit
// Materialization: every final binding stands for mult * prod(tail lengths)
// result tuples, whose values come from the binding and from each tail
// trie's rows (mixed radix over the tails, the last one fastest).

struct EmitDev {
    FrontierDev F;
    int nin;
    int in_var[FJ_MAX_VARS];
    int nin_h;
    int in_h_atom[FJ_MAX_ATOMS];
    int ntail;
    TailDev tail[FJ_MAX_NODES];
    int nhead;
    int head_src[FJ_MAX_VARS];    // >= 0: frontier value column; < 0: -(tail * FJ_MAX_COLS + c) - 1
    int32_t *out;
    u64 out_rows;                 // capacity of out in rows
};

// ------------------------------------------------------------ scan probe
// Specialised first node: the cover is a base table (or its selection)
// iterated directly and every other subatom is a probe of a root map keyed
// by cover columns.  The node's lookups run as rounds over a batch of cover
// rows (Section 4.3's batch, one lookup at a time over the whole batch).
// Round 0 probes every row of a tile of kTile positions, kTileRows per
// thread with their loads in flight together; the rows that hit join an LDS
// batch.  Once the batch could not take another tile, round j probes only
// the entries left by round j - 1, reading lookup j's key columns for those
// rows alone: every round's lanes are dense, the later rounds shrink with
// the selectivity, and key columns past the first are read only where a row
// is still alive.  A hit is kept per (lookup, batch entry) in LDS: its slot
// for a KM_K32 map, whose value is read only for the rows that pass every
// lookup, or its value for a KM_K64 map.

#ifndef FJ_TILE_ROWS
#define FJ_TILE_ROWS 2
#endif
constexpr int kTileRows = FJ_TILE_ROWS;
constexpr int kTile = 256 * kTileRows;
constexpr int kBatch = 2 * kTile;   // batch entries: room for another whole tile at every check
#ifndef FJ_ROUND_ROWS
#define FJ_ROUND_ROWS 2
#endif
constexpr int kRoundRows = FJ_ROUND_ROWS;   // batch entries per thread in flight in the later rounds
#ifndef FJ_SCAN_WAVES
#define FJ_SCAN_WAVES 1
#endif
static_assert(kBatch <= 65536, "batch entries are 16-bit");
constexpr int kScanMaxLookups = 8;

// The filter pass of a two-launch first node (k_scan_filter, below): tiles
// of kFiltRows rows per thread of one kFiltThreads workgroup per CU, dealt
// round robin; each wave writes its first-lookup hits to its own region of
// the list, which holds the rows the wave sees (kFiltRows x 64 per tile).
constexpr int kFiltThreads = 1024;
constexpr int kFiltRows = 8;
constexpr int kFiltTile = kFiltThreads * kFiltRows;
constexpr int kFiltWaves = kFiltThreads / 64;
constexpr int kFiltWaveTile = kFiltRows * 64;
static_assert(kFiltWaves == kScanListWaves, "list counters per filter-pass workgroup");
// Region of wave w of workgroup g (its first entry and capacity).
__host__ __device__ inline unsigned long long list_region(uint32_t g, uint32_t w, uint32_t ntiles, uint32_t G,
                                                          uint32_t &cap) {
    const unsigned long long full = ntiles / G, rem = ntiles % G;
    const unsigned long long tiles = full + (g < rem ? 1u : 0u);
    cap = (uint32_t)(tiles * kFiltWaveTile);
    return ((unsigned long long)g * full + (g < rem ? g : rem)) * (unsigned long long)kFiltTile +
           (unsigned long long)w * tiles * kFiltWaveTile;
}

struct ScanArgs {
    const int32_t *cols[FJ_MAX_COLS];
    int ncols;
    int vec;                  // no selection, rows in bounds, 16-byte aligned columns, r0 % 4 == 0
    const uint32_t *sel;      // selection of the cover relation, or null
    uint32_t nrows;           // rows of the cover relation's columns
    uint32_t r0;              // first cover position of this launch
    uint32_t n;               // cover positions in this launch
    int nl;
    ScanLookup lk[kScanMaxLookups];
    int nout;
    int out_col[FJ_MAX_VARS]; // output value column j <- cover column
    FrontierDev out;
    int emit, materialize;
    int ntail;
    int tail_lk[FJ_MAX_NODES];          // lookup whose child is the tail's trie, -1: a root
    const uint32_t *tail_len[FJ_MAX_NODES];
    uint32_t tail_npos[FJ_MAX_NODES];
    uint32_t tail_root_len[FJ_MAX_NODES];
    StatusDev *status;
    int count_stats;
    int node;
    u64 surv_base;            // survivor counter before this launch
    // direct emit (the first node is the last probing node and rows are
    // wanted): the flush writes result rows itself, placed by one atomic
    // reservation per wave on status->written (which may pass cap: the host
    // clamps it); no frontier, no emit launch
    int direct;
    const EmitDev *ed;        // head mapping, tails and output of the execution
    u64 cap;                  // output capacity in rows
    // two-launch first node: the filter pass writes the rows that pass the
    // first lookup's filter, and their keys, of wave w of workgroup g to its
    // region of l0_row / l0_key and their number to l0_cnt[g * kFiltWaves +
    // w]; k_scan_rounds probes them (l0_per consecutive regions a workgroup)
    uint32_t *l0_row, *l0_key, *l0_cnt;
    uint32_t l0_groups, l0_per;
};

// One row's probe of a root map in two steps, so that several rows' loads
// are in flight together: issue() hashes the key and loads its first bucket
// (KM_K32: the bucket's four keys, one 16-byte load; KM_K64: its two
// slots), resolve() scans it and walks on past full buckets.
struct RowProbe {
    uint4 q0, q1;
    u64 idx;     // first slot of the loaded bucket
    u64 key;     // KM_K32: the 32-bit key; KM_K64: the packed pair
    bool empty;  // the key equals the empty marker (reserved slot)
};

template <int MODE>
__device__ __forceinline__ void probe_issue(const ScanLookup &L, uint32_t k0, uint32_t k1, bool alive,
                                            RowProbe &rp) {
    rp.q1 = make_uint4(0, 0, 0, 0);
    // the load is not branched around: rows that need no bucket read
    // bucket 0, so the compiler keeps every row's load in flight
    if constexpr (MODE == KM_K32) {
        rp.key = k0;
        rp.empty = k0 == kEmpty32;
        rp.idx = k32_bucket(mix32(k0), L.mask);
        const u64 b = (alive && !rp.empty) ? rp.idx : 0;
        rp.q0 = *(const uint4 *)((const uint32_t *)L.table + k32_key_word(b));
    } else {
        rp.key = ((u64)k0 << 32) | k1;
        rp.empty = rp.key == kEmpty64;
        rp.idx = bucket_start<Slot64>(mix64(rp.key), L.mask);
        const uint4 *b = (const uint4 *)((const Slot64 *)L.table + ((alive && !rp.empty) ? rp.idx : 0));
        rp.q0 = b[0];
        rp.q1 = b[1];
    }
}

// Four KM_K32 keys in slot order: 1 = hit (its slot in s), 2 = miss (an
// empty slot comes first), 0 = full of other keys.  Branch-free: walking
// backwards, the earliest deciding slot wins.
__device__ __forceinline__ int scan_keys32(const uint4 &q, uint32_t key, int &s) {
    int st = 0, at = 0;
    st = q.w == key ? 1 : (q.w == kEmpty32 ? 2 : st);
    at = q.w == key ? 3 : at;
    st = q.z == key ? 1 : (q.z == kEmpty32 ? 2 : st);
    at = q.z == key ? 2 : at;
    st = q.y == key ? 1 : (q.y == kEmpty32 ? 2 : st);
    at = q.y == key ? 1 : at;
    st = q.x == key ? 1 : (q.x == kEmpty32 ? 2 : st);
    at = q.x == key ? 0 : at;
    s = at;
    return st;
}

// Two KM_K64 slots {key lo, key hi, val, pad}: as above, the value in val.
__device__ __forceinline__ int scan_slots64(const uint4 &a, const uint4 &b, u64 key, uint32_t &val) {
    int st = 0;
    uint32_t v = 0;
    const u64 kb = ((u64)b.y << 32) | b.x, ka = ((u64)a.y << 32) | a.x;
    st = kb == key ? 1 : (kb == kEmpty64 ? 2 : st);
    v = kb == key ? b.z : v;
    st = ka == key ? 1 : (ka == kEmpty64 ? 2 : st);
    v = ka == key ? a.z : v;
    val = v;
    return st;
}

// true on a hit; out = the slot (KM_K32) or the value (KM_K64)
template <int MODE>
__device__ __forceinline__ bool probe_resolve(const ScanLookup &L, RowProbe &rp, uint32_t &out) {
    if constexpr (MODE == KM_K32) {
        const uint32_t *T = (const uint32_t *)L.table;
        out = (uint32_t)(L.mask + 1);
        if (rp.empty) return T[k32_key_word(L.mask + 1)] != 0u;
        int s = 0;
        int st = scan_keys32(rp.q0, (uint32_t)rp.key, s);
        for (u64 n = kK32Bucket; st == 0 && n <= k32_part_mask(L.mask); n += kK32Bucket) {   // a full bucket (rare)
            rp.idx = k32_next(rp.idx, L.mask);
            rp.q0 = *(const uint4 *)(T + k32_key_word(rp.idx));
            st = scan_keys32(rp.q0, (uint32_t)rp.key, s);
        }
        out = (uint32_t)(rp.idx + s);
        return st == 1;
    } else {
        const Slot64 *T = (const Slot64 *)L.table;
        if (rp.empty) {
            const Slot64 rs = T[L.mask + 1];
            out = rs.val;
            return rs.key != 0;
        }
        int st = scan_slots64(rp.q0, rp.q1, rp.key, out);
        for (u64 n = 2; st == 0 && n <= L.mask; n += 2) {
            rp.idx = (rp.idx + 2) & L.mask;
            const uint4 *b = (const uint4 *)(T + rp.idx);
            rp.q0 = b[0];
            rp.q1 = b[1];
            st = scan_slots64(rp.q0, rp.q1, rp.key, out);
        }
        return st == 1;
    }
}

__device__ __forceinline__ uint32_t tile_row(const ScanArgs &a, uint32_t tile0, uint32_t p) {
    const uint32_t pos = a.r0 + tile0 + p;
    return a.sel ? a.sel[pos] : pos;
}

// A slot in an LDS list for each lane with pred, one LDS atomic per wave.
__device__ __forceinline__ uint32_t list_slot(bool pred, uint32_t *cnt) {
    const u64 mask = __ballot(pred);
    if (!mask) return 0;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt, (uint32_t)__popcll(mask));
    base = __shfl(base, leader, 64);
    return base + __popcll(mask & ((1ull << lane) - 1ull));
}

// Rows of a tile taken with positions strided by the workgroup size (a
// ragged tile, or a selection), and which are live; dead ones read row 0
// (the launch has nrows >= 1).
template <int NT, int ROWS>
__device__ __forceinline__ void round0_rows(const ScanArgs &a, uint32_t tile0, uint32_t tn, uint32_t *row,
                                            bool *alive) {
    StatusDev *status = a.status;
#pragma unroll
    for (int r = 0; r < ROWS; r++) {
        const uint32_t p = r * NT + threadIdx.x;
        alive[r] = p < tn;
        row[r] = tile_row(a, tile0, alive[r] ? p : 0u);   // position 0 of the tile exists
        alive[r] = alive[r] && CK(row[r] < a.nrows);
        row[r] = alive[r] ? row[r] : 0u;
    }
}

// LDS state of one workgroup: the batch of rows that passed round 0 (their
// rows and, per lookup, their hits) and the lists of batch entries that
// passed each later round.
struct ScanLds {
    uint32_t *bh;       // bh[j * nb + b]: lookup j's hit for batch entry b (dynamic LDS)
    uint32_t *brow;     // brow[b]: the entry's row of the cover relation
    uint16_t *lists;    // two lists of nb: entries alive after rounds 1, 2, ... (alternating)
    uint32_t *cnt;      // cnt[0]: batch entries; cnt[j]: entries alive after round j
    uint32_t nb;        // batch capacity in entries
};

// Direct emit of one chunk of final bindings, wave by wave (the thread's
// entry is entry i of the flush, with e result rows, 0 for none; fin lists
// the flush's batch entries, or null when entry i is batch entry i): a
// scan of the wave's row counts in registers, one reservation of the
// wave's rows in the output, then the wave writes them together, each row
// finding its lane by a search over the lanes' starts and its tail rows by
// mixed radix.  No LDS, so the kernel's occupancy is unchanged.
constexpr int kEmitFastTails = 4;   // up to this many tails, a row's loads are issued together
template <bool FAST>
__device__ __forceinline__ void scan_emit_wave(const ScanArgs &a, const uint32_t *bh, const uint32_t *brow,
                                            uint32_t nbs, const uint16_t *fin, uint32_t i, uint32_t nf, u64 e) {
    StatusDev *status = a.status;
    const EmitDev &d = *a.ed;
    const int lane = __lane_id();
    u64 x = e;
    for (int o = 1; o < 64; o <<= 1) {
        const u64 y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    const u64 wtot = __shfl(x, 63, 64);
    const u64 ex = x - e;
    if (wtot == 0) return;   // wave-uniform
    u64 base = 0;
    if (lane == 0) base = atomicAdd(&status->written, wtot);
    base = __shfl(base, 0, 64);
    const u64 room = base < a.cap ? a.cap - base : 0;
    const u64 nw = wtot < room ? wtot : room;   // rows past the output are counted, not written
    const uint32_t i_lane0 = i - (uint32_t)lane;
    for (u64 r0 = 0; r0 < nw; r0 += 64) {
        const u64 r = r0 + lane;
        // the lane t whose rows hold r: the largest t with ex_t <= r (every
        // lane takes part in the search's shuffles)
        int lo = 0, hi = 64;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (__shfl(ex, mid, 64) <= r) lo = mid; else hi = mid;
        }
        const u64 ex_t = __shfl(ex, lo, 64);
        if (r >= nw) continue;
        const uint32_t t = (uint32_t)lo;
        if (!CK(i_lane0 + t < nf)) continue;
        const uint32_t eb = fin ? fin[i_lane0 + t] : i_lane0 + t;
        u64 idx = r - ex_t;
        uint32_t rows[FJ_MAX_NODES];
        bool ok = true;
        if (FAST && d.ntail <= kEmitFastTails) {
            // few tails: each tail's length, then its row, all loaded before
            // any check (a check that reports keeps later loads behind it)
            uint32_t tp[kEmitFastTails], tn[kEmitFastTails], tps[kEmitFastTails];
            bool in = true;
#pragma unroll
            for (int q = 0; q < kEmitFastTails; q++) {
                tp[q] = 0;
                tn[q] = 1;
                if (q >= d.ntail) continue;
                tn[q] = a.tail_root_len[q];
                if (a.tail_lk[q] >= 0) {
                    tp[q] = bh[a.tail_lk[q] * nbs + eb];
                    const bool p_in = tp[q] < d.tail[q].L.npos;
                    tn[q] = p_in ? d.tail[q].L.len[tp[q]] : 0u;
                    in = in && p_in;
                }
            }
#pragma unroll
            for (int q = kEmitFastTails - 1; q >= 0; q--) {
                tps[q] = 0;
                if (q >= d.ntail) continue;
                in = in && tn[q] > 0;
                const uint32_t len = tn[q] > 0 ? tn[q] : 1u;
                tps[q] = tp[q] + (uint32_t)(idx % len);
                idx /= len;
                const TailDev &T = d.tail[q];
                in = in && (tps[q] < T.L.npos || (T.level == 0 && tps[q] < T.root_len));
            }
#pragma unroll
            for (int q = 0; q < kEmitFastTails; q++) {
                if (q >= d.ntail) continue;
                const TailDev &T = d.tail[q];
                const bool kv = T.nk == 1 && T.L.kv;
                const uint32_t x = in ? (kv ? (uint32_t)T.L.kv[tps[q]] : (T.L.offs ? T.L.offs[tps[q]] : tps[q])) : 0u;
                rows[q] = x;
                in = in && (kv || x < T.L.nrows);
            }
            ok = CK(in);
        } else {
        for (int q = d.ntail - 1; q >= 0 && ok; q--) {
            const TailDev &T = d.tail[q];
            uint32_t p = 0, len = a.tail_root_len[q];
            if (a.tail_lk[q] >= 0) {
                p = bh[a.tail_lk[q] * nbs + eb];
                ok = CK(p < T.L.npos);
                len = ok ? T.L.len[p] : 0u;
            }
            ok = ok && CK(len > 0);
            if (!ok) break;
            const uint32_t pos = p + (uint32_t)(idx % len);
            idx /= len;
            ok = CK(pos < T.L.npos || (T.level == 0 && pos < T.root_len));
            if (ok && T.nk == 1 && T.L.kv) {
                rows[q] = (uint32_t)T.L.kv[pos];   // the key kept beside the offset
                continue;
            }
            rows[q] = ok ? (T.L.offs ? T.L.offs[pos] : pos) : 0u;
            ok = ok && CK(rows[q] < T.L.nrows);
        }
        }
        if (!ok) continue;
        const uint32_t crow = brow[eb];
        int32_t *dst = d.out + (base + r) * (u64)d.nhead;
        // the row's values (FAST: eight columns' loads at a time before their
        // stores; the output may alias the columns, so a store keeps the next
        // load behind it)
        for (int j0 = 0; j0 < d.nhead; j0 += FAST ? 8 : 1) {
            constexpr int U = FAST ? 8 : 1;
            int32_t v[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int j = j0 + u;
                v[u] = 0;
                if (j >= d.nhead) continue;
                const int src = d.head_src[j];
                if (src >= 0) {
                    v[u] = a.cols[a.out_col[src]][crow];
                } else {
                    const int z = -src - 1;
                    const TailDev &T = d.tail[z / FJ_MAX_COLS];
                    v[u] = (T.nk == 1 && T.L.kv) ? (int32_t)rows[z / FJ_MAX_COLS]
                                                 : T.cols[T.kcol[z % FJ_MAX_COLS]][rows[z / FJ_MAX_COLS]];
                }
            }
#pragma unroll
            for (int u = 0; u < U; u++)
                if (j0 + u < d.nhead) dst[j0 + u] = v[u];
        }
    }
}

// Round 0, second half: scan the issued probes of the thread's rows; rows
// that hit join the batch.
template <int MODE, bool STATS>
__device__ __forceinline__ void round0_finish(const ScanArgs &a, const ScanLookup &L, const uint32_t *row,
                                              const bool *alive, RowProbe *pr, const ScanLds &S,
                                              uint32_t &nprobe, uint32_t &nhit) {
    StatusDev *status = a.status;
#pragma unroll
    for (int r = 0; r < kTileRows; r++) {
        bool hit = false;
        uint32_t v = 0;
        if (alive[r]) {
            if (STATS) nprobe++;
            hit = probe_resolve<MODE>(L, pr[r], v) && (MODE == KM_K32 || CK(v < L.cnpos));
            if (STATS && hit) nhit++;
        }
        const uint32_t b = list_slot(hit, &S.cnt[0]);
        if (hit) {
            S.brow[b] = row[r];
            S.bh[b] = v;
        }
    }
}

// Keys of one column for the thread's rows of a whole tile (VEC layout).
__device__ __forceinline__ void tile_keys(const int32_t *c, uint32_t row0, uint32_t *k) {
    if constexpr (kTileRows % 4 == 0) {
#pragma unroll
        for (int r = 0; r < kTileRows; r += 4) {
            const int4 x = *(const int4 *)(c + row0 + r);
            k[r] = x.x; k[r + 1] = x.y; k[r + 2] = x.z; k[r + 3] = x.w;
        }
    } else if constexpr (kTileRows == 2) {
        const int2 x = *(const int2 *)(c + row0);
        k[0] = x.x; k[1] = x.y;
    } else {
#pragma unroll
        for (int r = 0; r < kTileRows; r++) k[r] = (uint32_t)c[row0 + r];
    }
}

// Round j >= 1: lookup L over the n batch entries the previous round left
// (round 1: the whole batch), kRoundRows entries per thread in flight.
template <int NT, int MODE, bool STATS, int RR = kRoundRows>
__device__ __forceinline__ void scan_round(const ScanArgs &a, const ScanLookup &L, int j, uint32_t n,
                                           const ScanLds &S, uint32_t &nprobe, uint32_t &nhit) {
    StatusDev *status = a.status;
    const uint16_t *in = j == 1 ? nullptr : S.lists + ((j - 1) & 1) * S.nb;
    uint16_t *out = S.lists + (j & 1) * S.nb;
    const int32_t *c0 = a.cols[L.kc[0]];
    const int32_t *c1 = a.cols[MODE != KM_K32 ? L.kc[1] : L.kc[0]];
    for (uint32_t i0 = 0; i0 < n; i0 += NT * RR) {
        uint32_t b[RR], k0[RR], k1[RR];
        bool live[RR];
#pragma unroll
        for (int r = 0; r < RR; r++) {
            const uint32_t i = i0 + r * NT + threadIdx.x;
            live[r] = i < n;
            b[r] = live[r] ? (in ? in[i] : i) : 0u;   // entry 0 exists (n > 0)
            const uint32_t row = S.brow[b[r]];
            k0[r] = (uint32_t)c0[row];
            k1[r] = MODE != KM_K32 ? (uint32_t)c1[row] : 0u;
        }
        RowProbe pr[RR];
#pragma unroll
        for (int r = 0; r < RR; r++) probe_issue<MODE>(L, k0[r], k1[r], live[r], pr[r]);
#pragma unroll
        for (int r = 0; r < RR; r++) {
            bool hit = false;
            if (live[r]) {
                if (STATS) nprobe++;
                uint32_t v = 0;
                hit = probe_resolve<MODE>(L, pr[r], v) && (MODE == KM_K32 || CK(v < L.cnpos));
                if (hit) {
                    if (STATS) nhit++;
                    S.bh[j * S.nb + b[r]] = v;
                }
            }
            const uint32_t o = list_slot(hit, &S.cnt[j]);
            if (hit) out[o] = (uint16_t)b[r];
        }
    }
}

// Rounds 1..nl-1 over the batch, then the batch's results: counts (emit)
// and/or frontier rows (materialize, or a node that is not the last).  Every
// thread of the workgroup calls it; it leaves the batch empty.
template <int NT, bool STATS, bool FAST = false>
__device__ __forceinline__ void scan_flush(const ScanArgs &a, const ScanLds &S, uint32_t nb, u64 &tot,
                                           uint32_t &nprobe, uint32_t &nhit, u64 *red) {
    StatusDev *status = a.status;
    uint32_t nf = nb;
    int last = 0;
    for (int j = 1; j < a.nl && nf > 0; j++) {
        // (FAST: more entries a thread in flight, for batches flushed once)
        constexpr int RR = FAST ? 2 * kRoundRows : kRoundRows;
        if (a.lk[j].mode == KM_K32) scan_round<NT, KM_K32, STATS, RR>(a, a.lk[j], j, nf, S, nprobe, nhit);
        else scan_round<NT, KM_K64, STATS, RR>(a, a.lk[j], j, nf, S, nprobe, nhit);
        __syncthreads();
        nf = S.cnt[j];
        last = j;
    }
    if (nf > 0) {
        const uint16_t *fin = last == 0 ? nullptr : S.lists + (last & 1) * S.nb;
        const bool write = (!a.emit || a.materialize) && !a.direct;
        if (write) {
            if (threadIdx.x == 0) red[16] = atomicAdd(&a.status->survivors, (u64)nf);
            __syncthreads();
        }
        const u64 base = write ? red[16] - a.surv_base : 0;
        // chunks of NT entries, one per thread (all threads take part in
        // every chunk: the direct emit scans each chunk)
        for (uint32_t i0 = 0; i0 < nf; i0 += NT) {
            const uint32_t i = i0 + threadIdx.x;
            const bool live = i < nf;
            const uint32_t b = live ? (fin ? fin[i] : i) : 0u;
            bool ok;
            u64 e = 0, m = 1;
            if constexpr (FAST) {
                // slots of KM_K32 maps become their values (the child handles).
                // Here and below every load of an entry is issued before any of
                // its checks: a check that fails reports to the status block, so
                // the compiler keeps later loads behind it.
                uint32_t hv[kScanMaxLookups];
#pragma unroll
                for (int j = 0; j < kScanMaxLookups; j++) {
                    hv[j] = 0;
                    if (j < a.nl && live) {
                        const uint32_t x = S.bh[j * S.nb + b];
                        hv[j] = a.lk[j].mode == KM_K32 ? ((const uint32_t *)a.lk[j].table)[k32_key_word(x) + 4] : x;
                    }
                }
                bool in = live;
#pragma unroll
                for (int j = 0; j < kScanMaxLookups; j++)
                    if (j < a.nl) in = in && (a.lk[j].mode != KM_K32 || hv[j] < a.lk[j].cnpos);
                ok = live && CK(in);
                if (ok) {
#pragma unroll
                    for (int j = 0; j < kScanMaxLookups; j++)
                        if (j < a.nl) S.bh[j * S.nb + b] = hv[j];
                    uint32_t cl[kScanMaxLookups];
#pragma unroll
                    for (int j = 0; j < kScanMaxLookups; j++)
                        cl[j] = (j < a.nl && a.lk[j].child_leaf) ? a.lk[j].clen[hv[j]] : 1u;
                    uint32_t tl[FJ_MAX_NODES];
                    bool tin = true;
                    if (a.emit) {
#pragma unroll
                        for (int q = 0; q < FJ_MAX_NODES; q++) {
                            tl[q] = 1;
                            if (q >= a.ntail) continue;
                            if (a.tail_lk[q] < 0) { tl[q] = a.tail_root_len[q]; continue; }
                            const uint32_t th = hv[a.tail_lk[q] & (kScanMaxLookups - 1)];
                            const bool t_in = th < a.tail_npos[q];
                            tl[q] = t_in ? a.tail_len[q][th] : 0u;
                            tin = tin && t_in;
                        }
                    }
#pragma unroll
                    for (int j = 0; j < kScanMaxLookups; j++) m *= cl[j];
                    if (a.emit) {
                        e = m;
#pragma unroll
                        for (int q = 0; q < FJ_MAX_NODES; q++) e *= tl[q];
                        if (!CK(tin)) e = 0;
                        tot += e;
                    }
                }
            } else {
                // slots of KM_K32 maps become their values (the child handles)
                ok = live;
                for (int j = 0; j < a.nl && live; j++) {
                    const ScanLookup &L = a.lk[j];
                    if (L.mode != KM_K32) continue;
                    const uint32_t v = ((const uint32_t *)L.table)[k32_key_word(S.bh[j * S.nb + b]) + 4];
                    ok = ok && CK(v < L.cnpos);
                    S.bh[j * S.nb + b] = v;
                }
                if (ok) {
                    for (int j = 0; j < a.nl; j++)
                        if (a.lk[j].child_leaf) m *= a.lk[j].clen[S.bh[j * S.nb + b]];
                    if (a.emit) {
                        e = m;
                        for (int q = 0; q < a.ntail; q++) {
                            if (a.tail_lk[q] < 0) { e *= a.tail_root_len[q]; continue; }
                            const uint32_t th = S.bh[a.tail_lk[q] * S.nb + b];
                            if (!CK(th < a.tail_npos[q])) { e = 0; break; }
                            e *= a.tail_len[q][th];
                        }
                        tot += e;
                    }
                }
            }
            if (ok) {
                const u64 pos = base + i;
                if (write && CK(pos < a.out.cap)) {
                    const FrontierDev &O = a.out;
                    const uint32_t row = S.brow[b];
                    for (int j = 0; j < a.nout; j++) O.vals[(u64)j * O.cap + pos] = a.cols[a.out_col[j]][row];
                    for (int j = 0; j < a.nl; j++)
                        if (a.lk[j].hcol >= 0) O.hdl[(u64)a.lk[j].hcol * O.cap + pos] = S.bh[j * S.nb + b];
                    if (O.mult) O.mult[pos] = m;
                }
            }
            if (a.direct) scan_emit_wave<FAST>(a, S.bh, S.brow, S.nb, fin, i, nf, e);
        }
    }
    __syncthreads();   // every entry of the batch is read: empty it
    if (threadIdx.x <= kScanMaxLookups) S.cnt[threadIdx.x] = 0;
    __syncthreads();
}

// Persistent workgroups: workgroup g takes tiles g, g + G, g + 2G, ... and
// runs round 0 over each; when the batch could not take another whole tile
// (or the tiles run out) the later rounds run over the batch.  So the
// dependent latencies of the later rounds are paid once per batch, not once
// per tile.  A whole tile's keys (VEC layout) are loaded one tile ahead, so
// their latency hides behind the current tile's probes.
template <int MODE, bool STATS>
__device__ __forceinline__ void scan_tiles(const ScanArgs &a, const ScanLds &S, u64 &tot, uint32_t &nprobe,
                                           uint32_t &nhit, u64 *red) {
    const ScanLookup &L = a.lk[0];
    const int32_t *c0 = a.cols[L.kc[0]];
    const int32_t *c1 = a.cols[MODE == KM_K32 ? L.kc[0] : L.kc[1]];
    const uint32_t ntiles = (a.n + kTile - 1) / kTile;
    const uint32_t nfull = a.vec ? a.n / kTile : 0;   // tiles read with the VEC layout
    // keys of whole tiles, in two register sets used in turn (the loop is
    // unrolled by two), so that no loaded key is ever copied: a copy would
    // wait for its load
    uint32_t ka0[kTileRows], ka1[kTileRows], kb0[kTileRows], kb1[kTileRows];
    auto prefetch = [&](uint32_t t, uint32_t *k0, uint32_t *k1) {
        if (t < nfull) {
            const uint32_t row0 = a.r0 + t * kTile + threadIdx.x * kTileRows;
            tile_keys(c0, row0, k0);
            if constexpr (MODE != KM_K32) tile_keys(c1, row0, k1);
        }
    };
    // tile t with its keys in (k0, k1) if it is whole; prefetch the keys of
    // the workgroup's next tile into (n0, n1)
    auto tile = [&](uint32_t t, const uint32_t *k0, const uint32_t *k1, uint32_t *n0, uint32_t *n1) {
        const uint32_t tile0 = t * (uint32_t)kTile;
        const uint32_t tn = min((uint32_t)kTile, a.n - tile0);
        uint32_t row[kTileRows];
        bool alive[kTileRows];
        RowProbe pr[kTileRows];
        if (t < nfull) {
#pragma unroll
            for (int r = 0; r < kTileRows; r++) {
                row[r] = a.r0 + tile0 + threadIdx.x * kTileRows + r;
                alive[r] = true;
            }
#pragma unroll
            for (int r = 0; r < kTileRows; r++)
                probe_issue<MODE>(L, k0[r], MODE != KM_K32 ? k1[r] : 0u, true, pr[r]);
            prefetch(t + gridDim.x, n0, n1);
        } else {
            round0_rows<256, kTileRows>(a, tile0, tn, row, alive);
            uint32_t s0[kTileRows], s1[kTileRows];
#pragma unroll
            for (int r = 0; r < kTileRows; r++) {
                s0[r] = (uint32_t)c0[row[r]];
                s1[r] = MODE != KM_K32 ? (uint32_t)c1[row[r]] : 0u;
            }
#pragma unroll
            for (int r = 0; r < kTileRows; r++) probe_issue<MODE>(L, s0[r], s1[r], alive[r], pr[r]);
        }
        round0_finish<MODE, STATS>(a, L, row, alive, pr, S, nprobe, nhit);
        __syncthreads();
        const uint32_t nb = S.cnt[0];
        __syncthreads();   // read by every thread before the next tile adds to it: block-uniform
        if (nb > 0 && (nb > (uint32_t)(kBatch - kTile) || t + gridDim.x >= ntiles))
            scan_flush<256, STATS>(a, S, nb, tot, nprobe, nhit, red);
    };
    prefetch(blockIdx.x, ka0, ka1);
    for (uint32_t t = blockIdx.x; t < ntiles; t += 2 * gridDim.x) {
        tile(t, ka0, ka1, kb0, kb1);
        if (t + gridDim.x < ntiles) tile(t + gridDim.x, kb0, kb1, ka0, ka1);
    }
}

// A node with no lookups: every live cover row is a result.
template <bool STATS>
__device__ __forceinline__ void scan_all(const ScanArgs &a, const ScanLds &S, u64 &tot, uint32_t &nprobe,
                                         uint32_t &nhit, u64 *red) {
    const uint32_t ntiles = (a.n + kTile - 1) / kTile;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const uint32_t tile0 = t * (uint32_t)kTile;
        const uint32_t tn = min((uint32_t)kTile, a.n - tile0);
        uint32_t row[kTileRows];
        bool alive[kTileRows];
        round0_rows<256, kTileRows>(a, tile0, tn, row, alive);
#pragma unroll
        for (int r = 0; r < kTileRows; r++) {
            const uint32_t b = list_slot(alive[r], &S.cnt[0]);
            if (alive[r]) S.brow[b] = row[r];
        }
        __syncthreads();
        const uint32_t nb = S.cnt[0];
        __syncthreads();   // read by every thread before the next tile adds to it
        if (nb > 0 && (nb > (uint32_t)(kBatch - kTile) || t + gridDim.x >= ntiles))
            scan_flush<256, STATS>(a, S, nb, tot, nprobe, nhit, red);
    }
}

// A KM_K32 probe in two steps with only the key and the loaded bucket's
// keys held between them (the bucket is hashed again to resolve).
struct Probe32 {
    uint4 q;
    uint32_t key;
};

__device__ __forceinline__ void probe32_issue(const ScanLookup &L, uint32_t key, bool alive, Probe32 &rp) {
    rp.key = key;
    const u64 b = (alive && key != kEmpty32) ? k32_bucket(mix32(key), L.mask) : 0ull;
    rp.q = *(const uint4 *)((const uint32_t *)L.table + k32_key_word(b));
}

// true on a hit; out = its slot
__device__ __forceinline__ bool probe32_resolve(const ScanLookup &L, const Probe32 &rp, uint32_t &out) {
    const uint32_t *T = (const uint32_t *)L.table;
    out = (uint32_t)(L.mask + 1);
    if (rp.key == kEmpty32) return T[k32_key_word(L.mask + 1)] != 0u;
    u64 idx = k32_bucket(mix32(rp.key), L.mask);
    uint4 q = rp.q;
    int s = 0;
    int st = scan_keys32(q, rp.key, s);
    for (u64 n = kK32Bucket; st == 0 && n <= k32_part_mask(L.mask); n += kK32Bucket) {   // a full bucket (rare)
        idx = k32_next(idx, L.mask);
        q = *(const uint4 *)(T + k32_key_word(idx));
        st = scan_keys32(q, rp.key, s);
    }
    out = (uint32_t)(idx + s);
    return st == 1;
}

// The rounds pass of a two-launch first node: workgroup b takes the filter
// pass's regions [b l0_per, (b + 1) l0_per) as one sequence of rows, probes
// the first lookup for kListRows rows per thread at a time (every load in
// flight together), and the rows that hit join the batch; the later
// lookups run as rounds over each batch.  The first lookup's probes were
// counted by the filter pass (each row once); its hits are counted here.
constexpr int kListRows = 4;
constexpr int kListChunk = 256 * kListRows;
constexpr int kListPerMax = 8;   // regions a workgroup takes at most
static_assert(kListChunk <= kBatch, "a chunk's hits fit an empty batch");
template <bool STATS>
__device__ __forceinline__ void scan_list(const ScanArgs &a, const ScanLds &S, u64 &tot, uint32_t &nprobe,
                                          uint32_t &nhit, u64 *red) {
    StatusDev *status = a.status;
    const ScanLookup &L = a.lk[0];
    const uint32_t ftiles = (a.n + kFiltTile - 1) / kFiltTile;
    const uint32_t items = a.l0_groups * kFiltWaves;
    const uint32_t it0 = blockIdx.x * a.l0_per;
    const uint32_t nit = it0 < items ? min(a.l0_per, items - it0) : 0u;
    uint32_t cn[kListPerMax], total = 0;
#pragma unroll
    for (int k = 0; k < kListPerMax; k++) cn[k] = k < (int)nit ? a.l0_cnt[it0 + k] : 0u;
#pragma unroll
    for (int k = 0; k < kListPerMax; k++) total += cn[k];
    for (uint32_t c0 = 0; c0 < total; c0 += kListChunk) {
        uint32_t row[kListRows];
        bool live[kListRows];
        Probe32 pr[kListRows];
#pragma unroll
        for (int r = 0; r < kListRows; r++) {
            // entry e of the workgroup's sequence: its region and place
            uint32_t e = c0 + r * 256 + threadIdx.x;
            live[r] = e < total;
            uint32_t k = 0;
            bool found = false;
#pragma unroll
            for (int q = 0; q < kListPerMax; q++) {
                const bool here = !found && e < cn[q];
                k = here ? (uint32_t)q : k;
                found = found || here;
                e -= found ? 0u : cn[q];
            }
            uint32_t cap = 0;
            const u64 rs = live[r] ? list_region((it0 + k) / kFiltWaves, (it0 + k) % kFiltWaves, ftiles, a.l0_groups,
                                                 cap)
                                   : 0ull;
            live[r] = live[r] && CK(k < nit && e < cap);
            row[r] = live[r] ? a.l0_row[rs + e] : 0u;
            pr[r].key = live[r] ? a.l0_key[rs + e] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kListRows; r++) {
            live[r] = live[r] && CK(row[r] < a.nrows);
            probe32_issue(L, pr[r].key, live[r], pr[r]);
        }
#pragma unroll
        for (int r = 0; r < kListRows; r++) {
            uint32_t v = 0;
            const bool hit = live[r] && probe32_resolve(L, pr[r], v);
            if (STATS && hit) nhit++;
            const uint32_t b = list_slot(hit, &S.cnt[0]);
            if (hit) {
                S.brow[b] = row[r];
                S.bh[b] = v;
            }
        }
        __syncthreads();
        const uint32_t nb = S.cnt[0];
        __syncthreads();   // read by every thread before the next chunk adds to it
        // flushed when the next chunk's hits might not fit, or at the end
        const uint32_t next = c0 + kListChunk < total ? min((uint32_t)kListChunk, total - c0 - kListChunk) : 0u;
        if (nb > 0 && (next == 0 || nb + next > (uint32_t)kBatch))
            scan_flush<256, STATS, true>(a, S, nb, tot, nprobe, nhit, red);
    }
}

template <bool STATS>
__global__ void __launch_bounds__(256, FJ_SCAN_WAVES) k_scan_probe(ScanArgs a) {
    StatusDev *status = a.status;
    extern __shared__ uint32_t bh[];
    __shared__ uint32_t brow[kBatch];
    __shared__ uint16_t lists[2 * kBatch];
    __shared__ uint32_t cnt[kScanMaxLookups + 1];
    __shared__ u64 red[17];
    const ScanLds S{bh, brow, lists, cnt, (uint32_t)kBatch};
    if (threadIdx.x <= kScanMaxLookups) cnt[threadIdx.x] = 0;
    __syncthreads();
    uint32_t nprobe = 0, nhit = 0;
    u64 tot = 0;
    if (a.nl == 0) scan_all<STATS>(a, S, tot, nprobe, nhit, red);
    else if (a.lk[0].mode == KM_K32) scan_tiles<KM_K32, STATS>(a, S, tot, nprobe, nhit, red);
    else scan_tiles<KM_K64, STATS>(a, S, tot, nprobe, nhit, red);
    if (STATS) {
        u64 np = wave_sum_u64(nprobe), nh = wave_sum_u64(nhit);
        if (__lane_id() == 0 && (np | nh)) {
            atomicAdd(&a.status->probe[a.node], np);
            atomicAdd(&a.status->hit[a.node], nh);
        }
    }
    if (a.emit) block_add_count(tot, status, red);
}

// The rounds pass of a two-launch first node (its own kernel, so that the
// one-launch kernel's registers are not sized for both).
template <bool STATS>
__global__ void __launch_bounds__(256, FJ_SCAN_WAVES) k_scan_rounds(ScanArgs a) {
    StatusDev *status = a.status;
    extern __shared__ uint32_t bh[];
    __shared__ uint32_t brow[kBatch];
    __shared__ uint16_t lists[2 * kBatch];
    __shared__ uint32_t cnt[kScanMaxLookups + 1];
    __shared__ u64 red[17];
    const ScanLds S{bh, brow, lists, cnt, (uint32_t)kBatch};
    if (threadIdx.x <= kScanMaxLookups) cnt[threadIdx.x] = 0;
    __syncthreads();
    uint32_t nprobe = 0, nhit = 0;
    u64 tot = 0;
    scan_list<STATS>(a, S, tot, nprobe, nhit, red);
    if (STATS) {
        u64 np = wave_sum_u64(nprobe), nh = wave_sum_u64(nhit);
        if (__lane_id() == 0 && (np | nh)) {
            atomicAdd(&a.status->probe[a.node], np);
            atomicAdd(&a.status->hit[a.node], nh);
        }
    }
    if (a.emit) block_add_count(tot, status, red);
}

// ---------------------------------------------- filter pass of the scan
// The first node in two launches when its first lookup's map carries a
// membership filter (written with the map).  This pass streams the cover's
// first key column and tests each key against the filter held in LDS: a
// row whose key lacks one of its two bits misses the first lookup without
// touching the map.  On a selective join most rows leave here.  The others
// are written with their keys to the wave's own region of a list (placed by
// a scan over the wave's lanes: no atomics, no barriers), and k_scan_rounds
// probes them, many per thread at once, and runs the later lookups.  What
// bounds such a node is the chain of dependent memory round trips each
// wave makes; this pass makes none beyond its stream, which it keeps one
// tile ahead.  The filter takes 64 KB of LDS and the pass 64 registers a
// thread, so that two 1,024-thread workgroups share a CU; tiles are 8 rows
// per thread.

__device__ __forceinline__ bool bloom_pass(const uint32_t *filt, const ScanLookup &L, uint32_t key) {
    if (key == kEmpty32) return true;   // kept in the reserved slot, not in the filter
    const uint32_t h = mix32(key);
    const uint32_t bits = bloom_bits(h);
    return (filt[bloom_word(h, L.mask, L.bloom_shift)] & bits) == bits;
}

// Row r of the thread in filter-pass tile t (whole tiles: the thread's
// kFiltRows consecutive rows; a ragged tile or a selection: strided
// positions).
__device__ __forceinline__ uint32_t filt_row(const ScanArgs &a, uint32_t tile0, uint32_t tn, bool whole, int r,
                                             bool &alive) {
    StatusDev *status = a.status;
    if (whole) {
        alive = true;
        return a.r0 + tile0 + threadIdx.x * kFiltRows + r;
    }
    const uint32_t p = r * kFiltThreads + threadIdx.x;
    alive = p < tn;
    uint32_t row = tile_row(a, tile0, alive ? p : 0u);
    alive = alive && CK(row < a.nrows);
    return alive ? row : 0u;
}

template <bool STATS>
__global__ void __launch_bounds__(kFiltThreads, 8) k_scan_filter(ScanArgs a) {
    StatusDev *status = a.status;
    __shared__ uint4 filt4[kBloomWords / 4];
    const uint32_t *filt = (const uint32_t *)filt4;
    const ScanLookup &L = a.lk[0];
    {
        // the filter's words (a multiple of four), every load in flight at once
        constexpr int V = kBloomWords / 4 / kFiltThreads;
        const uint4 *src = (const uint4 *)L.bloom;
        const uint32_t nv = L.bloom_words / 4;
        uint4 v[V];
#pragma unroll
        for (int k = 0; k < V; k++) {
            const uint32_t i = k * kFiltThreads + threadIdx.x;
            v[k] = i < nv ? src[i] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int k = 0; k < V; k++) {
            const uint32_t i = k * kFiltThreads + threadIdx.x;
            if (i < nv) filt4[i] = v[k];
        }
    }
    __syncthreads();
    uint32_t nprobe = 0, nfilt = 0;
    const int32_t *c0 = a.cols[L.kc[0]];
    const uint32_t ntiles = (a.n + kFiltTile - 1) / kFiltTile;
    const uint32_t nfull = a.vec ? a.n / kFiltTile : 0;
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    uint32_t wcap;
    const u64 rs = list_region(blockIdx.x, wid, ntiles, gridDim.x, wcap);
    uint32_t *orow = a.l0_row + rs, *okey = a.l0_key + rs;
    uint32_t cnt = 0;   // hits the wave has written (wave-uniform)
    uint32_t ka[kFiltRows], kb[kFiltRows];
    auto prefetch = [&](uint32_t t, uint32_t *k) {
        if (t < nfull) {
            const int32_t *c = c0 + a.r0 + t * kFiltTile + threadIdx.x * kFiltRows;
#pragma unroll
            for (int r = 0; r < kFiltRows; r += 4) {
                const int4 x = *(const int4 *)(c + r);
                k[r] = x.x; k[r + 1] = x.y; k[r + 2] = x.z; k[r + 3] = x.w;
            }
        }
    };
    auto tile = [&](uint32_t t, const uint32_t *k, uint32_t *nk) {
        const uint32_t tile0 = t * (uint32_t)kFiltTile;
        const uint32_t tn = min((uint32_t)kFiltTile, a.n - tile0);
        const bool whole = t < nfull;
        uint32_t alive = 0, pass = 0;   // bit r: row r of the thread
        struct { uint32_t key; } pr[kFiltRows];
        if (whole) {
            alive = (1u << kFiltRows) - 1u;
#pragma unroll
            for (int r = 0; r < kFiltRows; r++) pr[r].key = k[r];
        } else {
#pragma unroll
            for (int r = 0; r < kFiltRows; r++) {
                bool al;
                const uint32_t rw = filt_row(a, tile0, tn, false, r, al);
                pr[r].key = al ? (uint32_t)c0[rw] : 0u;
                alive |= al ? 1u << r : 0u;
            }
        }
#pragma unroll
        for (int r = 0; r < kFiltRows; r++)
            pass |= (((alive >> r) & 1u) && bloom_pass(filt, L, pr[r].key)) ? 1u << r : 0u;
        prefetch(t + gridDim.x, nk);
        if (STATS) {
            nprobe += (uint32_t)__popc(alive);
            nfilt += (uint32_t)__popc(alive & ~pass);
        }
        // the wave's passing rows of the tile in (lane, row) order after its
        // earlier tiles' (a scan over the lanes, no barrier)
        const uint32_t h = (uint32_t)__popc(pass);
        uint32_t x = h;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        uint32_t off = cnt + x - h;
#pragma unroll
        for (int r = 0; r < kFiltRows; r++) {
            if (!((pass >> r) & 1u)) continue;
            bool al;
            if (CK(off < wcap)) {
                orow[off] = filt_row(a, tile0, tn, whole, r, al);
                okey[off] = pr[r].key;
            }
            off++;
        }
        cnt += __shfl(x, 63, 64);
    };
    prefetch(blockIdx.x, ka);
    for (uint32_t t = blockIdx.x; t < ntiles; t += 2 * gridDim.x) {
        tile(t, ka, kb);
        if (t + gridDim.x < ntiles) tile(t + gridDim.x, kb, ka);
    }
    if (lane == 0) a.l0_cnt[blockIdx.x * kFiltWaves + wid] = cnt;
    if (STATS) {
        u64 np = wave_sum_u64(nprobe), nf = wave_sum_u64(nfilt);
        if (__lane_id() == 0 && (np | nf)) {
            atomicAdd(&a.status->probe[a.node], np);
            atomicAdd(&a.status->filtered, nf);
        }
    }
}

// ------------------------------------------------------- emit (launches)
// Rows are laid out by a scan of the bindings' row counts.



__device__ __forceinline__ uint32_t emit_handle(const EmitDev &d, int atom, uint32_t e) {
    for (int j = 0; j < d.nin_h; j++)
        if (d.in_h_atom[j] == atom) return d.F.hdl[(u64)j * d.F.cap + e];
    return 0xFFFFFFFFu;
}

__device__ __forceinline__ uint32_t tail_len(const EmitDev &d, const TailDev &T, uint32_t e, uint32_t &p,
                                             StatusDev *status) {
    if (T.level == 0) { p = 0; return T.root_len; }
    p = emit_handle(d, T.atom, e);
    if (!CK(p < T.L.npos)) { p = 0; return 0u; }
    return T.L.len[p];
}

// Result rows of binding e (the multiplicity times every tail's length).
__device__ __forceinline__ u64 emit_rows_of(const EmitDev &d, uint32_t e, StatusDev *status) {
    if (!CK(e < d.F.cap)) return 0;
    u64 v = d.F.mult ? d.F.mult[e] : 1ull;
    for (int q = 0; q < d.ntail; q++) {
        uint32_t p;
        v *= tail_len(d, d.tail[q], e, p, status);
    }
    return v;
}

// Few bindings (E <= kEmitSmall): their counts, the scan into starts (with
// starts[E] = total) and the emit's place in the output (as
// k_scan_blocks_emit) in one workgroup.
constexpr int kEmitSmallThreads = 1024;
constexpr int kEmitSmallItems = 1;
constexpr uint32_t kEmitSmall = kEmitSmallThreads * kEmitSmallItems;

__global__ void __launch_bounds__(kEmitSmallThreads) k_emit_count_small(const EmitDev *__restrict__ dp, uint32_t E,
                                                                        u64 *starts, StatusDev *status, u64 cap) {
    __shared__ u64 lds[17];
    const EmitDev &d = *dp;
    u64 v[kEmitSmallItems];
    u64 sum = 0;
    const uint32_t e0 = threadIdx.x * kEmitSmallItems;
#pragma unroll
    for (int j = 0; j < kEmitSmallItems; j++) {
        v[j] = e0 + j < E ? emit_rows_of(d, e0 + j, status) : 0ull;
        sum += v[j];
    }
    u64 tot;
    u64 ex = block_excl_scan<u64>(sum, lds, tot);
#pragma unroll
    for (int j = 0; j < kEmitSmallItems; j++) {
        if (e0 + j < E) starts[e0 + j] = ex;
        ex += v[j];
    }
    if (threadIdx.x == 0) {
        starts[E] = tot;
        status->total = tot;
        const u64 base = status->written;
        const u64 rows = base < cap ? (tot < cap - base ? tot : cap - base) : 0;
        status->emit_base = base;
        status->emit_rows = rows;
        status->written = base + rows;
    }
}

__global__ void __launch_bounds__(256) k_emit_count(const EmitDev *__restrict__ dp, uint32_t E, u64 *cnt,
                                                    StatusDev *status) {
    uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < E) cnt[e] = emit_rows_of(*dp, e, status);
}

// Result row r, of binding e whose rows are [s0, s1), to output row o.
__device__ __forceinline__ void emit_row_at(const EmitDev &d, uint32_t E, uint32_t e, u64 s0, u64 s1, u64 r, u64 o,
                                            StatusDev *status) {
    if (!CK(e < E && e < d.F.cap && r >= s0 && r < s1 && o < d.out_rows)) return;
    u64 idx = r - s0;
    uint32_t rows[FJ_MAX_NODES];
    for (int q = d.ntail - 1; q >= 0; q--) {
        const TailDev &T = d.tail[q];
        uint32_t p;
        uint32_t len = tail_len(d, T, e, p, status);
        if (!CK(len > 0)) return;
        uint32_t i = (uint32_t)(idx % len);
        idx /= len;
        uint32_t pos = p + i;
        if (!CK(pos < T.L.npos || (T.level == 0 && pos < T.root_len))) return;
        if (T.nk == 1 && T.L.kv) {
            // a one-variable level keeps its key beside the offset: the
            // value is read there, with no gather through the row
            rows[q] = (uint32_t)T.L.kv[pos];
            continue;
        }
        rows[q] = T.L.offs ? T.L.offs[pos] : pos;
        if (!CK(rows[q] < T.L.nrows)) return;
    }
    int32_t *dst = d.out + o * (u64)d.nhead;
    for (int j = 0; j < d.nhead; j++) {
        int s = d.head_src[j];
        if (s >= 0) {
            dst[j] = d.F.vals[(u64)s * d.F.cap + e];
        } else {
            int z = -s - 1;
            int q = z / FJ_MAX_COLS, c = z % FJ_MAX_COLS;
            const TailDev &T = d.tail[q];
            dst[j] = (T.nk == 1 && T.L.kv) ? (int32_t)rows[q] : T.cols[T.kcol[c]][rows[q]];
        }
    }
}

// The binding of row r: r itself when every binding holds one row, else
// the largest e with starts[e] <= r.
__device__ __forceinline__ uint32_t binding_of(const u64 *starts, uint32_t E, u64 r) {
    uint32_t e = (uint32_t)(r < E ? r : E - 1);
    if (!(starts[e] <= r && r < starts[e + 1])) e = upper_entry(starts, 0, E, r);
    return e;
}

// Rows [0, emit_rows) of the current emit, at output rows emit_base + r
// (both set on the device by the emit's scan), grid-stride.  Each thread
// finds its row's binding on its own: with many waves in flight the search
// hides behind the row's gathers, which bound the kernel.
__global__ void __launch_bounds__(256) k_emit_rows(const EmitDev *__restrict__ dp, uint32_t E, const u64 *starts,
                                                   StatusDev *status) {
    const u64 nrows = status->emit_rows, base = status->emit_base;
    if (E == 0) return;
    for (u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x; r < nrows; r += (u64)gridDim.x * blockDim.x) {
        const uint32_t e = binding_of(starts, E, r);
        emit_row_at(*dp, E, e, starts[e], starts[e + 1], r, base + r, status);
    }
}

// Rows [first, first + n) of a factorized result to output rows [0, n).
__global__ void __launch_bounds__(256) k_emit_range(const EmitDev *__restrict__ dp, uint32_t E, const u64 *starts,
                                                    u64 first, u64 n, StatusDev *status) {
    if (E == 0) return;
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (u64)gridDim.x * blockDim.x) {
        const uint32_t e = binding_of(starts, E, first + i);
        emit_row_at(*dp, E, e, starts[e], starts[e + 1], first + i, i, status);
    }
}

// The emit of a node-0 scan's last tile, enqueued before its survivor count
// is known on the host: E = *surv - surv_base bindings, read here.  Up to
// kEmitSmall bindings it does what k_emit_count_small does (counts, scan,
// place), keeping the scan in LDS, and when the rows are at most kEmitFuse
// it also writes them, leaving emit_rows = 0; otherwise it leaves the status
// untouched for the host's general path after its wait.
constexpr u64 kEmitFuse = 1u << 16;

__global__ void __launch_bounds__(kEmitSmallThreads) k_emit_small_dev(const EmitDev *__restrict__ dp,
                                                                      const u64 *surv, u64 surv_base, u64 *starts,
                                                                      StatusDev *status, u64 cap) {
    __shared__ u64 lds[17];
    __shared__ u64 sst[kEmitSmall + 1];
    __shared__ u64 place[2];
    const EmitDev &d = *dp;
    const u64 En = *surv - surv_base;   // the same value for every thread
    if (En == 0 || En > kEmitSmall) return;
    const uint32_t E = (uint32_t)En;
    const uint32_t e = threadIdx.x;
    const u64 v = e < E ? emit_rows_of(d, e, status) : 0ull;
    u64 tot;
    const u64 ex = block_excl_scan<u64>(v, lds, tot);
    if (e < E) {
        starts[e] = ex;
        sst[e] = ex;
    }
    if (threadIdx.x == 0) {
        starts[E] = tot;
        sst[E] = tot;
        status->total = tot;
        const u64 base = status->written;
        const u64 rows = base < cap ? (tot < cap - base ? tot : cap - base) : 0;
        status->emit_base = base;
        status->written = base + rows;
        status->emit_rows = rows <= kEmitFuse ? 0ull : rows;
        place[0] = base;
        place[1] = rows;
    }
    __syncthreads();
    const u64 base = place[0], rows = place[1];
    if (rows > kEmitFuse) return;   // the host's k_emit_rows writes them
    for (u64 r = threadIdx.x; r < rows; r += blockDim.x) {
        uint32_t b = (uint32_t)(r < E ? r : E - 1);
        if (!(sst[b] <= r && r < sst[b + 1])) b = upper_entry_lds(sst, 0, E, r);
        emit_row_at(d, E, b, sst[b], sst[b + 1], r, base + r, status);
    }
}

// ------------------------------------------------------------- eager tries
// Queue every child trie of level L's forced tries for forcing (the simple
// trie of the paper's ablation builds every level ahead): position q of L
// starts a forced trie when st[q] holds its key count + 1; the child starts
// of its keys are kl[q .. q + keys).  root: L is a root level, whose one
// trie (position 0) may hold millions of keys: thread q takes its key q, up
// to nq; otherwise thread q takes the trie starting at position q < nq.
__device__ __forceinline__ void enqueue_child(const LevelDev &C, uint32_t s, uint32_t *fq_n, StatusDev *status) {
    if (!CK(s < C.npos)) return;
    if (atomicCAS(&C.st[s], 0u, kQueued) == 0u) {
        const uint32_t pos = atomicAdd(fq_n, 1u);
        if (CK(pos < C.npos)) C.fq[pos] = s;
    }
}

__global__ void __launch_bounds__(256) k_enqueue_children(LevelDev L, LevelDev C, uint32_t nq, int root,
                                                          uint32_t *fq_n, StatusDev *status) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    if (root) {
        const uint32_t st = L.st[0];
        if (st == 0 || st == kQueued || q >= st - 1 || !CK(q < L.npos)) return;
        enqueue_child(C, L.kl[q], fq_n, status);
        return;
    }
    if (!CK(q < L.npos)) return;
    const uint32_t st = L.st[q];
    if (st == 0 || st == kQueued) return;
    const uint32_t keys = st - 1;
    if (!CK((u64)q + keys <= L.npos)) return;
    for (uint32_t r = 0; r < keys; r++) enqueue_child(C, L.kl[q + r], fq_n, status);
}

// ----------------------------------------------------- materialized rows
// A materialized intermediate becomes a column-stored relation: row-major
// rows (n x m) to m columns, one thread per row, stores coalesced per column.
struct RowCols {
    int32_t *col[FJ_MAX_COLS];
};

__global__ void __launch_bounds__(256) k_rows_to_cols(const int32_t *__restrict__ rows, u64 n, int m, RowCols c) {
    const u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t *src = rows + r * (u64)m;
    for (int j = 0; j < m; j++) c.col[j][r] = src[j];
}

// ------------------------------------------------------------- launchers

static inline unsigned blocks_for(u64 n, unsigned t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_fill_u32(uint32_t *p, u64 n, uint32_t v, hipStream_t s) {
    if (!n) return hipSuccess;
    unsigned b = (unsigned)std::min<u64>(blocks_for(n, 256), 65535);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(b), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_list(const FillList *fl_dev, u64 total_words, const LevelDev &root, uint32_t nroot,
                            uint32_t *pre, hipStream_t s) {
    unsigned b = (unsigned)std::min<u64>(std::max<u64>(blocks_for(total_words, 256), 1), 4096);
    hipLaunchKernelGGL(k_fill_list, dim3(b), dim3(256), 0, s, fl_dev, root, nroot, pre);
    return hipGetLastError();
}

template <typename T>
static hipError_t scan_impl(const T *in, T *out, u64 n, T *bsum, T *total, hipStream_t s) {
    // out has n + 1 entries; out[n] = total; bsum needs ceil(n / kScanTile) + 1 entries
    u64 nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        hipLaunchKernelGGL(k_fill<T>, dim3(1), dim3(64), 0, s, out, (u64)1, (T)0);
        hipLaunchKernelGGL(k_fill<T>, dim3(1), dim3(64), 0, s, total, (u64)1, (T)0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_blocks<T>, dim3(1), dim3(kScanThreads), 0, s, bsum, nb, total, out + n);
    hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n,
                       (const T *)bsum);
    return hipGetLastError();
}

hipError_t launch_scan_u64(const u64 *in, u64 *out, u64 n, u64 *bsum, u64 *total, hipStream_t s) {
    return scan_impl<u64>(in, out, n, bsum, total, s);
}
hipError_t launch_scan_u32(const uint32_t *in, uint32_t *out, u64 n, uint32_t *bsum, uint32_t *total,
                           hipStream_t s) {
    return scan_impl<uint32_t>(in, out, n, bsum, total, s);
}

u64 filter_lt_blocks(u64 n) { return std::max<u64>((n + kFilterBlock - 1) / kFilterBlock, 1); }

hipError_t launch_filter_lt(const int32_t *col, u64 n, int32_t bound, uint32_t *out, uint32_t *bsum,
                            uint32_t *total, hipStream_t s) {
    const u64 nb = filter_lt_blocks(n);
    const int vec = ((uintptr_t)col % 16) == 0;
    hipLaunchKernelGGL(k_filter_count, dim3((unsigned)nb), dim3(256), 0, s, col, n, bound, vec, bsum);
    hipLaunchKernelGGL(k_scan_blocks<uint32_t>, dim3(1), dim3(kScanThreads), 0, s, bsum, nb, total,
                       (uint32_t *)nullptr);
    hipLaunchKernelGGL(k_filter_write, dim3((unsigned)nb), dim3(256), 0, s, col, n, bound, vec, (const uint32_t *)bsum,
                       out);
    return hipGetLastError();
}

hipError_t launch_filter_lt_group(int n, const int32_t *const *cols, const u64 *rows, const int32_t *bounds,
                                  uint32_t *const *outs, uint32_t *const *bsums, uint32_t *const *totals,
                                  hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n > FJ_MAX_ATOMS) return hipErrorInvalidValue;
    FilterGroup g;
    memset(&g, 0, sizeof(g));
    g.n = n;
    u64 nb = 0;
    for (int i = 0; i < n; i++) {
        g.col[i] = cols[i];
        g.rows[i] = rows[i];
        g.bound[i] = bounds[i];
        g.vec[i] = ((uintptr_t)cols[i] % 16) == 0;
        g.out[i] = outs[i];
        g.bsum[i] = bsums[i];
        g.total[i] = totals[i];
        g.bpre[i] = (uint32_t)nb;
        nb += std::max<u64>((rows[i] + kFilterGroupBlock - 1) / kFilterGroupBlock, 1);
    }
    if (nb > 0x7fffffffu) return hipErrorInvalidValue;
    g.bpre[n] = (uint32_t)nb;
    hipLaunchKernelGGL(k_filter_count_group, dim3((unsigned)nb), dim3(256), 0, s, g);
    hipLaunchKernelGGL(k_filter_write_group, dim3((unsigned)nb), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_enqueue_children(const LevelDev &L, const LevelDev &C, uint32_t nq, int root, uint32_t *fq_n,
                                   StatusDev *st, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    hipLaunchKernelGGL(k_enqueue_children, dim3(blocks_for(nq, 256)), dim3(256), 0, s, L, C, nq, root, fq_n, st);
    return hipGetLastError();
}

hipError_t launch_rows_to_cols(const int32_t *rows, u64 n, int m, int32_t *const *cols, hipStream_t s) {
    if (m < 1 || m > FJ_MAX_COLS) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    RowCols c;
    memset(&c, 0, sizeof(c));
    for (int j = 0; j < m; j++) c.col[j] = cols[j];
    hipLaunchKernelGGL(k_rows_to_cols, dim3(blocks_for(n, 256)), dim3(256), 0, s, rows, n, m, c);
    return hipGetLastError();
}

hipError_t launch_fq_lens(const LevelDev &L, const uint32_t *fq, uint32_t nh, uint32_t *lens, StatusDev *st,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_fq_lens, dim3(blocks_for(nh, 256)), dim3(256), 0, s, L, fq, nh, lens, st);
    return hipGetLastError();
}

hipError_t launch_force_phase(int phase, const ForceLaunch &f, hipStream_t s) {
    ForceArgs a;
    a.L = f.L; a.C = f.C;
    for (int c = 0; c < FJ_MAX_COLS; c++) a.cols[c] = f.cols[c];
    a.fq = f.fq; a.nh = f.nh; a.pre = f.pre; a.W = f.W;
    a.wslot = f.wslot; a.cntv = f.cntv; a.ex = f.ex;
    a.wcap = f.wcap; a.status = f.status;
    dim3 g(blocks_for(f.W, 256)), b(256);
    if (f.W == 0) return hipSuccess;
    switch (phase) {
        case 0: hipLaunchKernelGGL(k_force_insert, g, b, 0, s, a); break;
        case 1: hipLaunchKernelGGL(k_force_pack, g, b, 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_force_children, g, b, 0, s, a); break;
        case 3: hipLaunchKernelGGL(k_force_scatter, g, b, 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_group_fill(const FillBlock *fb, uint32_t nblocks, const GroupRoot *roots, int n, hipStream_t s) {
    const uint32_t g = nblocks + (uint32_t)((n + 255) / 256);
    if (g) hipLaunchKernelGGL(k_group_fill, dim3(g), dim3(256), 0, s, fb, nblocks, roots, n);
    return hipGetLastError();
}

hipError_t launch_group_force(int phase, const ForceArgs *descs, const u64 *wpre, int n, u64 wtot, hipStream_t s) {
    if (wtot == 0) return hipSuccess;
    dim3 g((unsigned)((wtot + 255) / 256)), b(256);
    switch (phase) {
        case 0: hipLaunchKernelGGL(k_group_force<0>, g, b, 0, s, descs, wpre, n, wtot); break;
        case 1: hipLaunchKernelGGL(k_group_force<1>, g, b, 0, s, descs, wpre, n, wtot); break;
        case 2: hipLaunchKernelGGL(k_group_force<2>, g, b, 0, s, descs, wpre, n, wtot); break;
        case 3: hipLaunchKernelGGL(k_group_force<3>, g, b, 0, s, descs, wpre, n, wtot); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Exclusive scan of n u32 values by one workgroup (n up to a few hundred
// thousand; for the grouped builds' per-range counts), out[n] = total.
__global__ void __launch_bounds__(1024) k_scan_small_u32(const uint32_t *in, uint32_t *out, uint32_t n) {
    __shared__ uint32_t lds[17];
    uint32_t carry = 0;
    for (uint32_t c = 0; c < n; c += 1024 * 4) {
        uint32_t v[4], sum = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t i = c + threadIdx.x * 4 + j;
            v[j] = i < n ? in[i] : 0u;
            sum += v[j];
        }
        uint32_t tot;
        uint32_t ex = carry + block_excl_scan<uint32_t>(sum, lds, tot);
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t i = c + threadIdx.x * 4 + j;
            if (i < n) out[i] = ex;
            ex += v[j];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) out[n] = carry;
}

hipError_t launch_scan_small_u32(const uint32_t *in, uint32_t *out, uint32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_small_u32, dim3(1), dim3(1024), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_part_phase(int phase, const PartArgs &a, hipStream_t s) {
    if (a.n <= 0 || a.nparts == 0) return hipSuccess;
    switch (phase) {
        case 0:
            if (a.nblocks || a.nroots > 0)
                hipLaunchKernelGGL(k_part_place, dim3(a.nblocks + (unsigned)(std::max(a.nroots, 0) + 255) / 256),
                                   dim3(256), 0, s, a);
            break;
        case 1: hipLaunchKernelGGL(k_part_build, dim3(a.nparts), dim3(kPartBuildThreads), 0, s, a); break;
        case 2: hipLaunchKernelGGL(k_part_ranks, dim3(a.nparts), dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_cover_choose(const NodeDev *nd, uint32_t E, uint8_t *cov, u64 *cnt, StatusDev *st, hipStream_t s) {
    hipLaunchKernelGGL(k_cover_choose, dim3(blocks_for(E, 256)), dim3(256), 0, s, nd, E, cov, cnt, st);
    return hipGetLastError();
}

hipError_t launch_cover_fill(const NodeDev *nd, uint32_t E, const uint8_t *cov, u64 *cnt, StatusDev *st,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_cover_fill, dim3(blocks_for(E, 256)), dim3(256), 0, s, nd, E, cov, cnt, st);
    return hipGetLastError();
}

hipError_t launch_probe(const ProbeLaunch &p, hipStream_t s) {
    ProbeArgs a;
    a.nd = p.nd; a.starts = p.starts; a.cov = p.cov; a.E = p.E; a.t0 = p.t0; a.n = p.n;
    a.din = p.din; a.din_j = p.din_j; a.dout = p.dout; a.dout_j = p.dout_j;
    a.status = p.status; a.count_stats = p.count_stats; a.dcap = p.dcap;
    a.surv_base = p.surv_base; a.def_base = p.def_base;
    a.chunk_e = nullptr;
    if (p.n == 0) return hipSuccess;
    int bs = p.block > 0 ? p.block : 256;
    const uint32_t nb = blocks_for(p.n, bs);
    if (!p.din && p.chunk_buf && p.chunk_cap >= (u64)nb + 1) {
        hipLaunchKernelGGL(k_chunk_entries, dim3((nb + 1 + 255) / 256), dim3(256), 0, s, p.starts, p.E, p.t0, p.n,
                           (uint32_t)bs, nb, p.chunk_buf);
        a.chunk_e = p.chunk_buf;
    }
    // the smallest instantiation whose bounds hold the query's slots and atoms
    if (p.max_slots <= 8 && p.max_atoms <= 8) hipLaunchKernelGGL((k_probe<8, 8>), dim3(nb), dim3(bs), 0, s, a);
    else if (p.max_slots <= 16 && p.max_atoms <= 16) hipLaunchKernelGGL((k_probe<16, 16>), dim3(nb), dim3(bs), 0, s, a);
    else hipLaunchKernelGGL((k_probe<FJ_MAX_VARS, FJ_MAX_ATOMS>), dim3(nb), dim3(bs), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_emit_count_small(const void *emit_dev, uint32_t E, u64 *starts, StatusDev *st, u64 cap,
                                   hipStream_t s) {
    if (E == 0 || E > kEmitSmall) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_emit_count_small, dim3(1), dim3(kEmitSmallThreads), 0, s, (const EmitDev *)emit_dev, E,
                       starts, st, cap);
    return hipGetLastError();
}

uint32_t emit_small_max() { return kEmitSmall; }

hipError_t launch_emit_small_dev(const void *emit_dev, const u64 *surv, u64 surv_base, u64 *starts, StatusDev *st,
                                 u64 cap, hipStream_t s) {
    hipLaunchKernelGGL(k_emit_small_dev, dim3(1), dim3(kEmitSmallThreads), 0, s, (const EmitDev *)emit_dev, surv,
                       surv_base, starts, st, cap);
    return hipGetLastError();
}

hipError_t launch_emit_count(const void *emit_dev, uint32_t E, u64 *cnt, StatusDev *st, hipStream_t s) {
    hipLaunchKernelGGL(k_emit_count, dim3(blocks_for(E, 256)), dim3(256), 0, s, (const EmitDev *)emit_dev, E, cnt,
                       st);
    return hipGetLastError();
}

hipError_t launch_emit_rows(const void *emit_dev, uint32_t E, const u64 *starts, u64 max_rows, StatusDev *st,
                            hipStream_t s) {
    if (!max_rows) return hipSuccess;
    const unsigned grid = (unsigned)std::min<u64>(blocks_for(max_rows, 256), 2048);
    hipLaunchKernelGGL(k_emit_rows, dim3(grid), dim3(256), 0, s, (const EmitDev *)emit_dev, E, starts, st);
    return hipGetLastError();
}

hipError_t launch_emit_range(const void *emit_dev, uint32_t E, const u64 *starts, u64 first, u64 n, StatusDev *st,
                             hipStream_t s) {
    if (!n) return hipSuccess;
    const unsigned grid = (unsigned)std::min<u64>(blocks_for(n, 256), 4096);
    hipLaunchKernelGGL(k_emit_range, dim3(grid), dim3(256), 0, s, (const EmitDev *)emit_dev, E, starts, first, n, st);
    return hipGetLastError();
}

hipError_t launch_scan_u64_emit(const u64 *in, u64 *out, u64 n, u64 *bsum, StatusDev *st, u64 cap, hipStream_t s) {
    if (n == 0) return hipErrorInvalidValue;
    const u64 nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_reduce<u64>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_blocks_emit, dim3(1), dim3(kScanThreads), 0, s, bsum, nb, out + n, st, cap);
    hipLaunchKernelGGL(k_scan_apply<u64>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n,
                       (const u64 *)bsum);
    return hipGetLastError();
}

hipError_t launch_scan_probe(const ScanLaunch &l, hipStream_t s) {
    if (l.nl > kScanMaxLookups) return hipErrorInvalidValue;
    if (l.n == 0) return hipSuccess;
    if (l.nrows == 0) return hipErrorInvalidValue;   // positions into an empty relation
    ScanArgs a;
    memset(&a, 0, sizeof(a));
    for (int c = 0; c < FJ_MAX_COLS; c++) a.cols[c] = l.cols[c];
    a.ncols = l.ncols; a.sel = l.sel; a.nrows = l.nrows; a.r0 = l.r0; a.n = l.n;
    // without a selection, positions are rows: they must exist
    if (!l.sel && (u64)l.r0 + l.n > l.nrows) return hipErrorInvalidValue;
    // 4-row vector loads: rows in bounds (no selection), 16-byte aligned
    // columns and a 4-aligned start
    a.vec = !l.sel && (l.r0 % 4) == 0;
    for (int c = 0; c < l.ncols; c++) a.vec = a.vec && ((uintptr_t)l.cols[c] % 16) == 0;
    a.nl = l.nl;
    for (int j = 0; j < l.nl; j++) {
        // KM_K32 hits are kept as 32-bit slot numbers
        if (l.lk[j].mode == KM_K32 && l.lk[j].mask >= 0xFFFFFFFFull) return hipErrorInvalidValue;
        a.lk[j] = l.lk[j];
    }
    a.nout = l.nout;
    for (int j = 0; j < l.nout; j++) a.out_col[j] = l.out_col[j];
    a.out = l.out; a.emit = l.emit; a.materialize = l.materialize;
    a.ntail = l.ntail;
    for (int q = 0; q < l.ntail; q++) {
        a.tail_lk[q] = l.tail_lk[q]; a.tail_len[q] = l.tail_len[q];
        a.tail_npos[q] = l.tail_npos[q]; a.tail_root_len[q] = l.tail_root_len[q];
    }
    a.status = l.status; a.count_stats = l.count_stats; a.node = l.node; a.surv_base = l.surv_base;
    if (l.direct && (!l.ed || !l.emit || l.materialize)) return hipErrorInvalidValue;
    a.direct = l.direct; a.ed = (const EmitDev *)l.ed; a.cap = l.cap;
    // persistent workgroups: as many as are resident at once, at most one
    // per tile
    constexpr int kMaxDevices = 64;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    const size_t lds = (size_t)l.nl * kBatch * sizeof(uint32_t);
    const void *fn = l.count_stats ? (const void *)k_scan_probe<true> : (const void *)k_scan_probe<false>;
    static int resident[2][kScanMaxLookups + 1][kMaxDevices];   // 0: not known yet
    int &res = resident[l.count_stats ? 1 : 0][l.nl][dev];
    if (res == 0) {
        int per_cu = 0, cus = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds);
        if (e != hipSuccess) return e;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        res = std::max(1, per_cu) * std::max(1, cus);
    }
    const ScanLookup &L0 = l.lk[0];
    if (l.nl >= 1 && L0.bloom && L0.mode == KM_K32 && l.l0_row && l.l0_key && l.l0_cnt &&
        scan_list_entries(l.n) <= l.l0_cap) {
        // the filter must be the map's: one word per 2^shift buckets
        if (L0.bloom_words < 4 || L0.bloom_words % 4 || L0.bloom_words > kBloomWords || L0.bloom_shift > 30 ||
            ((L0.mask + 1) >> (2 + L0.bloom_shift)) != L0.bloom_words)
            return hipErrorInvalidValue;
        const void *ffn = l.count_stats ? (const void *)k_scan_filter<true> : (const void *)k_scan_filter<false>;
        static int fres[2][kMaxDevices];   // 0: not known yet; -1: not launchable
        int &fr = fres[l.count_stats ? 1 : 0][dev];
        if (fr == 0) {
            int per_cu = 0, cus = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ffn, kFiltThreads, 0);
            if (e != hipSuccess) return e;
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) return e;
            fr = per_cu >= 1 ? per_cu * std::max(1, cus) : -1;
        }
        if (fr > 0) {
            const u64 ftiles = blocks_for(l.n, kFiltTile);
            const unsigned G = (unsigned)std::min<u64>(std::min<u64>(ftiles, (u64)fr), kScanListGroups);
            a.l0_row = l.l0_row;
            a.l0_key = l.l0_key;
            a.l0_cnt = l.l0_cnt;
            a.l0_groups = G;
            // the rounds pass: as many workgroups as are resident, each
            // taking l0_per consecutive regions
            const u64 items = (u64)G * kFiltWaves;
            a.l0_per = (uint32_t)std::min<u64>((items + res - 1) / res, kListPerMax);
            if (l.count_stats)
                hipExtLaunchKernelGGL(k_scan_filter<true>, dim3(G), dim3(kFiltThreads), 0, s, l.t_start, nullptr, 0, a);
            else
                hipExtLaunchKernelGGL(k_scan_filter<false>, dim3(G), dim3(kFiltThreads), 0, s, l.t_start, nullptr, 0, a);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            const unsigned grid = (unsigned)((items + a.l0_per - 1) / a.l0_per);
            if (l.count_stats)
                hipExtLaunchKernelGGL(k_scan_rounds<true>, dim3(grid), dim3(256), (uint32_t)lds, s, nullptr, l.t_stop, 0, a);
            else
                hipExtLaunchKernelGGL(k_scan_rounds<false>, dim3(grid), dim3(256), (uint32_t)lds, s, nullptr, l.t_stop, 0, a);
            return hipGetLastError();
        }
    }
    const unsigned grid = (unsigned)std::min<u64>(blocks_for(l.n, kTile), (u64)res);
    if (l.count_stats)
        hipExtLaunchKernelGGL(k_scan_probe<true>, dim3(grid), dim3(256), (uint32_t)lds, s, l.t_start, l.t_stop, 0, a);
    else
        hipExtLaunchKernelGGL(k_scan_probe<false>, dim3(grid), dim3(256), (uint32_t)lds, s, l.t_start, l.t_stop, 0, a);
    return hipGetLastError();
}

int scan_max_lookups() { return kScanMaxLookups; }

unsigned long long scan_list_entries(unsigned long long n) { return blocks_for(n, kFiltTile) * (u64)kFiltTile; }

size_t emit_dev_size() { return sizeof(EmitDev); }

void emit_dev_fill(void *host_buf, const FrontierDev &F, const int *in_var, int nin, const int *in_h_atom,
                   int nin_h, const TailDev *tails, int ntail, const int *head_src, int nhead, int32_t *out,
                   u64 out_rows) {
    EmitDev *d = (EmitDev *)host_buf;
    memset(d, 0, sizeof(EmitDev));
    d->F = F;
    d->nin = nin;
    for (int j = 0; j < d->nin; j++) d->in_var[j] = in_var[j];
    d->nin_h = nin_h;
    for (int j = 0; j < d->nin_h; j++) d->in_h_atom[j] = in_h_atom[j];
    d->ntail = ntail;
    for (int q = 0; q < ntail; q++) d->tail[q] = tails[q];
    d->nhead = nhead;
    for (int j = 0; j < nhead; j++) d->head_src[j] = head_src[j];
    d->out = out;
    d->out_rows = out_rows;
}

}  // namespace fj
