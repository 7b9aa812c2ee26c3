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
    int32_t v[FJ_MAX_COLS];
};

// Probing walks forward from the start of a 32-byte bucket (4 slots of 8 B,
// or 2 of 16 B), so that one pair of 16-byte loads usually settles a lookup.
// Insert and find use the same sequence.
#ifndef FJ_BUCKET_BYTES
#define FJ_BUCKET_BYTES 32
#endif
constexpr int kBucketBytes = FJ_BUCKET_BYTES;
template <typename SlotT> __device__ __forceinline__ u64 bucket_start(u64 h, u64 mask) {
    return (h & mask) & ~(u64)(kBucketBytes / sizeof(SlotT) - 1);
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
        const Slot32 *T = (const Slot32 *)L.table;
        uint32_t key = (uint32_t)k.v[0];
        if (key == kEmpty32) return T[mask + 1].key ? mask + 1 : ~0ull;
        u64 i = bucket_start<Slot32>(mix32(key), mask);
        for (u64 n = 0; n <= mask; n++) {
            uint32_t c = T[i].key;
            if (c == key) return i;
            if (c == kEmpty32) return ~0ull;
            i = (i + 1) & mask;
        }
    } else if (L.mode == KM_K64) {
        const Slot64 *T = (const Slot64 *)L.table;
        u64 key = pack64(L, k);
        if (key == kEmpty64) return T[mask + 1].key ? mask + 1 : ~0ull;
        u64 i = bucket_start<Slot64>(mix64(key), mask);
        for (u64 n = 0; n <= mask; n++) {
            u64 c = T[i].key;
            if (c == key) return i;
            if (c == kEmpty64) return ~0ull;
            i = (i + 1) & mask;
        }
    } else {
        const SlotRep *T = (const SlotRep *)L.table;
        u64 i = bucket_start<SlotRep>(rep_hash(k, L.nk), mask);
        for (u64 n = 0; n <= mask; n++) {
            u64 c = T[i].hr;
            if (c == kEmpty64) return ~0ull;
            if ((uint32_t)c == k.h && (uint32_t)(c >> 32) < L.nrows &&
                rep_equal(L, cols, (uint32_t)(c >> 32), k)) return i;
            i = (i + 1) & mask;
        }
    }
    return L.nslots;  // no empty slot: the map is corrupt (callers check the index)
}

__device__ __forceinline__ uint32_t slot_val(const LevelDev &L, u64 i) {
    if (L.mode == KM_K32) return ((const Slot32 *)L.table)[i].val;
    if (L.mode == KM_K64) return ((const Slot64 *)L.table)[i].val;
    return ((const SlotRep *)L.table)[i].val;
}

__device__ __forceinline__ void set_slot_val(const LevelDev &L, u64 i, uint32_t v) {
    if (L.mode == KM_K32) ((Slot32 *)L.table)[i].val = v;
    else if (L.mode == KM_K64) ((Slot64 *)L.table)[i].val = v;
    else ((SlotRep *)L.table)[i].val = v;
}

__device__ __forceinline__ uint32_t *slot_val_ptr(const LevelDev &L, u64 i) {
    if (L.mode == KM_K32) return &((Slot32 *)L.table)[i].val;
    if (L.mode == KM_K64) return &((Slot64 *)L.table)[i].val;
    return &((SlotRep *)L.table)[i].val;
}

// Insert-or-find for force(); `row` is the representative row for KM_REP.
__device__ __forceinline__ u64 table_insert(const LevelDev &L, const int32_t *const *cols, const Key &k,
                                            uint32_t row, bool &claimed) {
    const u64 mask = L.mask;
    claimed = false;
    if (L.mode == KM_K32) {
        Slot32 *T = (Slot32 *)L.table;
        uint32_t key = (uint32_t)k.v[0];
        if (key == kEmpty32) {
            claimed = atomicCAS(&T[mask + 1].key, 0u, 1u) == 0u;
            return mask + 1;
        }
        u64 i = bucket_start<Slot32>(mix32(key), mask);
        for (u64 n = 0; n <= mask; n++) {
            // the compare-and-swap returns the occupant: no separate read
            const uint32_t old = atomicCAS(&T[i].key, kEmpty32, key);
            if (old == kEmpty32) { claimed = true; return i; }
            if (old == key) return i;
            i = (i + 1) & mask;
        }
    } else if (L.mode == KM_K64) {
        Slot64 *T = (Slot64 *)L.table;
        u64 key = pack64(L, k);
        if (key == kEmpty64) {
            claimed = atomicCAS(&T[mask + 1].key, 0ull, 1ull) == 0ull;
            return mask + 1;
        }
        u64 i = bucket_start<Slot64>(mix64(key), mask);
        for (u64 n = 0; n <= mask; n++) {
            const u64 old = atomicCAS(&T[i].key, kEmpty64, key);
            if (old == kEmpty64) { claimed = true; return i; }
            if (old == key) return i;
            i = (i + 1) & mask;
        }
    } else {
        SlotRep *T = (SlotRep *)L.table;
        u64 mine = ((u64)row << 32) | k.h;
        u64 i = bucket_start<SlotRep>(rep_hash(k, L.nk), mask);
        for (u64 n = 0; n <= mask; n++) {
            u64 c = T[i].hr;         // may be stale-empty; the CAS settles it
            if (c == kEmpty64) {
                u64 old = atomicCAS(&T[i].hr, kEmpty64, mine);
                if (old == kEmpty64) { claimed = true; return i; }
                c = old;
            }
            if ((uint32_t)c == k.h && (uint32_t)(c >> 32) < L.nrows &&
                rep_equal(L, cols, (uint32_t)(c >> 32), k)) return i;
            i = (i + 1) & mask;
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

__global__ void k_table_init(void *table, u64 nslots, int mode) {
    // all slots empty; the reserved last slot starts at 0 (unclaimed)
    u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    u64 stride = (u64)gridDim.x * blockDim.x;
    for (; i < nslots; i += stride) {
        bool last = (i + 1 == nslots);
        if (mode == KM_K32) {
            Slot32 s; s.key = last ? 0u : kEmpty32; s.val = 0; ((Slot32 *)table)[i] = s;
        } else if (mode == KM_K64) {
            Slot64 s; s.key = last ? 0ull : kEmpty64; s.val = 0; s.pad = 0; ((Slot64 *)table)[i] = s;
        } else {
            SlotRep s; s.hr = kEmpty64; s.val = 0; s.pad = 0; ((SlotRep *)table)[i] = s;
        }
    }
}

// Fill a list of regions with periodic 32-bit patterns (table slots, zeroed
// state arrays) in one launch; also set the root handle and the one-handle
// force queue of the root.
__global__ void k_fill_list(const FillList *__restrict__ fl, LevelDev root, uint32_t nroot, uint32_t *pre) {
    const u64 stride = (u64)gridDim.x * blockDim.x;
    const u64 tid = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    for (int k = 0; k < fl->n; k++) {
        const FillRegion &r = fl->r[k];
        const u64 m = (u64)r.period - 1;   // periods are 1, 2 or 4
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

__device__ __forceinline__ uint32_t filter_bits(const int32_t *col, u64 n, int32_t bound, u64 first, bool vec) {
    uint32_t bits = 0;
    if (vec && first + kFilterRows <= n) {
        const int4 x = *(const int4 *)(col + first);
        bits = (uint32_t)(x.x < bound) | ((uint32_t)(x.y < bound) << 1) | ((uint32_t)(x.z < bound) << 2) |
               ((uint32_t)(x.w < bound) << 3);
    } else {
        for (int r = 0; r < kFilterRows; r++)
            if (first + r < n && col[first + r] < bound) bits |= 1u << r;
    }
    return bits;
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
    k.v[0] = k.v[1] = 0;
    if (todo)
        for (int c = 0; c < a.L.nk; c++) k.v[c] = a.cols[a.L.kcol[c]][row];
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
__global__ void __launch_bounds__(256) k_group_fill(const FillBlock *__restrict__ fb) {
    const FillBlock &b = fb[blockIdx.x];
    const u64 m = (u64)b.period - 1;
    uint32_t *p = b.p + b.start;
    const u64 n4 = b.n >> 2;
    const uint4 v = make_uint4(b.pat[0], b.pat[1 & m], b.pat[2 & m], b.pat[3 & m]);
    for (u64 i = threadIdx.x; i < n4; i += 256) ((uint4 *)p)[i] = v;
    for (u64 i = (n4 << 2) + threadIdx.x; i < b.n; i += 256) p[i] = b.pat[(b.start + i) & m];
}

// Per COLT: the root handle spans every root row; a built root with no rows
// is forced with no keys; the root's force queue holds the root handle.
__global__ void k_group_roots(const GroupRoot *__restrict__ r, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const GroupRoot &g = r[k];
    g.len[0] = g.nroot;
    g.st[0] = (g.built && g.nroot == 0) ? 1u : 0u;
    if (g.fq) g.fq[0] = 0;
    if (g.pre) { g.pre[0] = 0; g.pre[1] = g.nroot; }
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
template <int MV, int MA>
__global__ void __launch_bounds__(256) k_probe(ProbeArgs a) {
    __shared__ u64 red[17];
    const NodeDev &nd = *a.nd;
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
    bool ok = idx < a.n;
    if (ok) {
        if (a.din) { t = a.din[idx]; resume = a.din_j[idx]; } else { t = idx; }
        const u64 g = a.t0 + t;
        uint32_t lo = 0, hi = a.E;
        if (!a.din && a.chunk_e) {
            lo = a.chunk_e[blockIdx.x];
            hi = a.chunk_e[blockIdx.x + 1] + 1;
            ok = CK(lo < hi && hi <= a.E);
        }
        e = (!ok || a.E == 1) ? 0u : upper_entry(a.starts, lo, hi, g);
        ok = ok && CK(e < a.E && e < nd.in.cap && g >= a.starts[e] && g < a.starts[e + 1]);
    }
    if (ok) {
        const u64 i = a.t0 + t - a.starts[e];
        const FrontierDev &F = nd.in;
        for (int j = 0; j < nd.nin; j++) v[(j) & (MV - 1)] = F.vals[(u64)j * F.cap + e];
        for (int j = 0; j < nd.nin_h; j++) h[(nd.in_h_atom[j]) & (MA - 1)] = F.hdl[(u64)j * F.cap + e];
        mult = F.mult ? F.mult[e] : 1ull;
        // bind the cover tuple
        const uint8_t cb = a.cov[e];
        const int ci = cb & 0x7F;
        const SubDev &S = nd.sub[ci];
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
            const SubDev &P = nd.sub[j];
            const uint32_t ph = P.level == 0 ? 0u : h[(P.atom) & (MA - 1)];
            if (!CK(ph < P.L.npos)) { survive = false; break; }
            const uint32_t st = P.L.st[ph];
            if (st == 0 || st == kQueued) {
                if (!CK(P.level > 0)) { survive = false; break; }
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

// ------------------------------------------------------------ scan probe
// Specialised first node: the cover is a base table (or its selection)
// iterated directly and every other subatom is a probe of a root map keyed
// by cover columns.  Each thread takes kScanRows rows of a contiguous tile
// (coalesced, non-temporal column loads) and probes trie by trie across its
// rows, so the rows' independent probes are in flight together: the
// vectorized execution of Section 4.3 mapped onto one thread's registers.

#ifndef FJ_SCAN_ROWS
#define FJ_SCAN_ROWS 1
#endif
constexpr int kScanRows = FJ_SCAN_ROWS;
#ifndef FJ_SCAN_SPEC
#define FJ_SCAN_SPEC 1
#endif
constexpr int kScanSpec = FJ_SCAN_SPEC;   // lookups whose bucket loads are in flight together
constexpr int kScanMaxLookups = 8;

// Streaming loads of cover columns (read once).
__device__ __forceinline__ int32_t stream_load(const int32_t *p) {
#ifdef FJ_NT_LOADS
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

struct ScanArgs {
    const int32_t *cols[FJ_MAX_COLS];
    int ncols;
    int vec;                  // cover columns are 16-byte aligned: load 4 rows at once
    int keycol[FJ_MAX_COLS];  // nonzero for columns some lookup keys on
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
};

// Bucket of a root map, held as 16-byte vector registers.
constexpr int kBucketVec = kBucketBytes / 16;
struct Bucket { uint4 q[kBucketVec]; };

__device__ __forceinline__ void load_bucket(const void *T, u64 byte_off, Bucket &out) {
    const uint4 *src = (const uint4 *)((const char *)T + byte_off);
#pragma unroll
    for (int q = 0; q < kBucketVec; q++) out.q[q] = src[q];
}

// Scan a loaded bucket in slot order: 1 = hit, 2 = miss (empty slot), 0 = go
// on.  Branch-free: walking the slots backwards, the earliest slot that holds
// the key or is empty decides.
__device__ __forceinline__ int scan_bucket32(const Bucket &bk, uint32_t key, uint32_t &val) {
    int st = 0;
    uint32_t v = 0;
#pragma unroll
    for (int q = kBucketVec - 1; q >= 0; q--) {
        const uint32_t kz = bk.q[q].z, kx = bk.q[q].x;
        st = kz == key ? 1 : (kz == kEmpty32 ? 2 : st);
        v = kz == key ? bk.q[q].w : v;
        st = kx == key ? 1 : (kx == kEmpty32 ? 2 : st);
        v = kx == key ? bk.q[q].y : v;
    }
    val = v;
    return st;
}

__device__ __forceinline__ int scan_bucket64(const Bucket &bk, u64 key, uint32_t &val) {
    int st = 0;
    uint32_t v = 0;
#pragma unroll
    for (int q = kBucketVec - 1; q >= 0; q--) {
        const u64 k = ((u64)bk.q[q].y << 32) | bk.q[q].x;
        st = k == key ? 1 : (k == kEmpty64 ? 2 : st);
        v = k == key ? bk.q[q].z : v;
    }
    val = v;
    return st;
}

// One round of root-map probes for kScanRows rows: every row's bucket load
// is issued before any is examined.  Keys equal to the empty marker live in
// the reserved slot (mask + 1), whose key word is 1 once claimed.
template <int MODE>
__device__ __forceinline__ void scan_round(const ScanArgs &a, const ScanLookup &L, const uint32_t *row,
                                           bool *alive, bool vec, uint32_t *val) {
    typedef typename std::conditional<MODE == KM_K32, Slot32, Slot64>::type SlotT;
    typedef typename std::conditional<MODE == KM_K32, uint32_t, u64>::type KeyT;
    constexpr u64 B = kBucketBytes / sizeof(SlotT);
    const SlotT *T = (const SlotT *)L.table;
    const KeyT empty = MODE == KM_K32 ? (KeyT)kEmpty32 : (KeyT)kEmpty64;
    const int32_t *c0 = a.cols[L.kc[0]];
    const int32_t *c1 = a.cols[MODE == KM_K32 ? L.kc[0] : L.kc[1]];
    int32_t k0[kScanRows], k1[kScanRows];
    // keys: one 16-byte load per column when the thread's rows are
    // consecutive and all alive, else one load per live row
    bool all = vec;
#pragma unroll
    for (int r = 0; r < kScanRows; r++) all = all && alive[r];
    if constexpr (kScanRows == 4) {
        if (all) {
            const int4 x = *(const int4 *)(c0 + row[0]);
            k0[0] = x.x; k0[1] = x.y; k0[2] = x.z; k0[3] = x.w;
            if (MODE != KM_K32) {
                const int4 y = *(const int4 *)(c1 + row[0]);
                k1[0] = y.x; k1[1] = y.y; k1[2] = y.z; k1[3] = y.w;
            }
        }
    }
    if (!all || kScanRows != 4) {
#pragma unroll
        for (int r = 0; r < kScanRows; r++) {
            k0[r] = alive[r] ? c0[row[r]] : 0;
            if (MODE != KM_K32) k1[r] = alive[r] ? c1[row[r]] : 0;
        }
    }
    KeyT key[kScanRows];
    u64 idx[kScanRows];
    Bucket bk[kScanRows];
#pragma unroll
    for (int r = 0; r < kScanRows; r++) {
#pragma unroll
        for (int q = 0; q < kBucketVec; q++) bk[r].q[q] = make_uint4(0, 0, 0, 0);
        key[r] = MODE == KM_K32 ? (KeyT)(uint32_t)k0[r]
                                : (KeyT)((((u64)(uint32_t)k0[r]) << 32) | (uint32_t)k1[r]);
        const u64 h = MODE == KM_K32 ? (u64)mix32((uint32_t)key[r]) : mix64((u64)key[r]);
        idx[r] = bucket_start<SlotT>(h, L.mask);
        if (alive[r] && key[r] != empty) load_bucket(T, idx[r] * sizeof(SlotT), bk[r]);
    }
#pragma unroll
    for (int r = 0; r < kScanRows; r++) {
        if (!alive[r]) continue;
        if (key[r] == empty) {
            const SlotT rs = T[L.mask + 1];
            alive[r] = rs.key != 0;
            val[r] = rs.val;
            continue;
        }
        int st = MODE == KM_K32 ? scan_bucket32(bk[r], (uint32_t)key[r], val[r])
                                : scan_bucket64(bk[r], (u64)key[r], val[r]);
        for (u64 n = B; st == 0 && n <= L.mask; n += B) {   // a full bucket: go on (rare)
            idx[r] = (idx[r] + B) & L.mask;
            load_bucket(T, idx[r] * sizeof(SlotT), bk[r]);
            st = MODE == KM_K32 ? scan_bucket32(bk[r], (uint32_t)key[r], val[r])
                                : scan_bucket64(bk[r], (u64)key[r], val[r]);
        }
        alive[r] = st == 1;
    }
}

// One row, one lookup, in two steps: issue() computes the bucket and starts
// its load; resolve() scans it (and walks on in the rare full bucket).  A
// thread issues the loads of two lookups before resolving the first, since
// a bucket's address depends only on the row's key columns.
struct RowProbe {
    Bucket bk;
    u64 idx;
    u64 key;     // K32: the 32-bit key; K64: the packed pair
    bool empty;  // the key equals the empty marker (reserved slot)
};

__device__ __forceinline__ void probe_issue(const ScanLookup &L, uint32_t k0, uint32_t k1, bool alive,
                                            RowProbe &rp) {
#pragma unroll
    for (int q = 0; q < kBucketVec; q++) rp.bk.q[q] = make_uint4(0, 0, 0, 0);
    if (L.mode == KM_K32) {
        rp.key = k0;
        rp.empty = k0 == kEmpty32;
        rp.idx = bucket_start<Slot32>(mix32(k0), L.mask);
        if (alive && !rp.empty) load_bucket(L.table, rp.idx * sizeof(Slot32), rp.bk);
    } else {
        rp.key = ((u64)k0 << 32) | k1;
        rp.empty = rp.key == kEmpty64;
        rp.idx = bucket_start<Slot64>(mix64(rp.key), L.mask);
        if (alive && !rp.empty) load_bucket(L.table, rp.idx * sizeof(Slot64), rp.bk);
    }
}

__device__ __forceinline__ bool probe_resolve(const ScanLookup &L, RowProbe &rp, uint32_t &val) {
    if (L.mode == KM_K32) {
        const Slot32 *T = (const Slot32 *)L.table;
        if (rp.empty) { const Slot32 rs = T[L.mask + 1]; val = rs.val; return rs.key != 0; }
        constexpr u64 B = kBucketBytes / sizeof(Slot32);
        int st = scan_bucket32(rp.bk, (uint32_t)rp.key, val);
        for (u64 n = B; st == 0 && n <= L.mask; n += B) {
            rp.idx = (rp.idx + B) & L.mask;
            load_bucket(T, rp.idx * sizeof(Slot32), rp.bk);
            st = scan_bucket32(rp.bk, (uint32_t)rp.key, val);
        }
        return st == 1;
    }
    const Slot64 *T = (const Slot64 *)L.table;
    if (rp.empty) { const Slot64 rs = T[L.mask + 1]; val = rs.val; return rs.key != 0; }
    constexpr u64 B = kBucketBytes / sizeof(Slot64);
    int st = scan_bucket64(rp.bk, rp.key, val);
    for (u64 n = B; st == 0 && n <= L.mask; n += B) {
        rp.idx = (rp.idx + B) & L.mask;
        load_bucket(T, rp.idx * sizeof(Slot64), rp.bk);
        st = scan_bucket64(rp.bk, rp.key, val);
    }
    return st == 1;
}

template <bool STATS>
__global__ void __launch_bounds__(256) k_scan_probe(ScanArgs a) {
    StatusDev *status = a.status;
    // child handles of the thread's live rows, per lookup
    __shared__ uint32_t hs[kScanMaxLookups][256 * kScanRows];
    const uint32_t first = (blockIdx.x * 256u + threadIdx.x) * kScanRows;
    uint32_t row[kScanRows];
    bool alive[kScanRows];
    u64 mult[kScanRows];
    uint32_t nprobe = 0, nhit = 0;
#pragma unroll
    for (int r = 0; r < kScanRows; r++) {
        alive[r] = first + r < a.n;
        mult[r] = 1;
        row[r] = alive[r] ? a.r0 + first + r : 0u;
    }
    bool vec = a.vec;
    if (a.sel) {
#pragma unroll
        for (int r = 0; r < kScanRows; r++) row[r] = alive[r] ? a.sel[row[r]] : 0u;
        vec = false;
    }
#pragma unroll
    for (int r = 0; r < kScanRows; r++) alive[r] = alive[r] && CK(row[r] < a.nrows);
    if constexpr (kScanRows == 1) {
        // every lookup's key columns first (independent loads), then the
        // lookups in order, kScanSpec bucket loads in flight at a time
        uint32_t k0[kScanMaxLookups], k1[kScanMaxLookups];
#pragma unroll
        for (int j = 0; j < kScanMaxLookups; j++) {
            k0[j] = 0;
            k1[j] = 0;
            if (j < a.nl && alive[0]) {
                const ScanLookup &L = a.lk[j];
                k0[j] = (uint32_t)a.cols[L.kc[0]][row[0]];
                if (L.mode != KM_K32) k1[j] = (uint32_t)a.cols[L.kc[1]][row[0]];
            }
        }
#pragma unroll
        for (int j0 = 0; j0 < kScanMaxLookups; j0 += kScanSpec) {
            if (j0 >= a.nl || !__any(alive[0])) break;
            const bool two = kScanSpec == 2 && j0 + 1 < a.nl;
            RowProbe p0, p1;
            probe_issue(a.lk[j0], k0[j0], k1[j0], alive[0], p0);
            if (two) probe_issue(a.lk[j0 + 1], k0[j0 + 1], k1[j0 + 1], alive[0], p1);
#pragma unroll
            for (int h = 0; h < 2; h++) {
                const int j = j0 + h;
                if (h == 1 && !two) break;
                const ScanLookup &L = a.lk[j];
                if (!alive[0]) continue;
                if (STATS) nprobe++;
                uint32_t v = 0;
                alive[0] = probe_resolve(L, h == 0 ? p0 : p1, v);
                if (!alive[0]) continue;
                if (!CK(v < L.cnpos)) { alive[0] = false; continue; }
                if (STATS) nhit++;
                hs[j][threadIdx.x] = v;
                if (L.child_leaf) mult[0] *= L.clen[v];
            }
        }
    }
    // trie by trie over this thread's rows (Section 4.3's vectorized order)
    for (int j = 0; j < a.nl && kScanRows > 1; j++) {
        const ScanLookup &L = a.lk[j];
        uint32_t val[kScanRows];
        if (STATS) {
#pragma unroll
            for (int r = 0; r < kScanRows; r++) nprobe += alive[r];
        }
        if (L.mode == KM_K32) scan_round<KM_K32>(a, L, row, alive, vec, val);
        else scan_round<KM_K64>(a, L, row, alive, vec, val);
#pragma unroll
        for (int r = 0; r < kScanRows; r++) {
            if (!alive[r]) continue;
            if (!CK(val[r] < L.cnpos)) { alive[r] = false; continue; }
            if (STATS) nhit++;
            hs[j][threadIdx.x * kScanRows + r] = val[r];
            if (L.child_leaf) mult[r] *= L.clen[val[r]];
        }
    }
    if (STATS) {
        u64 np = wave_sum_u64(nprobe), nh = wave_sum_u64(nhit);
        if (__lane_id() == 0 && (np | nh)) {
            atomicAdd(&a.status->probe[a.node], np);
            atomicAdd(&a.status->hit[a.node], nh);
        }
    }
    bool any = false;
#pragma unroll
    for (int r = 0; r < kScanRows; r++) any |= alive[r];
    if (!__any(any)) return;   // the common case: no survivor in the whole wave
    if (a.emit) {
        u64 tot = 0;
#pragma unroll
        for (int r = 0; r < kScanRows; r++) {
            if (!alive[r]) continue;
            u64 e = mult[r];
            for (int q = 0; q < a.ntail; q++) {
                if (a.tail_lk[q] < 0) { e *= a.tail_root_len[q]; continue; }
                const uint32_t th = hs[a.tail_lk[q]][threadIdx.x * kScanRows + r];
                if (!CK(th < a.tail_npos[q])) { e = 0; break; }
                e *= a.tail_len[q][th];
            }
            tot += e;
        }
        // one atomic per wave, spread over the partial counters
        tot = wave_sum_u64(tot);
        if (__lane_id() == 0 && tot)
            atomicAdd(&status->count_part[((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) % kCountParts) *
                                          kPartStride],
                      tot);
    }
    if (!a.emit || a.materialize) {
#pragma unroll
        for (int r = 0; r < kScanRows; r++) {
            const u64 pos = wave_reserve(alive[r], &a.status->survivors) - a.surv_base;
            if (!alive[r] || !CK(pos < a.out.cap)) continue;
            const FrontierDev &O = a.out;
            for (int j = 0; j < a.nout; j++) O.vals[(u64)j * O.cap + pos] = a.cols[a.out_col[j]][row[r]];
            for (int j = 0; j < a.nl; j++)
                if (a.lk[j].hcol >= 0) O.hdl[(u64)a.lk[j].hcol * O.cap + pos] = hs[j][threadIdx.x * kScanRows + r];
            if (O.mult) O.mult[pos] = mult[r];
        }
    }
}

// ------------------------------------------------------------------- emit
// Materialization: every final binding stands for mult * prod(tail lengths)
// result tuples; rows are laid out by a scan of those counts.

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

__global__ void __launch_bounds__(256) k_emit_count(const EmitDev *__restrict__ dp, uint32_t E, u64 *cnt,
                                                    StatusDev *status) {
    const EmitDev &d = *dp;
    uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= E) return;
    if (!CK(e < d.F.cap)) { cnt[e] = 0; return; }
    u64 v = d.F.mult ? d.F.mult[e] : 1ull;
    for (int q = 0; q < d.ntail; q++) {
        uint32_t p;
        v *= tail_len(d, d.tail[q], e, p, status);
    }
    cnt[e] = v;
}

__global__ void __launch_bounds__(256) k_emit_rows(const EmitDev *__restrict__ dp, uint32_t E, const u64 *starts,
                                                   u64 nrows, u64 base, StatusDev *status) {
    const EmitDev &d = *dp;
    u64 r = (u64)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrows) return;
    uint32_t e = E == 1 ? 0u : upper_entry(starts, 0, E, r);
    if (!CK(e < E && e < d.F.cap && r >= starts[e] && r < starts[e + 1] && base + r < d.out_rows)) return;
    u64 idx = r - starts[e];
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
        rows[q] = T.L.offs ? T.L.offs[pos] : pos;
        if (!CK(rows[q] < T.L.nrows)) return;
    }
    int32_t *o = d.out + (base + r) * (u64)d.nhead;
    for (int j = 0; j < d.nhead; j++) {
        int s = d.head_src[j];
        if (s >= 0) {
            o[j] = d.F.vals[(u64)s * d.F.cap + e];
        } else {
            int z = -s - 1;
            int q = z / FJ_MAX_COLS, c = z % FJ_MAX_COLS;
            const TailDev &T = d.tail[q];
            o[j] = T.cols[T.kcol[c]][rows[q]];
        }
    }
}

// ------------------------------------------------------------- launchers

static inline unsigned blocks_for(u64 n, unsigned t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_fill_u32(uint32_t *p, u64 n, uint32_t v, hipStream_t s) {
    if (!n) return hipSuccess;
    unsigned b = (unsigned)std::min<u64>(blocks_for(n, 256), 65535);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(b), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_table_init(void *table, u64 nslots, int mode, hipStream_t s) {
    unsigned b = (unsigned)std::min<u64>(blocks_for(nslots, 256), 65535);
    hipLaunchKernelGGL(k_table_init, dim3(b), dim3(256), 0, s, table, nslots, mode);
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

hipError_t launch_filter_lt(const int32_t *col, u64 n, int32_t bound, uint32_t *out, uint32_t *bsum,
                            uint32_t *total, hipStream_t s) {
    const u64 nb = std::max<u64>((n + kFilterBlock - 1) / kFilterBlock, 1);
    const int vec = ((uintptr_t)col % 16) == 0;
    hipLaunchKernelGGL(k_filter_count, dim3((unsigned)nb), dim3(256), 0, s, col, n, bound, vec, bsum);
    hipLaunchKernelGGL(k_scan_blocks<uint32_t>, dim3(1), dim3(kScanThreads), 0, s, bsum, nb, total,
                       (uint32_t *)nullptr);
    hipLaunchKernelGGL(k_filter_write, dim3((unsigned)nb), dim3(256), 0, s, col, n, bound, vec, (const uint32_t *)bsum,
                       out);
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
    if (nblocks) hipLaunchKernelGGL(k_group_fill, dim3(nblocks), dim3(256), 0, s, fb);
    if (n) hipLaunchKernelGGL(k_group_roots, dim3((n + 255) / 256), dim3(256), 0, s, roots, n);
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

hipError_t launch_emit_count(const void *emit_dev, uint32_t E, u64 *cnt, StatusDev *st, hipStream_t s) {
    hipLaunchKernelGGL(k_emit_count, dim3(blocks_for(E, 256)), dim3(256), 0, s, (const EmitDev *)emit_dev, E, cnt,
                       st);
    return hipGetLastError();
}

hipError_t launch_emit_rows(const void *emit_dev, uint32_t E, const u64 *starts, u64 nrows, u64 base,
                            StatusDev *st, hipStream_t s) {
    if (!nrows) return hipSuccess;
    hipLaunchKernelGGL(k_emit_rows, dim3(blocks_for(nrows, 256)), dim3(256), 0, s, (const EmitDev *)emit_dev, E,
                       starts, nrows, base, st);
    return hipGetLastError();
}

hipError_t launch_scan_probe(const ScanLaunch &l, hipStream_t s) {
    if (l.nl > kScanMaxLookups) return hipErrorInvalidValue;
    if (l.n == 0) return hipSuccess;
    ScanArgs a;
    memset(&a, 0, sizeof(a));
    for (int c = 0; c < FJ_MAX_COLS; c++) a.cols[c] = l.cols[c];
    a.ncols = l.ncols; a.sel = l.sel; a.nrows = l.nrows; a.r0 = l.r0; a.n = l.n;
    // 4-row vector loads need 16-byte aligned columns and a 4-aligned start
    a.vec = kScanRows == 4 && (l.r0 % 4) == 0;
    for (int c = 0; c < l.ncols; c++) a.vec = a.vec && ((uintptr_t)l.cols[c] % 16) == 0;
    a.nl = l.nl;
    for (int j = 0; j < l.nl; j++) {
        a.lk[j] = l.lk[j];
        a.keycol[l.lk[j].kc[0]] = 1;
        if (l.lk[j].mode == KM_K64) a.keycol[l.lk[j].kc[1]] = 1;
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
    if (l.count_stats)
        hipLaunchKernelGGL(k_scan_probe<true>, dim3(blocks_for(l.n, 256 * kScanRows)), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_scan_probe<false>, dim3(blocks_for(l.n, 256 * kScanRows)), dim3(256), 0, s, a);
    return hipGetLastError();
}

int scan_max_lookups() { return kScanMaxLookups; }

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
