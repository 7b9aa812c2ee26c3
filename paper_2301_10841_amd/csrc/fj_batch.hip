// Batched counting for plans that probe only root maps: one persistent
// kernel drains a static queue of (query, row chunk) work items; each thread
// runs the join of Section 3.3 (figure "fj-algo") depth first for one row of
// the first node's cover, iterating later nodes' covers by offset and
// probing root maps, and adds the multiplicities of its results.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fj_dev.h"
#include "fj_launch.h"

namespace fj {

typedef unsigned long long u64;

__device__ __noinline__ void fjb_bad(StatusDev *st, int line) {
    atomicCAS(&st->err_line, 0u, (uint32_t)line);
    atomicAdd(&st->err_count, 1u);
}
#define BCK(cond) ((cond) ? true : (fjb_bad(status, __LINE__), false))

__device__ __forceinline__ uint32_t bmix32(uint32_t h) {
    h ^= h >> 16; h *= 0x85ebca6bu; h ^= h >> 13; h *= 0xc2b2ae35u; h ^= h >> 16;
    return h;
}
__device__ __forceinline__ u64 bmix64(u64 k) {
    k ^= k >> 33; k *= 0xff51afd7ed558ccdull; k ^= k >> 33; k *= 0xc4ceb9fe1a85ec53ull; k ^= k >> 33;
    return k;
}

// get() on a root map: the child start, or ~0u.  Same probe sequence as the
// maps' builder: 32-byte buckets walked forward; the empty-marker key lives
// in the reserved slot after the last bucket.
// Per-thread variables and handles live in LDS: entry i of a thread is at
// [i * blockDim.x + threadIdx.x], so a wave touches consecutive banks.
struct Lane {
    int32_t *v;     // variable values
    uint32_t *h;    // handles per atom
    __device__ __forceinline__ int32_t &var(int i) const { return v[i * blockDim.x + threadIdx.x]; }
    __device__ __forceinline__ uint32_t &hdl(int a) const { return h[a * blockDim.x + threadIdx.x]; }
};

// get() on a root map: the child start (and, for 16-byte slots, the child's
// length in *clen), or ~0u.
__device__ __forceinline__ uint32_t root_get(const BLookup &L, const Lane &ln, uint32_t *clen) {
    if (L.mode == KM_K32) {
        // buckets of four keys, then their four values
        const uint32_t *T = (const uint32_t *)L.table;
        const uint32_t key = (uint32_t)ln.var(L.kslot[0]);
        if (key == kEmpty32) {
            const u64 w = k32_key_word(L.mask + 1);
            return T[w] ? T[w + 4] : ~0u;
        }
        u64 i = (bmix32(key) & L.mask) & ~(u64)(kK32Bucket - 1);
        for (u64 n = 0; n <= k32_part_mask(L.mask); n += kK32Bucket) {
            const u64 w = k32_key_word(i);
            const uint4 q = *(const uint4 *)(T + w);
            const uint32_t ks[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int s = 0; s < 4; s++) {
                if (ks[s] == key) return T[w + 4 + s];
                if (ks[s] == kEmpty32) return ~0u;
            }
            i = k32_next(i, L.mask);
        }
    } else {
        const Slot64 *T = (const Slot64 *)L.table;
        const u64 key = ((u64)(uint32_t)ln.var(L.kslot[0]) << 32) | (uint32_t)ln.var(L.kslot[1]);
        if (key == kEmpty64) {
            *clen = T[L.mask + 1].pad;
            return T[L.mask + 1].key ? T[L.mask + 1].val : ~0u;
        }
        u64 i = (bmix64(key) & L.mask) & ~1ull;   // 2 slots of 16 bytes
        for (u64 n = 0; n <= L.mask; n++) {
            const Slot64 sl = T[i];
            if (sl.key == key) { *clen = sl.pad; return sl.val; }
            if (sl.key == kEmpty64) return ~0u;
            i = (i + 1) & L.mask;
        }
    }
    return ~0u;
}

// Probe node k's lookups for the current binding; false on the first miss.
__device__ __forceinline__ bool probe_node(const BNode &N, const Lane &ln, u64 &mult, StatusDev *status) {
    for (int j = 0; j < N.nl; j++) {
        const BLookup &L = N.lk[j];
        uint32_t clen = 0;
        const uint32_t s = root_get(L, ln, &clen);
        if (s == ~0u) return false;
        if (!BCK(s < L.cnpos)) return false;
        if (L.child_leaf) mult *= L.mode == KM_K64 ? clen : L.clen[s];
        else ln.hdl(L.atom) = s;
    }
    return true;
}

// The join below node K for one binding, depth first.  The recursion is
// unrolled at compile time (K is a template argument), so every depth keeps
// its iterator in registers; the variable and handle arrays are indexed only
// by values of the query's descriptor, which are the same for the whole
// workgroup.
template <int K>
__device__ __forceinline__ void dfs(const BQuery &Q, const Lane &ln, u64 mult, u64 &total, StatusDev *status) {
    if (K >= Q.nexec) {
        // the remaining nodes are single-cover products
        u64 e = mult;
        for (int q = 0; q < Q.ntail; q++) {
            if (Q.tail_root[q]) { e *= Q.tail_root_len[q]; continue; }
            const uint32_t th = ln.hdl(Q.tail_atom[q]);
            if (!BCK(th < Q.tail_npos[q])) return;
            e *= Q.tail_len[q][th];
        }
        total += e;
        return;
    }
    if constexpr (K < kBMaxNodes) {
        const BNode &N = Q.node[K];
        const uint32_t base = ln.hdl(N.catom);
        if (!BCK(base < N.npos)) return;
        const uint32_t lim = N.len[base];
        for (uint32_t pos = 0; pos < lim; pos++) {
            const uint32_t p = base + pos;
            if (!BCK(p < N.npos)) return;
            if (N.kv) {
                ln.var(N.kslot[0]) = N.kv[p];
            } else {
                const uint32_t rw = N.offs[p];
                if (!BCK(rw < N.nrows)) return;
                for (int c = 0; c < N.nk; c++) ln.var(N.kslot[c]) = N.kcol[c][rw];
            }
            u64 mm = mult;
            if (!probe_node(N, ln, mm, status)) continue;
            dfs<K + 1>(Q, ln, mm, total, status);
        }
    }
}

// Node 1 for the node-0 bindings of a whole wave, balanced over its lanes:
// the (binding, child offset) pairs of the 64 lanes are numbered by a wave
// scan of the bindings' child counts and dealt out to the lanes in turn, so
// a binding with many children (a heavy key under skew) does not keep the
// rest of the wave idle.  A lane takes a pair's binding from its owner's
// lane state (LDS) into its own scratch state and goes on depth first.
// Called by every lane of the wave (lim = 0 for lanes with no binding).
__device__ __forceinline__ void expand_node1(const BQuery &Q, const Lane &ln, const Lane &sc, uint32_t base,
                                             uint32_t lim, u64 m, u64 &total, StatusDev *status) {
    const BNode &N = Q.node[1];
    const int lane = threadIdx.x & 63;
    const int wbase = threadIdx.x & ~63;
    u64 x = lim;   // inclusive prefix of the child counts over the wave
    for (int o = 1; o < 64; o <<= 1) {
        const u64 y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    const u64 tot = __shfl(x, 63, 64);
    __builtin_amdgcn_wave_barrier();
    for (u64 t0 = 0; t0 < tot; t0 += 64) {
        const u64 t = t0 + lane;
        int lo = 0, hi = 63;   // owner: the first lane whose prefix exceeds t
#pragma unroll
        for (int step = 0; step < 6; step++) {
            const int mid = (lo + hi) >> 1;
            if (__shfl(x, mid, 64) > t) hi = mid;
            else lo = mid + 1;
        }
        const u64 xo = __shfl(x, lo, 64);
        const uint32_t limo = __shfl(lim, lo, 64);
        const uint32_t baseo = __shfl(base, lo, 64);
        const u64 mo = __shfl(m, lo, 64);
        if (t >= tot) continue;
        const uint32_t pos = (uint32_t)(t - (xo - limo));
        const int otid = wbase + lo;
        for (int v = 0; v < Q.nvars; v++) sc.var(v) = ln.v[v * blockDim.x + otid];
        for (int a = 0; a < Q.natoms; a++) sc.hdl(a) = ln.h[a * blockDim.x + otid];
        __builtin_amdgcn_wave_barrier();
        const uint32_t p = baseo + pos;
        if (!BCK(pos < limo && p < N.npos)) continue;
        if (N.kv) {
            sc.var(N.kslot[0]) = N.kv[p];
        } else {
            const uint32_t rw = N.offs[p];
            if (!BCK(rw < N.nrows)) continue;
            for (int c = 0; c < N.nk; c++) sc.var(N.kslot[c]) = N.kcol[c][rw];
        }
        u64 mm = mo;
        if (!probe_node(N, sc, mm, status)) continue;
        dfs<2>(Q, sc, mm, total, status);
    }
}

__global__ void __launch_bounds__(512) k_batch_dfs(const BQuery *__restrict__ qs, const BItem *__restrict__ items,
                                                   uint32_t nitems, u64 *counts, StatusDev *status, int lv,
                                                   int la) {
    extern __shared__ uint32_t lds[];
    __shared__ u64 red[16];
    // two lane states per thread, each lv variables and la handles (the
    // batch's largest counts): its own (node 0) and a scratch one (node 1
    // pairs dealt to it by expand_node1)
    const uint32_t per = (uint32_t)(lv + la) * blockDim.x;
    const Lane ln{(int32_t *)lds, lds + lv * blockDim.x};
    const Lane sc{(int32_t *)(lds + per), lds + per + lv * blockDim.x};
    for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BItem item = items[it];
        const BQuery &Q = qs[item.q];
        u64 total = 0;
        // the same number of rounds for every lane, so that node 1 can be
        // expanded by the whole wave
        for (uint32_t rb = item.r0; rb < item.r1; rb += blockDim.x) {
            const uint32_t r = rb + threadIdx.x;
            // node 0: the cover is a base table (or its selection)
            const BNode &N0 = Q.node[0];
            bool ok = r < item.r1;
            u64 m = 1;
            if (ok) {
                const uint32_t row = N0.offs ? N0.offs[r] : r;
                ok = BCK(row < N0.nrows);
                if (ok) {
                    for (int c = 0; c < N0.nk; c++) ln.var(N0.kslot[c]) = N0.kcol[c][row];
                    ok = probe_node(N0, ln, m, status);
                }
            }
            if (Q.nexec == 1) {
                if (ok) dfs<1>(Q, ln, m, total, status);
                continue;
            }
            uint32_t base = 0, lim = 0;
            if (ok) {
                const BNode &N1 = Q.node[1];
                base = ln.hdl(N1.catom);
                if (BCK(base < N1.npos)) lim = N1.len[base];
            }
            expand_node1(Q, ln, sc, base, lim, m, total, status);
        }
        // one atomic per work item
        for (int o = 32; o > 0; o >>= 1) total += __shfl_xor(total, o, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = total;
        __syncthreads();
        if (threadIdx.x == 0) {
            u64 t = 0;
            for (int w = 0; w < (int)(blockDim.x >> 6); w++) t += red[w];
            if (t) atomicAdd(&counts[item.q], t);
        }
        __syncthreads();
    }
}

__global__ void k_zero_u64(u64 *p, uint32_t n) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

hipError_t launch_batch_dfs(const BQuery *qs, const BItem *items, uint32_t nitems, u64 *counts, StatusDev *status,
                            int block, int grid, int lv, int la, hipStream_t s) {
    if (nitems == 0) return hipSuccess;
    if (block > 512 || lv < 1 || lv > kBMaxVars || la < 1 || la > FJ_MAX_ATOMS) return hipErrorInvalidValue;
    const size_t lds = 2 * sizeof(uint32_t) * (size_t)(lv + la) * block;
    hipLaunchKernelGGL(k_batch_dfs, dim3(grid), dim3(block), lds, s, qs, items, nitems, counts, status, lv, la);
    return hipGetLastError();
}

hipError_t launch_zero_u64(u64 *p, uint32_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_zero_u64, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace fj
