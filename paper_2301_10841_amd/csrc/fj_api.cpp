// libfj: the C-ABI of include/fj.h.  Host orchestration of the Free Join
// executor: contexts, COLT construction (Section 3.3 build phase, Section 4.2),
// the depth-first, tiled execution of plan nodes with lazy forcing
// (Section 3.3 join phase, Sections 4.3 and 4.4) and output emission.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "fj.h"
#include "fj_dev.h"
#include "fj_host.h"
#include "fj_launch.h"
#include "fj_plan.h"

using fj::FrontierDev;
using fj::LevelDev;
using fj::NodeDev;
using fj::StatusDev;
using fj::SubDev;
using fj::TailDev;
typedef unsigned long long u64;

namespace {

thread_local std::string g_err;

fj_status fail(fj_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define FJ_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? FJ_ERR_OOM : FJ_ERR_HIP,                 \
                        std::string(#call) + ": " + hipGetErrorString(e_));                  \
    } while (0)

#define FJ_TRY(expr)                         \
    do {                                     \
        fj_status s_ = (expr);               \
        if (s_ != FJ_OK) return s_;          \
    } while (0)

template <typename T>
fj_status dalloc(T **p, size_t n) {
    *p = nullptr;
    hipError_t e = hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(FJ_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return FJ_OK;
}

// A device buffer that only grows.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    fj_status ensure(size_t want, hipStream_t s) {
        if (want <= bytes) return FJ_OK;
        if (p) {
            hipStreamSynchronize(s);
            hipFree(p);
            p = nullptr;
            bytes = 0;
        }
        size_t b = std::max<size_t>(want, 256);
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) { p = nullptr; return fail(FJ_ERR_OOM, "hipMalloc of scratch failed"); }
        bytes = b;
        return FJ_OK;
    }
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T> T *as(size_t byte_off = 0) const { return (T *)((char *)p + byte_off); }
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

// ------------------------------------------------------------------ context

struct fj_ctx {
    int device = 0;
    int num_cus = 256;
    hipStream_t stream = nullptr;
    fj_options opt{};
    StatusDev *status_d = nullptr;
    StatusDev *status_h = nullptr;  // pinned
    uint32_t *ftotal_h = nullptr;   // pinned, mapped: a batch of selections' counts, stored by the GPU
    uint32_t *noalloc = nullptr;    // this device's fixed scratch array (fj_filter_lt_noalloc)
    // per-node execution buffers
    DevBuf front[FJ_MAX_NODES + 1];
    DevBuf nodebuf[FJ_MAX_NODES];   // starts | cnt | cov
    DevBuf defer;                   // two deferred lists
    DevBuf force;                   // force scratch
    DevBuf scanb;                   // block sums for scans
    DevBuf desc;                    // node + emit descriptors
    DevBuf emitbuf;                 // emit counts and starts
    DevBuf l0buf;                   // a two-launch first node's list of first-lookup hits
    DevBuf chunkb;                  // per-block binding bounds of a probe launch
    DevBuf sketch;                  // column sketch table and results
    struct ColtGroup *group = nullptr;  // fj_colt_rebuild_many's descriptors and scratch
    struct ColtGroup *group1 = nullptr; // single rebuilds of roots built range by range
    unsigned long long *sketch_h = nullptr;  // pinned sketch results
    void *desc_h = nullptr;         // pinned staging for descriptors
    size_t desc_h_bytes = 0;
    hipEvent_t desc_done = nullptr; // the last copy out of desc_h has finished
    std::vector<char> desc_last;    // the descriptors last copied to the device
    void *desc_last_dev = nullptr;  // and where they went
    // timing
    struct Pending { int cls; hipEvent_t a, b; };
    std::vector<hipEvent_t> pool;
    std::vector<Pending> pending;
    double ms[FJ_T_COUNT] = {0};
    uint64_t launches[FJ_T_COUNT] = {0};
};

namespace {

// Events around the launches of one kernel class (by_launch: the launches
// record them themselves, through hipExtLaunchKernel, with no packets of
// their own in the stream).
struct Timer {
    fj_ctx *c;
    int cls;
    bool by_launch;
    hipEvent_t a = nullptr, b = nullptr;
    Timer(fj_ctx *ctx, int k, bool by_launch_ = false) : c(ctx), cls(k), by_launch(by_launch_) {
        if (!on()) return;
        a = get();
        b = get();
        if (!by_launch) hipEventRecord(a, c->stream);
    }
    ~Timer() {
        if (!on()) return;
        if (!by_launch) hipEventRecord(b, c->stream);
        c->pending.push_back({cls, a, b});
    }
    bool on() const { return c->opt.timing == 2 ? cls == FJ_T_PROBE0 : c->opt.timing != 0; }
    hipEvent_t get() {
        if (!c->pool.empty()) {
            hipEvent_t e = c->pool.back();
            c->pool.pop_back();
            return e;
        }
        hipEvent_t e;
        hipEventCreate(&e);
        return e;
    }
};

fj_status sync_status(fj_ctx *c) {
    FJ_HIP(hipMemcpyAsync(c->status_h, c->status_d, sizeof(StatusDev), hipMemcpyDeviceToHost, c->stream));
    FJ_HIP(hipStreamSynchronize(c->stream));
    if (c->status_h->err_count) {
        std::string msg = "device bounds check failed (fj_kernels.hip line " +
                          std::to_string(c->status_h->err_line) + ", " +
                          std::to_string(c->status_h->err_count) + " times)";
        // report once, then let the context continue
        hipMemsetAsync(&c->status_d->err_line, 0, 2 * sizeof(uint32_t), c->stream);
        hipStreamSynchronize(c->stream);
        return fail(FJ_ERR_INTERNAL, msg);
    }
    return FJ_OK;
}

fj_status zero_status_field(fj_ctx *c, size_t off, size_t bytes) {
    FJ_HIP(hipMemsetAsync((char *)c->status_d + off, 0, bytes, c->stream));
    return FJ_OK;
}

fj_status scan_u64(fj_ctx *c, const u64 *in, u64 *out, u64 n) {
    size_t nb = (n + 1023) / 1024 + 1;
    FJ_TRY(c->scanb.ensure(nb * sizeof(u64), c->stream));
    Timer t(c, FJ_T_SCAN);
    FJ_HIP(fj::launch_scan_u64(in, out, n, c->scanb.as<u64>(), &c->status_d->total, c->stream));
    return FJ_OK;
}

fj_status scan_u32(fj_ctx *c, const uint32_t *in, uint32_t *out, u64 n) {
    size_t nb = (n + 1023) / 1024 + 1;
    FJ_TRY(c->scanb.ensure(nb * sizeof(uint32_t), c->stream));
    Timer t(c, FJ_T_SCAN);
    FJ_HIP(fj::launch_scan_u32(in, out, n, c->scanb.as<uint32_t>(), &c->status_d->total32, c->stream));
    return FJ_OK;
}

}  // namespace

// -------------------------------------------------------------------- COLTs

struct fj_colt {
    int device = 0;
    int atom = -1;
    int ncols = 0;
    int nlev = 0;
    const int32_t *cols[FJ_MAX_COLS] = {nullptr};
    const uint32_t *sel = nullptr;
    int64_t nrows = 0;
    uint32_t nroot = 0;      // rows the root ranges over
    uint32_t cap_rows = 0;   // rows the buffers were sized for
    bool root_built = false;
    bool root_lazy = false;  // unbuilt root that a probe may force (its map is allocated)
    bool root_part = false;  // root map (KM_K32) built range by range by the grouped path
    bool root_keys = true;   // a built root also lists its keys (some node iterates it, or the
                             // simple trie forces its children up front); else it is only probed
    uint32_t *bloom_buf = nullptr;   // the root map's key filter (kBloomWords), if it may have one
    int lev_nk[fj::kMaxLevels] = {0};
    int lev_var[fj::kMaxLevels][FJ_MAX_COLS] = {{0}};
    LevelDev lev[fj::kMaxLevels + 1];
    u64 table_slots[fj::kMaxLevels] = {0};   // slots of each level's map in use (reserved slot included)
    u64 table_cap[fj::kMaxLevels] = {0};     // slots each level's map was allocated for
    // Regions a (re)build initialises: the root level's counters and map and
    // every level's state words.  An inner level's counters and map are
    // initialised before its first force after a rebuild (lev_ready).
    fj::FillList fill_h{};
    fj::FillList *fill_dev = nullptr;
    u64 fill_words = 0;
    fj::FillList fill_lev_h[fj::kMaxLevels]{};
    fj::FillList *fill_lev_dev[fj::kMaxLevels] = {nullptr};
    u64 fill_lev_words[fj::kMaxLevels] = {0};
    bool lev_ready[fj::kMaxLevels] = {false};
    bool fill_stale = true;   // the device copies of the fill lists are out of date
    u64 sized_rows = ~0ull;   // the root rows the maps and fill lists were last sized for
    std::vector<std::pair<void *, size_t>> allocs;   // pooled device buffers and their sizes
};

namespace {

int key_mode(int level, int nk) {
    if (nk == 0) return fj::KM_ZERO;
    if (level == 0 && nk == 1) return fj::KM_K32;
    if ((level == 0 && nk == 2) || (level > 0 && nk == 1)) return fj::KM_K64;
    return fj::KM_REP;
}

// Map capacity for at most `rows` keys: a power of two of at least twice the
// rows, so linear probing always ends at an empty slot.
u64 map_cap(u64 rows) {
    u64 cap = 16;
    while (cap < 2 * rows) cap <<= 1;
    return cap;
}

size_t slot_bytes(int mode) {
    return mode == fj::KM_K32 ? 2 * sizeof(uint32_t) : (mode == fj::KM_K64 ? sizeof(fj::Slot64) : sizeof(fj::SlotRep));
}

template <typename T>
fj_status colt_alloc(fj_colt *t, T **p, size_t n) {
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    void *q = nullptr;
    FJ_TRY(fj::pool_alloc(t->device, bytes, &q));
    *p = (T *)q;
    t->allocs.push_back({q, bytes});
    return FJ_OK;
}

// Device buffers for every level; contents are initialised by colt_reset.
fj_status colt_allocate(fj_colt *t) {
    const size_t n = std::max<uint32_t>(t->cap_rows, 1);
    t->bloom_buf = nullptr;
    for (int l = 0; l <= t->nlev; l++) {
        LevelDev &L = t->lev[l];
        memset(&L, 0, sizeof(L));
        L.npos = (uint32_t)n;
        L.nrows = (uint32_t)t->nrows;
        bool leaf = (l == t->nlev);
        if (l > 0) FJ_TRY(colt_alloc(t, &L.offs, n));
        FJ_TRY(colt_alloc(t, &L.len, n));
        if (leaf) continue;
        // a level below the root keyed by one variable keeps that key beside
        // each offset (written when its parent is forced)
        if (l > 0 && t->lev_nk[l] == 1) FJ_TRY(colt_alloc(t, &L.kv, n));
        FJ_TRY(colt_alloc(t, &L.st, n));
        if (l == 0 && !t->root_built && !t->root_lazy && t->nlev == 1) {
            // a base table only ever iterated directly: no map, no scratch
            L.nk = t->lev_nk[l];
            L.mode = fj::KM_ZERO;
            continue;
        }
        FJ_TRY(colt_alloc(t, &L.kl, n));
        if (t->lev_nk[l] == 1) {
            // forced handles list their keys and each key's offset count
            FJ_TRY(colt_alloc(t, &L.kk, n));
            FJ_TRY(colt_alloc(t, &L.kn, n));
        }
        FJ_TRY(colt_alloc(t, &L.rank_ctr, n));
        FJ_TRY(colt_alloc(t, &L.cnt, n));
        FJ_TRY(colt_alloc(t, &L.fq, n));
        L.nk = t->lev_nk[l];
        L.mode = key_mode(l, L.nk);
        L.local = l > 0 && (L.mode == fj::KM_K64 || L.mode == fj::KM_REP);
        if (L.mode != fj::KM_ZERO) {
            // sized for the capacity; each (re)build uses the part its rows need
            const u64 cap = map_cap(n);
            L.mask = cap - 1;
            L.nslots = cap + 1;
            t->table_slots[l] = cap + 1;
            t->table_cap[l] = cap;
            char *tb = nullptr;
            FJ_TRY(colt_alloc(t, &tb, L.mode == fj::KM_K32 ? fj::k32_table_words(cap) * sizeof(uint32_t)
                                                           : (cap + 1) * slot_bytes(L.mode)));
            L.table = tb;
            if (l == 0 && L.mode == fj::KM_K32 && t->root_built) FJ_TRY(colt_alloc(t, &t->bloom_buf, fj::kBloomWords));
        }
    }
    return FJ_OK;
}

// Callers make sure no queued work still uses the buffers.
void colt_free_all(fj_colt *t) {
    for (const auto &a : t->allocs) fj::pool_free(t->device, a.first, a.second);
    t->allocs.clear();
    t->sized_rows = ~0ull;
}

}  // namespace

static fj_status colt_level_ready(fj_ctx *c, fj_colt *t, int l);

// Scratch layout of one force: lens (nh) | pre (nh + 1) | wslot (W) |
// cntv (W, 64-bit) | ex (W + 1, 64-bit).
struct ForceScratch {
    size_t off_pre, off_w, off_c, off_e;
    ForceScratch(uint32_t nh, u64 wmax) {
        off_pre = align256(sizeof(uint32_t) * nh);
        off_w = align256(off_pre + sizeof(uint32_t) * (nh + 1));
        off_c = align256(off_w + sizeof(uint32_t) * (wmax + 1));
        off_e = align256(off_c + sizeof(u64) * (wmax + 1));
    }
    size_t bytes(u64 wmax) const { return off_e + align256(sizeof(u64) * (wmax + 2)); }
};

// Force every handle queued on level l of colt t (the queue holds nh handle
// starts; W is their total length when the caller knows it, else ~0).
// pre_ready: the prefix of the handle lengths is already in scratch (the
// single root handle, written by the COLT init kernel).
static fj_status force_queue(fj_ctx *c, fj_colt *t, int l, uint32_t nh, u64 W_known, int timer_cls,
                             fj_stats *stats, int node, bool pre_ready = false) {
    if (nh == 0) return FJ_OK;
    FJ_TRY(colt_level_ready(c, t, l));
    LevelDev &L = t->lev[l];
    LevelDev &C = t->lev[l + 1];
    u64 Wmax = W_known != ~0ull ? W_known : t->nroot;
    ForceScratch fs(nh, Wmax);
    FJ_TRY(c->force.ensure(fs.bytes(Wmax), c->stream));
    uint32_t *lens = c->force.as<uint32_t>(0);
    uint32_t *pre = c->force.as<uint32_t>(fs.off_pre);
    Timer tm(c, timer_cls);
    if (!pre_ready) {
        FJ_HIP(fj::launch_fq_lens(L, L.fq, nh, lens, c->status_d, c->stream));
        FJ_TRY(scan_u32(c, lens, pre, nh));
    }
    u64 W = W_known;
    if (W == ~0ull) {
        FJ_TRY(sync_status(c));
        W = c->status_h->total32;
    }
    if (W > Wmax) return fail(FJ_ERR_INTERNAL, "forced offsets exceed the relation size");
    fj::ForceLaunch f;
    f.L = L;
    f.C = C;
    for (int j = 0; j < FJ_MAX_COLS; j++) f.cols[j] = t->cols[j];
    f.fq = L.fq;
    f.nh = nh;
    f.pre = pre;
    f.W = (uint32_t)W;
    f.wslot = c->force.as<uint32_t>(fs.off_w);
    f.cntv = c->force.as<u64>(fs.off_c);
    f.ex = c->force.as<u64>(fs.off_e);
    f.wcap = (uint32_t)(Wmax + 1);
    f.status = c->status_d;
    FJ_HIP(fj::launch_force_phase(0, f, c->stream));   // insert and count
    FJ_HIP(fj::launch_force_phase(1, f, c->stream));   // (1, count) per new key
    FJ_TRY(scan_u64(c, f.cntv, f.ex, W));               // ranks and child starts
    FJ_HIP(fj::launch_force_phase(2, f, c->stream));   // publish children
    FJ_HIP(fj::launch_force_phase(3, f, c->stream));   // scatter offsets
    if (stats && node >= 0) {
        stats->forced[node] += nh;
        stats->forced_offsets[node] += W;
    }
    return FJ_OK;
}

// The regions a (re)build initialises (the root level's counters and map,
// every level's state words) and, per inner level, the counters and map its
// first force initialises, for a root over `rows` rows: positions past them
// are never touched.  Map slots start empty, the reserved slot unclaimed.
// Host lists only (colt_fill_upload copies them to the device).
static fj_status colt_fill_list(fj_colt *t, u64 rows) {
    bool overflow = false;
    auto add = [&](fj::FillList &fl, u64 &total, uint32_t *p, u64 nwords, std::initializer_list<uint32_t> pat) {
        if (!p || !nwords) return;
        if (fl.n >= fj::kMaxFill || (pat.size() != 1 && pat.size() != 2 && pat.size() != 4 && pat.size() != 8)) {
            overflow = true;   // the fill kernels take periods of 1, 2, 4 or 8 words
            return;
        }
        fj::FillRegion &r = fl.r[fl.n++];
        r.p = p;
        r.nwords = nwords;
        r.period = (int)pat.size();
        int i = 0;
        for (uint32_t v : pat) r.pat[i++] = v;
        total += nwords;
    };
    const u64 n = std::max<u64>(std::min<u64>(rows, t->cap_rows), 1);
    memset(&t->fill_h, 0, sizeof(t->fill_h));
    t->fill_words = 0;
    for (int l = 0; l < t->nlev; l++) {
        LevelDev &L = t->lev[l];
        // (the root's state word is set with the root handle, not filled; a
        // root built range by range clears level 1's state words itself)
        if (l > 0 && !(l == 1 && t->root_part)) add(t->fill_h, t->fill_words, L.st, n, {0u});
        fj::FillList &fl = l == 0 ? t->fill_h : t->fill_lev_h[l];
        u64 &words = l == 0 ? t->fill_words : t->fill_lev_words[l];
        if (l > 0) {
            memset(&fl, 0, sizeof(fl));
            words = 0;
        }
        if (!L.cnt) continue;  // directly iterated base table
        // (the counters serve the force passes, which a root built range
        // by range does not use)
        if (!(l == 0 && t->root_part)) add(fl, words, L.cnt, n, {0u});
        if (!L.table || (l == 0 && t->root_part)) continue;
        const u64 ns = t->table_slots[l];
        uint32_t *T = (uint32_t *)L.table;
        if (L.mode == fj::KM_K32) {
            // buckets of four empty keys and four zero values (the insert
            // counts a key's rows in its value); the reserved slot unclaimed
            const u64 kw = fj::k32_key_word(ns - 1);
            add(fl, words, T, kw, {fj::kEmpty32, fj::kEmpty32, fj::kEmpty32, fj::kEmpty32, 0u, 0u, 0u, 0u});
            add(fl, words, T + kw, fj::k32_table_words(ns - 1) - kw, {0u});
        } else if (L.mode == fj::KM_K64) {
            add(fl, words, T, 4 * (ns - 1), {fj::kEmpty32, fj::kEmpty32, 0u, 0u});
            add(fl, words, T + 4 * (ns - 1), 4, {0u});
        } else {
            add(fl, words, T, 4 * ns, {fj::kEmpty32, fj::kEmpty32, 0u, 0u});
        }
    }
    if (overflow) return fail(FJ_ERR_UNSUPPORTED, "too many COLT levels");
    return FJ_OK;
}

// Size every level's map for the rows the root now ranges over (within the
// capacity it was allocated for) and recompute the fill lists; the device
// copies are marked stale when they change.
static fj_status colt_size(fj_colt *t) {
    const u64 rows = std::max<uint32_t>(t->nroot, 1);
    const bool part_was = t->root_part;
    for (int l = 0; l < t->nlev; l++) {
        LevelDev &L = t->lev[l];
        if (!L.table || rows == t->sized_rows) continue;
        const u64 cap = std::min(map_cap(rows), t->table_cap[l]);
        L.mask = cap - 1;
        L.nslots = cap + 1;
        t->table_slots[l] = cap + 1;
    }
    // a built KM_K32 root of at most kMaxParts ranges is built range by
    // range, which writes its whole table: the fill lists leave it out
    {
        const LevelDev &R = t->lev[0];
        const u64 cap = R.mask + 1, psz = std::min<u64>(cap, fj::kK32Part);
        t->root_part = t->root_built && t->nroot > 0 && t->nlev >= 1 && R.table && R.mode == fj::KM_K32 &&
                       cap / psz <= fj::kMaxParts;
        // its key filter: at most kBloomWords words of 2^s buckets each,
        // and at least one word per build range
        LevelDev &Rw = t->lev[0];
        Rw.bloom = nullptr;
        Rw.bloom_shift = 0;
        if (t->root_part && t->bloom_buf) {
            uint32_t sh = 0;
            while (((cap / fj::kK32Bucket) >> sh) > fj::kBloomWords) sh++;
            if (((psz / fj::kK32Bucket) >> sh) >= 1) {
                Rw.bloom = t->bloom_buf;
                Rw.bloom_shift = sh;
            }
        }
    }
    if (rows == t->sized_rows && part_was == t->root_part) return FJ_OK;   // as the last sizing left them
    const fj::FillList old = t->fill_h;
    std::vector<fj::FillList> old_lev(t->fill_lev_h, t->fill_lev_h + fj::kMaxLevels);
    FJ_TRY(colt_fill_list(t, rows));
    if (memcmp(&old, &t->fill_h, sizeof(old)) != 0 ||
        memcmp(old_lev.data(), t->fill_lev_h, sizeof(fj::FillList) * fj::kMaxLevels) != 0)
        t->fill_stale = true;
    t->sized_rows = rows;
    return FJ_OK;
}

// Device copies of the fill lists, (re)written when stale.  Rare (the rows
// changed): waits for the work queued so far, which may still read them.
static fj_status colt_fill_upload(fj_ctx *c, fj_colt *t) {
    if (!t->fill_stale) return FJ_OK;
    FJ_HIP(hipStreamSynchronize(c->stream));
    if (!t->fill_dev) FJ_TRY(colt_alloc(t, &t->fill_dev, 1));
    FJ_HIP(hipMemcpy(t->fill_dev, &t->fill_h, sizeof(t->fill_h), hipMemcpyHostToDevice));
    for (int l = 1; l < t->nlev; l++) {
        if (!t->fill_lev_dev[l]) FJ_TRY(colt_alloc(t, &t->fill_lev_dev[l], 1));
        FJ_HIP(hipMemcpy(t->fill_lev_dev[l], &t->fill_lev_h[l], sizeof(fj::FillList), hipMemcpyHostToDevice));
    }
    t->fill_stale = false;
    return FJ_OK;
}

// Initialise inner level l's counters and map before its first force since
// the last rebuild.
static fj_status colt_level_ready(fj_ctx *c, fj_colt *t, int l) {
    if (l == 0 || t->lev_ready[l]) return FJ_OK;
    if (t->fill_lev_words[l]) {
        LevelDev none;
        memset(&none, 0, sizeof(none));
        FJ_HIP(fj::launch_fill_list(t->fill_lev_dev[l], t->fill_lev_words[l], none, 0, nullptr, c->stream));
    }
    t->lev_ready[l] = true;
    return FJ_OK;
}

// The simple trie of the paper's ablation: every level below the root is
// forced now, level by level, each trie of level l being a child of a
// forced trie of level l - 1.
static fj_status colt_force_all(fj_ctx *c, fj_colt *t) {
    if (c->opt.trie != 2 || !t->root_built || t->nroot == 0) return FJ_OK;
    for (int l = 1; l < t->nlev; l++) {
        const int slot = t->atom * fj::kMaxLevels + l;
        const size_t off = offsetof(StatusDev, fq_n) + sizeof(uint32_t) * slot;
        FJ_TRY(zero_status_field(c, off, sizeof(uint32_t)));
        {
            Timer tm(c, FJ_T_BUILD);
            // the root's one trie has at most nroot keys; below it a trie
            // starts at any of the nroot positions
            FJ_HIP(fj::launch_enqueue_children(t->lev[l - 1], t->lev[l], t->nroot, l == 1 ? 1 : 0,
                                               &c->status_d->fq_n[slot], c->status_d, c->stream));
        }
        FJ_TRY(sync_status(c));
        const uint32_t nh = c->status_h->fq_n[slot];
        FJ_TRY(force_queue(c, t, l, nh, ~0ull, FJ_T_BUILD, nullptr, -1));
        FJ_TRY(zero_status_field(c, off, sizeof(uint32_t)));
    }
    return FJ_OK;
}

static fj_status colt_rebuild_group(fj_ctx *c, fj_colt *t);

static fj_status colt_reset(fj_ctx *c, fj_colt *t) {
    FJ_TRY(colt_size(t));
    FJ_TRY(colt_fill_upload(c, t));
    if (t->root_part) return colt_rebuild_group(c, t);
    for (int l = 0; l <= t->nlev; l++) t->lev[l].nrows = (uint32_t)t->nrows;
    for (int l = 0; l < t->nlev; l++) t->lev_ready[l] = false;
    LevelDev &R = t->lev[0];
    R.offs = const_cast<uint32_t *>(t->sel);
    const bool force_root = t->root_built && t->nroot > 0;
    uint32_t *pre = nullptr;
    if (force_root) {
        ForceScratch fs(1, t->nroot);
        FJ_TRY(c->force.ensure(fs.bytes(t->nroot), c->stream));
        pre = c->force.as<uint32_t>(fs.off_pre);
    }
    {
        Timer tm(c, FJ_T_BUILD);
        FJ_HIP(fj::launch_fill_list(t->fill_dev, t->fill_words, R, t->nroot, pre, c->stream));
    }
    if (t->root_built) {
        if (t->nroot == 0) {
            FJ_HIP(fj::launch_fill_u32(R.st, 1, 1u, c->stream));  // forced, no keys
        } else {
            FJ_TRY(force_queue(c, t, 0, 1, t->nroot, FJ_T_BUILD, nullptr, -1, true));
        }
    }
    return colt_force_all(c, t);
}

// ---------------------------------------------------------- grouped rebuilds
// The root builds of many COLTs in one launch per phase (fill, root words,
// the four force passes and one scan), with descriptors and scratch owned by
// the group.  Member k's work items are the rows of its root when the root
// map is built.

struct ColtGroup {
    int n = 0;
    u64 wtot = 0;
    uint32_t nfill = 0;
    // members whose KM_K32 root maps are built range by range
    int npm = 0;
    bool part_keys = false;   // some such member lists its root's keys (the rank pass runs)
    uint32_t nparts = 0, nblocks = 0;
    u64 wp = 0;
    DevBuf meta;   // descs | wpre | roots | pre | part members | fill blocks
    DevBuf work;   // wslot | cntv | ex | block sums | total | range arrays
    size_t o_wpre = 0, o_roots = 0, o_pre = 0, o_pmem = 0, o_fill = 0, o_mop = 0, o_mob = 0, meta_bytes = 0;
    size_t w_cntv = 0, w_ex = 0, w_bsum = 0, w_total = 0;
    size_t w_prow = 0, w_pkey = 0, w_pkv = 0, w_scnt = 0, w_poff = 0, w_pdist = 0, w_rstart = 0, w_pbsum = 0;
    std::vector<char> stage, last;   // host image of meta, and the last one uploaded
    std::vector<char> last_key;      // the inputs that image was made from
    char *stage_h = nullptr;         // pinned copy source
    size_t stage_h_bytes = 0;
    void release() {
        meta.release();
        work.release();
        if (stage_h) hipHostFree(stage_h);
        stage_h = nullptr;
        stage_h_bytes = 0;
        last.clear();
        last_key.clear();
    }
};

static void destroy_group(ColtGroup *g) {
    if (!g) return;
    g->release();
    delete g;
}

namespace {

constexpr u64 kFillChunk = 4096;   // words per fill block

// Lay out and upload the group's descriptors for the COLTs' current
// relations; wcap_min sizes the scratch (at least the current total).
template <typename T>
void key_put(std::vector<char> &key, const T &v) {
    const char *b = (const char *)&v;
    key.insert(key.end(), b, b + sizeof(T));
}

fj_status group_prepare(fj_ctx *c, ColtGroup &G, fj_colt *const *colts, int n, u64 wcap_min) {
    // every member starts over: the root ranges over the current relation,
    // inner levels are initialised again before their first force
    for (int k = 0; k < n; k++) {
        fj_colt *t = colts[k];
        for (int l = 0; l <= t->nlev; l++) t->lev[l].nrows = (uint32_t)t->nrows;
        for (int l = 0; l < t->nlev; l++) t->lev_ready[l] = false;
        t->lev[0].offs = const_cast<uint32_t *>(t->sel);
    }
    // the uploaded image depends only on these inputs: when they are the
    // last call's (a query rebuilt step after step), it is still current
    std::vector<char> key;
    key.reserve(64 + (size_t)n * (2 * sizeof(LevelDev) + sizeof(fj::FillList) + 128));
    key_put(key, n);
    key_put(key, wcap_min);
    for (int k = 0; k < n; k++) {
        const fj_colt *t = colts[k];
        key_put(key, t);
        key_put(key, t->nroot);
        key_put(key, t->root_built);
        key_put(key, t->root_part);
        key_put(key, t->root_keys);
        key_put(key, t->nrows);
        key_put(key, t->sel);
        key_put(key, t->cols);
        key_put(key, t->lev[0]);
        key_put(key, t->lev[1]);
        key_put(key, t->fill_h);
    }
    if (!G.last.empty() && key == G.last_key && G.n == n) return FJ_OK;
    G.last_key.clear();
    G.n = n;
    // the general path takes the built roots not built range by range
    std::vector<u64> wpre(n + 1, 0);
    std::vector<fj::PartMember> pm;
    u64 wp = 0, nslots = 0, noff = 0;
    uint32_t nparts = 0, nblocks = 0;
    for (int k = 0; k < n; k++) {
        const fj_colt *t = colts[k];
        wpre[k + 1] = wpre[k] + ((t->root_built && t->nroot > 0 && !t->root_part) ? t->nroot : 0);
        if (!t->root_part) continue;
        const u64 cap = t->lev[0].mask + 1, psz = std::min<u64>(cap, fj::kK32Part);
        fj::PartMember m;
        m.desc = k;
        m.np = (uint32_t)(cap / psz);
        m.plog = 0;
        while ((1ull << m.plog) < psz) m.plog++;
        m.part_base = nparts;
        m.block_base = nblocks;
        m.item_base = (uint32_t)wp;
        m.W = t->nroot;
        m.keys = t->root_keys ? 1 : 0;
        m.slot_base = nslots;
        nslots += (u64)m.np << m.plog;
        if (wp + t->nroot > 0xFFFFFFFFull) return fail(FJ_ERR_UNSUPPORTED, "grouped roots of 2^32 rows or more");
        // place slices: whole chunks, at most kMaxPlaceBlocks of them
        const u64 W = t->nroot, chunks = (W + fj::kPlaceChunk - 1) / fj::kPlaceChunk;
        const u64 cpb = (chunks + fj::kMaxPlaceBlocks - 1) / fj::kMaxPlaceBlocks;   // chunks per block
        m.ipb = (uint32_t)(cpb * fj::kPlaceChunk);
        m.nb = (uint32_t)((W + m.ipb - 1) / m.ipb);
        m.off_base = noff;
        noff += (u64)(m.np + 1) * m.nb;
        m.clear_cst = (t->nlev >= 2 && t->lev[1].st) ? 1 : 0;   // left out of its fill list
        nparts += m.np;
        nblocks += m.nb;
        wp += t->nroot;
        pm.push_back(m);
    }
    G.wtot = wpre[n];
    G.npm = (int)pm.size();
    G.part_keys = false;
    for (int k = 0; k < n; k++) G.part_keys = G.part_keys || (colts[k]->root_part && colts[k]->root_keys);
    G.nparts = nparts;
    G.nblocks = nblocks;
    G.wp = wp;
    const u64 wcap = std::max<u64>(G.wtot, wcap_min);
    // work layout: the general path's per-item scratch, then the range arrays
    G.w_cntv = align256(sizeof(uint32_t) * (wcap + 1));
    G.w_ex = G.w_cntv + align256(sizeof(u64) * (wcap + 1));
    G.w_bsum = G.w_ex + align256(sizeof(u64) * (wcap + 2));
    G.w_total = G.w_bsum + align256(sizeof(u64) * (wcap / 1024 + 2));
    const size_t item_bytes = align256(sizeof(uint32_t) * (wp + 1));
    G.w_prow = G.w_total + 256;
    G.w_pkey = G.w_prow + item_bytes;
    G.w_pkv = G.w_pkey + item_bytes;
    G.w_scnt = G.w_pkv + item_bytes;
    G.w_poff = G.w_scnt + align256(sizeof(uint32_t) * (nslots + 1));
    G.w_pdist = G.w_poff + align256(sizeof(uint32_t) * (noff + 1));
    G.w_rstart = G.w_pdist + align256(sizeof(uint32_t) * (nparts + 1));
    G.w_pbsum = G.w_rstart + align256(sizeof(uint32_t) * (nparts + 1));
    const size_t work_bytes = G.w_pbsum + align256(sizeof(uint32_t) * (nparts / 1024 + 2)) + 256;
    FJ_TRY(G.work.ensure(work_bytes, c->stream));
    std::vector<fj::FillBlock> fb;
    for (int k = 0; k < n; k++) {
        const fj::FillList &fl = colts[k]->fill_h;
        for (int r = 0; r < fl.n; r++)
            for (u64 off = 0; off < fl.r[r].nwords; off += kFillChunk) {
                fj::FillBlock b;
                b.p = fl.r[r].p;
                b.start = off;
                b.n = std::min<u64>(kFillChunk, fl.r[r].nwords - off);
                for (int q = 0; q < 8; q++) b.pat[q] = fl.r[r].pat[q];
                b.period = fl.r[r].period;
                fb.push_back(b);
            }
    }
    if (fb.size() > 0x7fffffff) return fail(FJ_ERR_UNSUPPORTED, "too many fill blocks");
    G.nfill = (uint32_t)fb.size();
    G.o_wpre = align256(sizeof(fj::ForceArgs) * n);
    G.o_roots = G.o_wpre + align256(sizeof(u64) * (n + 1));
    G.o_pre = G.o_roots + align256(sizeof(fj::GroupRoot) * n);
    G.o_pmem = G.o_pre + align256(sizeof(uint32_t) * 2 * n);
    G.o_fill = G.o_pmem + align256(sizeof(fj::PartMember) * std::max<size_t>(pm.size(), 1));
    // each range's and each place block's member, so that a workgroup finds
    // its member with one load
    G.o_mop = G.o_fill + align256(sizeof(fj::FillBlock) * std::max<size_t>(fb.size(), 1));
    G.o_mob = G.o_mop + align256(sizeof(uint32_t) * std::max<u64>(nparts, 1));
    G.meta_bytes = G.o_mob + align256(sizeof(uint32_t) * std::max<u64>(nblocks, 1));
    FJ_TRY(G.meta.ensure(G.meta_bytes, c->stream));
    char *meta = G.meta.as<char>();
    uint32_t *wslot = G.work.as<uint32_t>();
    u64 *cntv = G.work.as<u64>(G.w_cntv), *ex = G.work.as<u64>(G.w_ex);
    G.stage.assign(G.meta_bytes, 0);
    char *h = G.stage.data();
    fj::ForceArgs *descs = (fj::ForceArgs *)h;
    fj::GroupRoot *roots = (fj::GroupRoot *)(h + G.o_roots);
    memcpy(h + G.o_wpre, wpre.data(), sizeof(u64) * (n + 1));
    for (int k = 0; k < n; k++) {
        fj_colt *t = colts[k];
        LevelDev &R = t->lev[0];
        uint32_t *pre_d = (uint32_t *)(meta + G.o_pre) + 2 * k;
        fj::ForceArgs &a = descs[k];
        a.L = R;
        a.C = t->lev[1];
        for (int j = 0; j < FJ_MAX_COLS; j++) a.cols[j] = t->cols[j];
        a.fq = R.fq;
        a.nh = 1;
        a.pre = pre_d;
        a.W = (uint32_t)(wpre[k + 1] - wpre[k]);
        a.wcap = a.W + 1;
        a.wslot = wslot + wpre[k];
        a.cntv = cntv + wpre[k];
        a.ex = ex + wpre[k];
        a.status = c->status_d;
        fj::GroupRoot &g = roots[k];
        g.len = R.len;
        g.st = R.st;
        g.fq = R.fq;
        g.pre = t->root_built ? pre_d : nullptr;
        g.nroot = t->nroot;
        g.built = t->root_built ? 1 : 0;
    }
    if (!pm.empty()) memcpy(h + G.o_pmem, pm.data(), sizeof(fj::PartMember) * pm.size());
    {
        uint32_t *mop = (uint32_t *)(h + G.o_mop), *mob = (uint32_t *)(h + G.o_mob);
        for (size_t k = 0; k < pm.size(); k++) {
            for (uint32_t q = 0; q < pm[k].np; q++) mop[pm[k].part_base + q] = (uint32_t)k;
            for (uint32_t q = 0; q < pm[k].nb; q++) mob[pm[k].block_base + q] = (uint32_t)k;
        }
    }
    if (!fb.empty()) memcpy(h + G.o_fill, fb.data(), sizeof(fj::FillBlock) * fb.size());
    if (G.stage != G.last) {
        FJ_HIP(hipStreamSynchronize(c->stream));   // the pinned source may still be in use
        if (G.stage_h_bytes < G.meta_bytes) {
            if (G.stage_h) hipHostFree(G.stage_h);
            G.stage_h = nullptr;
            G.stage_h_bytes = 0;
            FJ_HIP(hipHostMalloc((void **)&G.stage_h, G.meta_bytes, hipHostMallocDefault));
            G.stage_h_bytes = G.meta_bytes;
        }
        memcpy(G.stage_h, h, G.meta_bytes);
        FJ_HIP(hipMemcpyAsync(meta, G.stage_h, G.meta_bytes, hipMemcpyHostToDevice, c->stream));
        G.last = G.stage;
    }
    G.last_key = std::move(key);
    return FJ_OK;
}

// The launches of a grouped rebuild (no allocation, no host synchronization).
fj_status group_launch(fj_ctx *c, ColtGroup &G) {
    char *meta = G.meta.as<char>();
    const fj::ForceArgs *descs = (const fj::ForceArgs *)meta;
    const u64 *wpre = (const u64 *)(meta + G.o_wpre);
    Timer tm(c, FJ_T_BUILD);
    // with nothing to fill and no general-path member, the place pass of
    // the range builds writes the root words (one launch less)
    const bool roots_in_place = G.nfill == 0 && G.wtot == 0 && G.nparts > 0 && G.nblocks > 0;
    if (!roots_in_place)
        FJ_HIP(fj::launch_group_fill((const fj::FillBlock *)(meta + G.o_fill), G.nfill,
                                     (const fj::GroupRoot *)(meta + G.o_roots), G.n, c->stream));
    if (G.wtot > 0) {
        FJ_HIP(fj::launch_group_force(0, descs, wpre, G.n, G.wtot, c->stream));   // insert and count
        FJ_HIP(fj::launch_group_force(1, descs, wpre, G.n, G.wtot, c->stream));   // (1, count) per new key
        FJ_HIP(fj::launch_scan_u64(G.work.as<u64>(G.w_cntv), G.work.as<u64>(G.w_ex), G.wtot,
                                   G.work.as<u64>(G.w_bsum), G.work.as<u64>(G.w_total), c->stream));
        FJ_HIP(fj::launch_group_force(2, descs, wpre, G.n, G.wtot, c->stream));   // publish children
        FJ_HIP(fj::launch_group_force(3, descs, wpre, G.n, G.wtot, c->stream));   // scatter offsets
    }
    if (G.nparts > 0) {
        // KM_K32 roots range by range: place by slice, build, rank
        fj::PartArgs pa;
        memset(&pa, 0, sizeof(pa));
        pa.descs = descs;
        pa.mem = (const fj::PartMember *)(meta + G.o_pmem);
        pa.mop = (const uint32_t *)(meta + G.o_mop);
        pa.mob = (const uint32_t *)(meta + G.o_mob);
        pa.n = G.npm;
        pa.nblocks = G.nblocks;
        pa.nparts = G.nparts;
        pa.items = (uint32_t)G.wp;
        pa.poff = G.work.as<uint32_t>(G.w_poff);
        pa.prow = G.work.as<uint32_t>(G.w_prow);
        pa.pkey = G.work.as<uint32_t>(G.w_pkey);
        pa.pkv = G.work.as<uint32_t>(G.w_pkv);
        pa.scnt = G.work.as<uint32_t>(G.w_scnt);
        pa.pdist = G.work.as<uint32_t>(G.w_pdist);
        if (roots_in_place) {
            pa.roots = (const fj::GroupRoot *)(meta + G.o_roots);
            pa.nroots = G.n;
        }
        pa.rstart = G.work.as<uint32_t>(G.w_rstart);
        pa.status = c->status_d;
        uint32_t *pbsum = G.work.as<uint32_t>(G.w_pbsum);
        // few ranges: the rank pass sums the distinct counts it needs (no
        // scan launch); more: the scan runs in one workgroup, or in three
        // launches beyond 32,768 ranges
        pa.inline_scan = G.nparts <= 2048 ? 1 : 0;
        // roots that are only probed need no key list: the build pass marks
        // each forced, and the rank pass (run when some root lists its keys)
        // skips them
        auto scan = [&](const uint32_t *in, uint32_t *out) -> hipError_t {
            if (pa.inline_scan) return hipSuccess;
            return G.nparts <= 32768 ? fj::launch_scan_small_u32(in, out, G.nparts, c->stream)
                                     : fj::launch_scan_u32(in, out, G.nparts, pbsum, out + G.nparts, c->stream);
        };
        FJ_HIP(fj::launch_part_phase(0, pa, c->stream));
        FJ_HIP(fj::launch_part_phase(1, pa, c->stream));
        if (G.part_keys) {
            FJ_HIP(scan(pa.pdist, pa.rstart));
            FJ_HIP(fj::launch_part_phase(2, pa, c->stream));
        }
    }
    return FJ_OK;
}

}  // namespace

// One COLT's root built range by range, through the grouped path (its own
// group, so that fj_colt_rebuild_many's cached descriptors stay valid).
static fj_status colt_rebuild_group(fj_ctx *c, fj_colt *t) {
    if (!c->group1) c->group1 = new ColtGroup();
    fj_colt *one[1] = {t};
    FJ_TRY(group_prepare(c, *c->group1, one, 1, 0));
    FJ_TRY(group_launch(c, *c->group1));
    return colt_force_all(c, t);
}

static fj_status check_relation(const fj_relation *r, int arity) {
    if (!r) return fail(FJ_ERR_ARG, "null relation");
    if (r->ncols != arity) return fail(FJ_ERR_ARG, "relation arity does not match the atom");
    if (r->nrows < 0 || r->nrows >= (int64_t(1) << 31)) return fail(FJ_ERR_UNSUPPORTED, "nrows must be below 2^31");
    for (int j = 0; j < arity; j++)
        if (!r->cols[j] && r->nrows > 0) return fail(FJ_ERR_ARG, "null column");
    if (r->sel && (r->nsel < 0 || r->nsel > r->nrows)) return fail(FJ_ERR_ARG, "nsel out of range");
    return FJ_OK;
}

namespace fj {
// Device buffers of freed COLTs and intermediates, kept per (device, size)
// for later allocations of the same size: a query's COLTs are allocated when
// built and freed after the run, and rebuilding the same query's COLTs then
// costs no hipMalloc.  At most kPoolMaxBytes are held; the rest is freed.
namespace {
constexpr size_t kPoolMaxBytes = size_t(4) << 30;
std::mutex g_pool_mu;
std::multimap<std::pair<int, size_t>, void *> g_pool;
size_t g_pool_held = 0;
}  // namespace

fj_status pool_alloc(int device, size_t bytes, void **out) {
    *out = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        auto it = g_pool.find({device, bytes});
        if (it != g_pool.end()) {
            *out = it->second;
            g_pool.erase(it);
            g_pool_held -= bytes;
            return FJ_OK;
        }
    }
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) {
        *out = nullptr;
        return fail(FJ_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return FJ_OK;
}

void pool_free(int device, void *p, size_t bytes) {
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        if (g_pool_held + bytes <= kPoolMaxBytes) {
            g_pool.insert({{device, bytes}, p});
            g_pool_held += bytes;
            return;
        }
    }
    hipFree(p);
}

hipStream_t ctx_stream(const fj_ctx *c) { return c->stream; }
int ctx_device(const fj_ctx *c) { return c->device; }
fj_status set_error(fj_status st, const std::string &msg) { return fail(st, msg); }
}  // namespace fj

extern "C" {

const char *fj_last_error(void) { return g_err.c_str(); }

fj_status fj_ctx_create(int device, void *stream, const fj_options *opt, fj_ctx **out) {
    if (!out) return fail(FJ_ERR_ARG, "null out");
    *out = nullptr;
    int ndev = 0;
    FJ_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(FJ_ERR_ARG, "no such device");
    FJ_HIP(hipSetDevice(device));
    fj_ctx *c = new fj_ctx();
    c->device = device;
    c->stream = (hipStream_t)stream;
    {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
            c->num_cus = prop.multiProcessorCount;
    }
    if (opt) c->opt = *opt;
    if (c->opt.tile <= 0) c->opt.tile = 1 << 24;
    if (c->opt.tile > (int64_t(1) << 30)) c->opt.tile = int64_t(1) << 30;
    if (c->opt.block <= 0) c->opt.block = 256;
    if (c->opt.block % 64 || c->opt.block > 1024) { delete c; return fail(FJ_ERR_ARG, "block must be a multiple of 64, at most 1024"); }
    hipError_t e = hipMalloc((void **)&c->status_d, sizeof(StatusDev));
    if (e != hipSuccess) { delete c; return fail(FJ_ERR_OOM, "status block"); }
    e = hipHostMalloc((void **)&c->status_h, sizeof(StatusDev), hipHostMallocDefault);
    if (e != hipSuccess) { hipFree(c->status_d); delete c; return fail(FJ_ERR_OOM, "pinned status block"); }
    memset(c->status_h, 0, sizeof(StatusDev));
    e = hipHostMalloc((void **)&c->ftotal_h, sizeof(uint32_t) * FJ_MAX_ATOMS,
                      hipHostMallocMapped | hipHostMallocCoherent);
    if (e != hipSuccess) { c->ftotal_h = nullptr; fj_ctx_destroy(c); return fail(FJ_ERR_OOM, "pinned selection counts"); }
    e = hipMemset(c->status_d, 0, sizeof(StatusDev));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { fj_ctx_destroy(c); return fail(FJ_ERR_HIP, "status block initialisation failed"); }
    if (fj::noalloc_scratch(device, &c->noalloc) != FJ_OK) {
        std::string keep = g_err;
        fj_ctx_destroy(c);
        return fail(FJ_ERR_HIP, keep);
    }
    *out = c;
    return FJ_OK;
}

void fj_ctx_destroy(fj_ctx *c) {
    if (!c) return;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    for (auto &b : c->front) b.release();
    for (auto &b : c->nodebuf) b.release();
    c->defer.release();
    c->force.release();
    c->scanb.release();
    c->desc.release();
    c->emitbuf.release();
    c->l0buf.release();
    c->chunkb.release();
    c->sketch.release();
    if (c->sketch_h) hipHostFree(c->sketch_h);
    destroy_group(c->group);
    destroy_group(c->group1);
    if (c->desc_h) hipHostFree(c->desc_h);
    if (c->desc_done) hipEventDestroy(c->desc_done);
    for (auto &p : c->pending) { hipEventDestroy(p.a); hipEventDestroy(p.b); }
    for (auto e : c->pool) hipEventDestroy(e);
    if (c->status_d) hipFree(c->status_d);
    if (c->status_h) hipHostFree(c->status_h);
    if (c->ftotal_h) hipHostFree(c->ftotal_h);
    delete c;
}

fj_status fj_timings(fj_ctx *c, double *ms, uint64_t *launches) {
    if (!c) return fail(FJ_ERR_ARG, "null ctx");
    FJ_HIP(hipStreamSynchronize(c->stream));
    for (auto &p : c->pending) {
        float m = 0;
        // (a pair a launch did not record, one that launched nothing, is skipped)
        if (hipEventElapsedTime(&m, p.a, p.b) == hipSuccess) {
            c->ms[p.cls] += m;
            c->launches[p.cls] += 1;
        } else {
            (void)hipGetLastError();
        }
        c->pool.push_back(p.a);
        c->pool.push_back(p.b);
    }
    c->pending.clear();
    for (int i = 0; i < FJ_T_COUNT; i++) {
        if (ms) ms[i] = c->ms[i];
        if (launches) launches[i] = c->launches[i];
    }
    return FJ_OK;
}

fj_status fj_timings_reset(fj_ctx *c) {
    if (!c) return fail(FJ_ERR_ARG, "null ctx");
    FJ_TRY(fj_timings(c, nullptr, nullptr));
    for (int i = 0; i < FJ_T_COUNT; i++) { c->ms[i] = 0; c->launches[i] = 0; }
    return FJ_OK;
}

fj_status fj_set_timing(fj_ctx *c, int32_t mode) {
    if (!c) return fail(FJ_ERR_ARG, "null ctx");
    if (mode < 0 || mode > 2) return fail(FJ_ERR_ARG, "timing mode is 0, 1 or 2");
    c->opt.timing = mode;
    return FJ_OK;
}

// ------------------------------------------------------------------- plans

fj_status fj_plan_from_binary(const fj_query *q, const int32_t *order, int32_t n, uint32_t flags,
                              fj_plan **out) {
    if (!q || !order || !out) return fail(FJ_ERR_ARG, "null argument");
    *out = nullptr;
    fj_plan *p = new fj_plan();
    std::string err;
    fj_status st = fj::plan_from_binary(*q, order, n, (flags & FJ_FACTOR) != 0, p, err);
    if (st != FJ_OK) { delete p; return fail(st, err); }
    *out = p;
    return FJ_OK;
}

fj_status fj_plan_from_nodes(const fj_query *q, int32_t nnodes, const int32_t *node_nsub, const int32_t *sub_atom,
                             const int32_t *sub_nvars, const int32_t *sub_vars, fj_plan **out) {
    if (!q || !node_nsub || !sub_atom || !sub_nvars || !sub_vars || !out) return fail(FJ_ERR_ARG, "null argument");
    *out = nullptr;
    if (nnodes < 1 || nnodes > FJ_MAX_NODES) return fail(FJ_ERR_UNSUPPORTED, "nnodes out of range");
    std::vector<std::vector<fj::Subatom>> nodes(nnodes);
    int idx = 0;
    for (int k = 0; k < nnodes; k++) {
        if (node_nsub[k] < 1 || node_nsub[k] > FJ_MAX_ATOMS) return fail(FJ_ERR_PLAN_INVALID, "bad node size");
        for (int s = 0; s < node_nsub[k]; s++, idx++) {
            fj::Subatom sa;
            sa.atom = sub_atom[idx];
            sa.nv = sub_nvars[idx];
            if (sa.nv < 0 || sa.nv > FJ_MAX_COLS) return fail(FJ_ERR_PLAN_INVALID, "bad subatom size");
            for (int j = 0; j < sa.nv; j++) {
                sa.vars[j] = sub_vars[idx * FJ_MAX_COLS + j];
                if (sa.vars[j] < 0 || sa.vars[j] >= FJ_MAX_VARS) return fail(FJ_ERR_PLAN_INVALID, "bad variable");
            }
            nodes[k].push_back(sa);
        }
    }
    fj_plan *p = new fj_plan();
    std::string err;
    fj_status st = fj::plan_from_nodes(*q, nodes, p, err);
    if (st != FJ_OK) { delete p; return fail(st, err); }
    *out = p;
    return FJ_OK;
}

fj_status fj_plan_get(const fj_plan *p, int32_t *nnodes, int32_t *node_nsub, int32_t *sub_atom,
                      int32_t *sub_nvars, int32_t *sub_vars, int32_t cap_sub) {
    if (!p || !nnodes || !node_nsub || !sub_atom || !sub_nvars || !sub_vars) return fail(FJ_ERR_ARG, "null argument");
    int idx = 0;
    *nnodes = (int32_t)p->nodes.size();
    for (size_t k = 0; k < p->nodes.size(); k++) {
        node_nsub[k] = (int32_t)p->nodes[k].size();
        for (const auto &s : p->nodes[k]) {
            if (idx >= cap_sub) return fail(FJ_ERR_ARG, "cap_sub too small");
            sub_atom[idx] = s.atom;
            sub_nvars[idx] = s.nv;
            for (int j = 0; j < FJ_MAX_COLS; j++) sub_vars[idx * FJ_MAX_COLS + j] = j < s.nv ? s.vars[j] : -1;
            idx++;
        }
    }
    return FJ_OK;
}

void fj_plan_free(fj_plan *p) { delete p; }

// --------------------------------------------------------------- selection

fj_status fj_filter_lt(fj_ctx *c, const int32_t *col, int64_t nrows, int32_t bound, uint32_t *out_sel,
                       int64_t *out_n) {
    if (!c || !out_n || nrows < 0 || (nrows > 0 && (!col || !out_sel))) return fail(FJ_ERR_ARG, "bad argument");
    if (nrows >= (int64_t(1) << 32)) return fail(FJ_ERR_UNSUPPORTED, "nrows must be below 2^32");
    FJ_HIP(hipSetDevice(c->device));
    *out_n = 0;
    if (nrows == 0) return FJ_OK;
    FJ_TRY(c->scanb.ensure(((u64)nrows / 1024 + 2) * sizeof(uint32_t), c->stream));
    {
        Timer t(c, FJ_T_FILTER);
        FJ_HIP(fj::launch_filter_lt(col, (u64)nrows, bound, out_sel, c->scanb.as<uint32_t>(),
                                    &c->status_d->total32, c->stream));
    }
    FJ_TRY(sync_status(c));
    *out_n = (int64_t)c->status_h->total32;
    return FJ_OK;
}

fj_status fj_filter_lt_noalloc(fj_ctx *c, const int32_t *col, int64_t nrows, int32_t bound, uint32_t *out_sel,
                               int64_t *out_n) {
    if (!c || !out_n || nrows < 0 || (nrows > 0 && (!col || !out_sel))) return fail(FJ_ERR_ARG, "bad argument");
    *out_n = 0;
    const u64 words = fj::noalloc_scratch_words();
    if (nrows > 0 && fj::filter_lt_blocks((u64)nrows) > words)
        return fail(FJ_ERR_UNSUPPORTED, "nrows above the allocation-free limit of " +
                                            std::to_string(words * 1024) + " rows");
    if (!c->noalloc) return fail(FJ_ERR_HIP, "the context has no scratch array");
    FJ_HIP(hipSetDevice(c->device));
    if (nrows == 0) return FJ_OK;
    // the block sums go to the fixed array and the total to the context's
    // status block; both are written before they are read, so nothing is
    // cleared first
    FJ_HIP(fj::launch_filter_lt(col, (u64)nrows, bound, out_sel, c->noalloc, &c->status_d->total32, c->stream));
    FJ_TRY(sync_status(c));
    *out_n = (int64_t)c->status_h->total32;
    return FJ_OK;
}

fj_status fj_filter_lt_batch(fj_ctx *c, int32_t n, const int32_t *const *cols, const int64_t *nrows,
                             const int32_t *bounds, uint32_t *const *outs, int64_t *counts) {
    if (!c || n < 0 || n > FJ_MAX_ATOMS || (n && (!cols || !nrows || !bounds || !outs || !counts)))
        return fail(FJ_ERR_ARG, "bad argument");
    FJ_HIP(hipSetDevice(c->device));
    size_t off[FJ_MAX_ATOMS + 1] = {0};
    for (int i = 0; i < n; i++) {
        if (nrows[i] < 0 || nrows[i] >= (int64_t(1) << 32)) return fail(FJ_ERR_ARG, "nrows out of range");
        if (nrows[i] > 0 && (!cols[i] || !outs[i])) return fail(FJ_ERR_ARG, "null buffer");
        off[i + 1] = off[i] + align256(((u64)nrows[i] / 1024 + 2) * sizeof(uint32_t));
    }
    FJ_TRY(c->scanb.ensure(off[n] + 256, c->stream));
    // (each non-empty selection's last block stores its total: no clearing)
    {
        // the non-empty selections in one grouped pass of two launches
        const int32_t *gc[FJ_MAX_ATOMS];
        u64 gr[FJ_MAX_ATOMS];
        int32_t gb[FJ_MAX_ATOMS];
        uint32_t *go[FJ_MAX_ATOMS], *gs[FJ_MAX_ATOMS], *gt[FJ_MAX_ATOMS];
        int m = 0;
        for (int i = 0; i < n; i++) {
            if (nrows[i] <= 0) continue;
            gc[m] = cols[i];
            gr[m] = (u64)nrows[i];
            gb[m] = bounds[i];
            go[m] = outs[i];
            gs[m] = c->scanb.as<uint32_t>(off[i]);
            gt[m] = &c->ftotal_h[i];
            m++;
        }
        Timer t(c, FJ_T_FILTER);
        FJ_HIP(fj::launch_filter_lt_group(m, gc, gr, gb, go, gs, gt, c->stream));
    }
    // the totals land in mapped host memory: no copy, only the wait
    FJ_HIP(hipStreamSynchronize(c->stream));
    const volatile uint32_t *ft = c->ftotal_h;
    for (int i = 0; i < n; i++) counts[i] = nrows[i] > 0 ? (int64_t)ft[i] : 0;
    return FJ_OK;
}

// ------------------------------------------------------------------- COLTs

fj_status fj_sketch_relation(fj_ctx *c, const fj_relation *rel, fj_sketch *out) {
    if (!c || !rel || !out) return fail(FJ_ERR_ARG, "null argument");
    if (rel->ncols < 1 || rel->ncols > FJ_MAX_COLS) return fail(FJ_ERR_ARG, "relation arity out of range");
    if (rel->nrows < 0 || rel->nrows >= (int64_t(1) << 31)) return fail(FJ_ERR_ARG, "nrows out of range");
    const bool use_sel = rel->sel != nullptr;
    const int64_t n = use_sel ? rel->nsel : rel->nrows;
    if (n < 0 || n > rel->nrows) return fail(FJ_ERR_ARG, "nsel out of range");
    for (int j = 0; j < rel->ncols; j++)
        if (n && !rel->cols[j]) return fail(FJ_ERR_ARG, "null column");
    FJ_HIP(hipSetDevice(c->device));
    memset(out, 0, sizeof(*out));
    out->rows = n;
    out->ncols = rel->ncols;
    // table of at least twice the rows, so linear probing always ends
    uint64_t cap = 256;
    while (cap < 2 * (uint64_t)n) cap <<= 1;
    const uint32_t max_blocks = 2048;
    const size_t o_cnt = align256(cap * 4), o_part = o_cnt + align256(cap * 4),
                 o_res = o_part + align256(size_t(max_blocks) * fj::kSketchTop * 4),
                 total = o_res + align256(fj::kSketchRes * 8);
    FJ_TRY(c->sketch.ensure(total, c->stream));
    if (!c->sketch_h) {
        hipError_t e = hipHostMalloc((void **)&c->sketch_h, fj::kSketchRes * 8 * FJ_MAX_COLS, hipHostMallocDefault);
        if (e != hipSuccess) { c->sketch_h = nullptr; return fail(FJ_ERR_OOM, "pinned sketch results"); }
    }
    for (int j = 0; j < rel->ncols; j++) {
        fj::SketchLaunch a{};
        a.col = rel->cols[j];
        a.sel = use_sel ? rel->sel : nullptr;
        a.n = (uint32_t)n;
        a.keys = c->sketch.as<uint32_t>(0);
        a.cnt = c->sketch.as<uint32_t>(o_cnt);
        a.mask = (uint32_t)(cap - 1);
        a.part = c->sketch.as<uint32_t>(o_part);
        a.max_blocks = max_blocks;
        a.res = c->sketch.as<unsigned long long>(o_res);
        FJ_HIP(fj::launch_sketch(a, c->stream));
        FJ_HIP(hipMemcpyAsync(c->sketch_h + j * fj::kSketchRes, a.res, fj::kSketchRes * 8, hipMemcpyDeviceToHost,
                              c->stream));
    }
    FJ_HIP(hipStreamSynchronize(c->stream));
    for (int j = 0; j < rel->ncols; j++) {
        const unsigned long long *r = c->sketch_h + j * fj::kSketchRes;
        out->distinct[j] = (int64_t)r[fj::kSkDistinct];
        for (int k = 0; k < FJ_SKETCH_TOPK; k++) out->top[j][k] = (int64_t)r[fj::kSkTop + k];
    }
    return FJ_OK;
}

// Whether a node of the plan iterates atom a's root (its level-0 subatom is
// a pure cover of the node), or the simple trie forces the root's children
// up front: then a built root lists its keys by rank as well as its map.
static bool root_needs_keys(const fj_ctx *c, const fj_plan *p, int a) {
    if (c->opt.trie == 2 && p->nlev[a] > 1) return true;
    for (size_t k = 0; k < p->nodes.size(); k++)
        for (int i : p->layout[k].pure)
            if (p->nodes[k][i].atom == a && p->sub_level[k][i] == 0) return true;
    return false;
}

fj_status fj_build_colt(fj_ctx *c, const fj_query *q, const fj_plan *p, int32_t atom, const fj_relation *rel,
                        fj_colt **out) {
    if (!c || !q || !p || !out) return fail(FJ_ERR_ARG, "null argument");
    *out = nullptr;
    if (atom < 0 || atom >= q->natoms || atom >= p->q.natoms) return fail(FJ_ERR_ARG, "atom out of range");
    FJ_TRY(check_relation(rel, q->atoms[atom].arity));
    FJ_HIP(hipSetDevice(c->device));
    fj_colt *t = new fj_colt();
    t->device = c->device;
    t->atom = atom;
    t->ncols = rel->ncols;
    for (int j = 0; j < rel->ncols; j++) t->cols[j] = rel->cols[j];
    t->sel = rel->sel;
    t->nrows = rel->nrows;
    t->nroot = (uint32_t)(rel->sel ? rel->nsel : rel->nrows);
    t->cap_rows = t->nroot;
    // the ablation's tries build every root map ahead
    t->root_built = p->root_built[atom] || c->opt.trie >= 1;
    t->root_lazy = !t->root_built && p->root_lazy[atom];
    t->root_keys = root_needs_keys(c, p, atom);
    t->nlev = p->nlev[atom];
    for (int l = 0; l < t->nlev; l++) {
        const fj::Subatom &s = p->lev[atom][l];
        t->lev_nk[l] = s.nv;
        for (int j = 0; j < s.nv; j++) t->lev_var[l][j] = s.vars[j];
    }
    fj_status st = colt_allocate(t);
    if (st == FJ_OK) {
        // key columns of every level
        for (int l = 0; l < t->nlev; l++)
            for (int j = 0; j < t->lev_nk[l]; j++)
                for (int cc = 0; cc < q->atoms[atom].arity; cc++)
                    if (q->atoms[atom].vars[cc] == t->lev_var[l][j]) t->lev[l].kcol[j] = cc;
        st = colt_reset(c, t);
        if (st == FJ_OK) st = sync_status(c);
    }
    if (st != FJ_OK) {
        std::string keep = g_err;
        hipStreamSynchronize(c->stream);
        colt_free_all(t);
        delete t;
        g_err = keep;
        return st;
    }
    *out = t;
    return FJ_OK;
}

fj_status fj_colt_rebuild(fj_ctx *c, fj_colt *t, const fj_relation *rel) {
    if (!c || !t || !rel) return fail(FJ_ERR_ARG, "null argument");
    FJ_TRY(check_relation(rel, t->ncols));
    uint32_t nroot = (uint32_t)(rel->sel ? rel->nsel : rel->nrows);
    if (nroot > t->cap_rows) return fail(FJ_ERR_ARG, "relation grew beyond the COLT's capacity");
    FJ_HIP(hipSetDevice(c->device));
    for (int j = 0; j < rel->ncols; j++) t->cols[j] = rel->cols[j];
    t->sel = rel->sel;
    t->nrows = rel->nrows;
    t->nroot = nroot;
    return colt_reset(c, t);
}

fj_status fj_colt_rebuild_many(fj_ctx *c, int32_t n, fj_colt *const *colts, const fj_relation *rels) {
    if (!c || n < 0 || (n > 0 && (!colts || !rels))) return fail(FJ_ERR_ARG, "null argument");
    if (n == 0) return FJ_OK;
    for (int k = 0; k < n; k++) {
        if (!colts[k]) return fail(FJ_ERR_ARG, "null COLT");
        FJ_TRY(check_relation(&rels[k], colts[k]->ncols));
        const uint32_t nroot = (uint32_t)(rels[k].sel ? rels[k].nsel : rels[k].nrows);
        if (nroot > colts[k]->cap_rows) return fail(FJ_ERR_ARG, "relation grew beyond the COLT's capacity");
        if (colts[k]->device != c->device) return fail(FJ_ERR_ARG, "COLT of another device");
    }
    for (int k = 0; k < n; k++)
        for (int j = k + 1; j < n; j++)
            if (colts[k] == colts[j]) return fail(FJ_ERR_ARG, "a COLT is listed twice");
    FJ_HIP(hipSetDevice(c->device));
    for (int k = 0; k < n; k++) {
        fj_colt *t = colts[k];
        const fj_relation &r = rels[k];
        for (int j = 0; j < r.ncols; j++) t->cols[j] = r.cols[j];
        t->sel = r.sel;
        t->nrows = r.nrows;
        t->nroot = (uint32_t)(r.sel ? r.nsel : r.nrows);
        FJ_TRY(colt_size(t));
        FJ_TRY(colt_fill_upload(c, t));
    }
    if (!c->group) c->group = new ColtGroup();
    FJ_TRY(group_prepare(c, *c->group, colts, n, 0));
    FJ_TRY(group_launch(c, *c->group));
    for (int k = 0; k < n; k++) FJ_TRY(colt_force_all(c, colts[k]));
    return FJ_OK;
}

fj_status fj_select_rebuild(fj_ctx *c, int32_t nsel, const int32_t *atoms, const int32_t *cols,
                            const int32_t *bounds, int32_t n, fj_colt *const *colts, fj_relation *rels) {
    if (!c || nsel < 0 || nsel > FJ_MAX_ATOMS || n < 0 || (nsel && (!atoms || !cols || !bounds)) ||
        (n && (!colts || !rels)))
        return fail(FJ_ERR_ARG, "bad argument");
    const int32_t *cp[FJ_MAX_ATOMS];
    int64_t nr[FJ_MAX_ATOMS], cnt[FJ_MAX_ATOMS];
    uint32_t *outs[FJ_MAX_ATOMS];
    for (int i = 0; i < nsel; i++) {
        const int a = atoms[i];
        if (a < 0 || a >= n) return fail(FJ_ERR_ARG, "selection atom out of range");
        for (int j = 0; j < i; j++)
            if (atoms[j] == a) return fail(FJ_ERR_ARG, "an atom is selected twice");
        const fj_relation &r = rels[a];
        if (cols[i] < 0 || cols[i] >= r.ncols || r.ncols > FJ_MAX_COLS)
            return fail(FJ_ERR_ARG, "selection column out of range");
        if (r.nrows > 0 && !r.sel) return fail(FJ_ERR_ARG, "a selected relation needs its selection buffer");
        cp[i] = r.cols[cols[i]];
        nr[i] = r.nrows;
        outs[i] = const_cast<uint32_t *>(r.sel);
    }
    if (nsel) FJ_TRY(fj_filter_lt_batch(c, nsel, cp, nr, bounds, outs, cnt));
    for (int i = 0; i < nsel; i++) rels[atoms[i]].nsel = cnt[i];
    return fj_colt_rebuild_many(c, n, colts, rels);
}

void fj_colt_free(fj_colt *t) {
    if (!t) return;
    hipSetDevice(t->device);
    hipDeviceSynchronize();
    colt_free_all(t);
    delete t;
}

}  // extern "C"

// --------------------------------------------------------------------- join

namespace {

struct Exec {
    fj_ctx *c;
    const fj_plan *p;
    fj_colt *const *colts;
    int32_t *out;
    u64 cap;
    u64 written = 0;
    fj_stats *stats;
    int tail_from;
    int nnodes;
    u64 C;                              // tile / frontier capacity
    FrontierDev F[FJ_MAX_NODES + 1];
    NodeDev *nd_d = nullptr;            // device node descriptors
    void *emit_d = nullptr;             // device emit descriptor
    std::vector<TailDev> tails;
    std::vector<int> head_src;
    uint32_t *dA = nullptr, *dB = nullptr;
    uint8_t *dA_j = nullptr, *dB_j = nullptr;
    fj_result *res = nullptr;           // factorized: keep the final bindings instead of rows
    bool emit_pending = false;          // the last scan tile's emit was enqueued before its count was known
    u64 emit_pending_base = 0;          // the survivor counter before that tile
};

void fill_level_sub(SubDev &S, const fj_colt *t, int level) {
    S.L = t->lev[level];
    S.C = t->lev[level + 1];
    for (int j = 0; j < FJ_MAX_COLS; j++) S.cols[j] = t->cols[j];
    S.root_len = t->nroot;
}

fj_status force_pending_queues(Exec &x, int node, const std::vector<std::pair<int, int>> &queues) {
    fj_ctx *c = x.c;
    bool any = false;
    for (auto &al : queues) {
        int a = al.first, l = al.second;
        uint32_t nh = c->status_h->fq_n[a * fj::kMaxLevels + l];
        if (!nh) continue;
        any = true;
        FJ_TRY(force_queue(c, x.colts[a], l, nh, ~0ull, FJ_T_FORCE, x.stats, node));
    }
    if (any) FJ_TRY(zero_status_field(c, offsetof(StatusDev, fq_n), sizeof(c->status_h->fq_n)));
    return FJ_OK;
}

fj_status emit_rows(Exec &x, uint32_t E) {
    // materialize the result rows of E final bindings in frontier F[tail_from]
    // the emit's place in the output is decided on the device, so no wait
    // here; the host copy of the status is as fresh as the caller's last
    // sync, which came after every earlier emit
    fj_ctx *c = x.c;
    x.written = c->status_h->written;
    if (!x.out || E == 0 || x.written >= x.cap) return FJ_OK;
    u64 *cnt = c->emitbuf.as<u64>();
    u64 *starts = c->emitbuf.as<u64>(align256(sizeof(u64) * x.C));
    if (E <= fj::emit_small_max()) {
        // few bindings: counts, scan and placement in one launch
        Timer t(c, FJ_T_EMIT);
        FJ_HIP(fj::launch_emit_count_small(x.emit_d, E, starts, c->status_d, x.cap, c->stream));
    } else {
        {
            Timer t(c, FJ_T_EMIT);
            FJ_HIP(fj::launch_emit_count(x.emit_d, E, cnt, c->status_d, c->stream));
        }
        size_t nb = (E + 1023) / 1024 + 1;
        FJ_TRY(c->scanb.ensure(nb * sizeof(u64), c->stream));
        Timer t(c, FJ_T_SCAN);
        FJ_HIP(fj::launch_scan_u64_emit(cnt, starts, E, c->scanb.as<u64>(), c->status_d, x.cap, c->stream));
    }
    {
        Timer t(c, FJ_T_EMIT);
        FJ_HIP(fj::launch_emit_rows(x.emit_d, E, starts, x.cap - x.written, c->status_d, c->stream));
    }
    return FJ_OK;
}

}  // namespace

// A factorized result (fj_execute_factorized): the final bindings (values,
// handles and multiplicities, structure of arrays of capacity cap, in one
// pooled buffer) with what expanding them into rows needs.
struct fj_result {
    int device = 0;
    int nvals = 0, nhdl = 0;
    u64 E = 0, cap = 0;
    void *buf = nullptr;
    size_t bytes = 0;
    int32_t *vals = nullptr;
    uint32_t *hdl = nullptr;
    u64 *mult = nullptr;
    u64 count = 0;
    std::vector<int> in_var, in_hatom, head_src;
    std::vector<TailDev> tails;
    u64 *starts = nullptr;      // E + 1 scanned row counts, once expanded
    size_t starts_bytes = 0;
    void *emit_d = nullptr;     // device emit descriptor
    std::vector<char> emit_h;   // its host copy
    ~fj_result() {
        fj::pool_free(device, buf, bytes);
        fj::pool_free(device, starts, starts_bytes);
        fj::pool_free(device, emit_d, fj::emit_dev_size());
    }
};

namespace {

// Room for `want` bindings, keeping those held (the caller's stream orders
// the copies; the old buffer is freed once they are done).
fj_status result_reserve(fj_ctx *c, fj_result *r, u64 want) {
    if (want <= r->cap) return FJ_OK;
    const u64 ncap = std::max<u64>(std::max<u64>(want, 2 * r->cap), 1024);
    const size_t bv = align256(sizeof(int32_t) * ncap * r->nvals), bh = align256(sizeof(uint32_t) * ncap * r->nhdl);
    const size_t bytes = bv + bh + align256(sizeof(u64) * ncap);
    void *nb = nullptr;
    FJ_TRY(fj::pool_alloc(r->device, bytes, &nb));
    int32_t *nv = (int32_t *)nb;
    uint32_t *nh = (uint32_t *)((char *)nb + bv);
    u64 *nm = (u64 *)((char *)nb + bv + bh);
    if (r->E) {
        for (int j = 0; j < r->nvals; j++)
            FJ_HIP(hipMemcpyAsync(nv + j * ncap, r->vals + j * r->cap, sizeof(int32_t) * r->E,
                                  hipMemcpyDeviceToDevice, c->stream));
        for (int j = 0; j < r->nhdl; j++)
            FJ_HIP(hipMemcpyAsync(nh + j * ncap, r->hdl + j * r->cap, sizeof(uint32_t) * r->E,
                                  hipMemcpyDeviceToDevice, c->stream));
        FJ_HIP(hipMemcpyAsync(nm, r->mult, sizeof(u64) * r->E, hipMemcpyDeviceToDevice, c->stream));
        FJ_HIP(hipStreamSynchronize(c->stream));
    }
    fj::pool_free(r->device, r->buf, r->bytes);
    r->buf = nb;
    r->bytes = bytes;
    r->vals = nv;
    r->hdl = nh;
    r->mult = nm;
    r->cap = ncap;
    return FJ_OK;
}

// The E final bindings of the current tile (frontier F[tail_from]) join the
// factorized result.
fj_status result_keep(Exec &x, uint32_t E) {
    fj_ctx *c = x.c;
    fj_result *r = x.res;
    if (E == 0) return FJ_OK;
    if (r->E + E > 0xFFFFFFFFull) return fail(FJ_ERR_UNSUPPORTED, "a factorized result holds 2^32 bindings or more");
    FJ_TRY(result_reserve(c, r, r->E + E));
    const FrontierDev &F = x.F[x.tail_from];
    for (int j = 0; j < r->nvals; j++)
        FJ_HIP(hipMemcpyAsync(r->vals + j * r->cap + r->E, F.vals + j * F.cap, sizeof(int32_t) * E,
                              hipMemcpyDeviceToDevice, c->stream));
    for (int j = 0; j < r->nhdl; j++)
        FJ_HIP(hipMemcpyAsync(r->hdl + j * r->cap + r->E, F.hdl + j * F.cap, sizeof(uint32_t) * E,
                              hipMemcpyDeviceToDevice, c->stream));
    if (F.mult) {
        FJ_HIP(hipMemcpyAsync(r->mult + r->E, F.mult, sizeof(u64) * E, hipMemcpyDeviceToDevice, c->stream));
    } else {
        // the single empty binding of a plan that is all products
        static const u64 one = 1;
        FJ_HIP(hipMemcpyAsync(r->mult + r->E, &one, sizeof(u64), hipMemcpyHostToDevice, c->stream));
        FJ_HIP(hipStreamSynchronize(c->stream));
    }
    r->E += E;
    return FJ_OK;
}

// A tile's final bindings: expanded into rows, kept factorized, or (count
// only) dropped.
fj_status emit_or_keep(Exec &x, uint32_t E) {
    if (x.res) return result_keep(x, E);
    if (x.out) return emit_rows(x, E);
    return FJ_OK;
}

// The first node can use the specialised scan-probe kernel when its only
// pure cover is a base table iterated directly and every other subatom
// probes a root map keyed by one or two cover columns.
bool scan_eligible(const Exec &x, int &cover_sub) {
    const fj_plan *p = x.p;
    if (x.tail_from < 1) return false;
    const auto &L = p->layout[0];
    if (L.pure.size() != 1) return false;
    cover_sub = L.pure[0];
    const auto &node = p->nodes[0];
    int ca = node[cover_sub].atom;
    if (x.colts[ca]->root_built || p->nlev[ca] != 1) return false;
    int nl = 0;
    for (size_t i = 0; i < node.size(); i++) {
        if ((int)i == cover_sub) continue;
        const fj_colt *t = x.colts[node[i].atom];
        const LevelDev &R = t->lev[0];
        if (p->sub_level[0][i] != 0 || !x.colts[node[i].atom]->root_built) return false;
        if (!(R.mode == fj::KM_K32 || (R.mode == fj::KM_K64 && R.nk == 2))) return false;
        nl++;
    }
    if (nl > fj::scan_max_lookups()) return false;
    for (int q = 0; q < (int)x.tails.size(); q++)
        if (x.tails[q].level > 1) return false;
    return true;
}

fj_status exec_scan_node(Exec &x, int cover_sub, u64 T, uint32_t r0_limit);

fj_status exec_node(Exec &x, int k, uint32_t E) {
    fj_ctx *c = x.c;
    int cover_sub = -1;
    if (k == 0 && !c->opt.generic && scan_eligible(x, cover_sub)) {
        const fj_colt *ct = x.colts[x.p->nodes[0][cover_sub].atom];
        return exec_scan_node(x, cover_sub, ct->nroot, 0);
    }
    const NodeDev *nd = x.nd_d + k;
    const fj_plan *p = x.p;
    u64 *starts = c->nodebuf[k].as<u64>(0);
    u64 *cnt = c->nodebuf[k].as<u64>(align256(sizeof(u64) * (x.C + 1)));
    uint8_t *cov = c->nodebuf[k].as<uint8_t>(align256(sizeof(u64) * (x.C + 1)) + align256(sizeof(u64) * x.C));
    // queues this node can fill: its subatoms' (atom, level)
    std::vector<std::pair<int, int>> queues;
    for (size_t i = 0; i < p->nodes[k].size(); i++) queues.push_back({p->nodes[k][i].atom, p->sub_level[k][i]});

    const uint32_t pend_base = c->status_h->pending;
    {
        Timer t(c, FJ_T_COVER);
        FJ_HIP(fj::launch_cover_choose(nd, E, cov, cnt, c->status_d, c->stream));
    }
    FJ_TRY(scan_u64(c, cnt, starts, E));
    FJ_TRY(sync_status(c));
    if (c->status_h->pending != pend_base) {
        FJ_TRY(force_pending_queues(x, k, queues));
        {
            Timer t(c, FJ_T_COVER);
            FJ_HIP(fj::launch_cover_fill(nd, E, cov, cnt, c->status_d, c->stream));
        }
        FJ_TRY(scan_u64(c, cnt, starts, E));
        FJ_TRY(sync_status(c));
    }
    const u64 T = c->status_h->total;
    if (x.stats) x.stats->cover[k] += T;
    const bool emit = (k == x.tail_from - 1);
    for (u64 t0 = 0; t0 < T; t0 += x.C) {
        uint32_t n = (uint32_t)std::min<u64>(x.C, T - t0);
        // counters never reset: entries of this tile start at their bases
        const u64 surv_base = c->status_h->survivors;
        u64 def_base = c->status_h->deferred;
        fj::ProbeLaunch pl;
        pl.nd = nd;
        pl.starts = starts;
        pl.cov = cov;
        pl.E = E;
        pl.t0 = t0;
        pl.n = n;
        pl.din = nullptr;
        pl.din_j = nullptr;
        pl.dout = x.dA;
        pl.dout_j = x.dA_j;
        pl.status = c->status_d;
        pl.count_stats = x.stats != nullptr;
        pl.block = c->opt.block;
        pl.dcap = (uint32_t)x.C;
        pl.surv_base = surv_base;
        pl.def_base = def_base;
        {
            const u64 need = (u64)n / 64 + 2;   // blocks of at least 64 threads, plus the sentinel
            FJ_TRY(c->chunkb.ensure(need * sizeof(uint32_t), c->stream));
            pl.chunk_buf = c->chunkb.as<uint32_t>();
            pl.chunk_cap = c->chunkb.bytes / sizeof(uint32_t);
            pl.max_slots = p->q.nvars;
            pl.max_atoms = p->q.natoms;
        }
        {
            Timer t(c, k == 0 ? FJ_T_PROBE0 : FJ_T_PROBE);
            FJ_HIP(fj::launch_probe(pl, c->stream));
        }
        if (x.stats) x.stats->tiles++;
        FJ_TRY(sync_status(c));
        uint32_t *din = x.dA, *dout = x.dB;
        uint8_t *din_j = x.dA_j, *dout_j = x.dB_j;
        int rounds = 0;
        while (c->status_h->deferred != def_base) {
            // each round forces the tries the deferred tuples met, so a tuple
            // advances by at least one lookup per round
            if (++rounds > (int)p->nodes[k].size() + 1)
                return fail(FJ_ERR_INTERNAL, "lazy forcing made no progress");
            uint32_t nd_n = (uint32_t)(c->status_h->deferred - def_base);
            def_base = c->status_h->deferred;
            if (x.stats) x.stats->deferred += nd_n;
            FJ_TRY(force_pending_queues(x, k, queues));
            pl.din = din;
            pl.din_j = din_j;
            pl.dout = dout;
            pl.dout_j = dout_j;
            pl.n = nd_n;
            pl.def_base = def_base;
            {
                Timer t(c, FJ_T_PROBE);
                FJ_HIP(fj::launch_probe(pl, c->stream));
            }
            FJ_TRY(sync_status(c));
            std::swap(din, dout);
            std::swap(din_j, dout_j);
        }
        const uint32_t surv = (uint32_t)(c->status_h->survivors - surv_base);
        if (x.stats && !emit) x.stats->survivors[k] += surv;
        if (emit) {
            FJ_TRY(emit_or_keep(x, surv));
        } else if (surv) {
            FJ_TRY(exec_node(x, k + 1, surv));
        }
    }
    return FJ_OK;
}

fj_status exec_scan_node(Exec &x, int cover_sub, u64 T, uint32_t) {
    fj_ctx *c = x.c;
    const fj_plan *p = x.p;
    const auto &node = p->nodes[0];
    const fj_colt *ct = x.colts[node[cover_sub].atom];
    const fj::Subatom &cs = node[cover_sub];
    fj::ScanLaunch sl;
    memset(&sl, 0, sizeof(sl));
    for (int j = 0; j < FJ_MAX_COLS; j++) sl.cols[j] = ct->cols[j];
    sl.ncols = ct->ncols;
    sl.sel = ct->sel;
    sl.nrows = (uint32_t)ct->nrows;
    auto cover_col = [&](int var) {
        for (int j = 0; j < cs.nv; j++)
            if (cs.vars[j] == var) return ct->lev[0].kcol[j];
        return -1;
    };
    const auto &LN = p->layout[1];
    for (size_t i = 0; i < node.size(); i++) {
        if ((int)i == cover_sub) continue;
        const int a = node[i].atom;
        const fj_colt *t = x.colts[a];
        fj::ScanLookup &L = sl.lk[sl.nl++];
        L.table = t->lev[0].table;
        L.mask = t->lev[0].mask;
        L.mode = t->lev[0].mode;
        for (int j = 0; j < node[i].nv; j++) L.kc[j] = cover_col(node[i].vars[j]);
        L.child_leaf = p->nlev[a] == 1;
        L.clen = t->lev[1].len;
        L.cnpos = t->lev[1].npos;
        L.hcol = -1;
        for (size_t h = 0; h < LN.in_hatom.size(); h++)
            if (LN.in_hatom[h] == a) L.hcol = (int)h;
        L.bloom = nullptr;
        L.bloom_shift = 0;
        L.bloom_words = 0;
        if (sl.nl == 1 && !c->opt.no_filter && L.mode == fj::KM_K32 && t->lev[0].bloom) {
            // the first lookup's key filter, when its words hold few keys
            // (two bits each of 32: at most 12 keys a word on average)
            const u64 words = (L.mask + 1) >> (2 + t->lev[0].bloom_shift);
            if (words >= 1 && words <= fj::kBloomWords && (u64)t->nroot <= 12 * words) {
                L.bloom = t->lev[0].bloom;
                L.bloom_shift = t->lev[0].bloom_shift;
                L.bloom_words = (uint32_t)words;
            }
        }
    }
    if (sl.nl >= 1 && sl.lk[0].bloom) {
        // the list of first-lookup hits the filter pass hands to the rounds
        const u64 ent = fj::scan_list_entries(std::min<u64>(x.C, T));
        const size_t rb = align256(sizeof(uint32_t) * ent);
        FJ_TRY(c->l0buf.ensure(2 * rb + sizeof(uint32_t) * fj::kScanListGroups * fj::kScanListWaves, c->stream));
        sl.l0_row = c->l0buf.as<uint32_t>();
        sl.l0_key = c->l0buf.as<uint32_t>(rb);
        sl.l0_cnt = c->l0buf.as<uint32_t>(2 * rb);
        sl.l0_cap = ent;
    }
    sl.nout = (int)LN.in_var.size();
    for (int j = 0; j < sl.nout; j++) sl.out_col[j] = cover_col(LN.in_var[j]);
    sl.out = x.F[1];
    sl.emit = x.tail_from == 1;
    // rows wanted from the first node: the kernel writes them itself
    sl.direct = sl.emit && x.out && !x.res;
    sl.ed = x.emit_d;
    sl.cap = x.cap;
    sl.materialize = sl.emit && !sl.direct && (x.out != nullptr || x.res != nullptr);
    if (sl.emit) {
        sl.ntail = (int)x.tails.size();
        for (int q = 0; q < sl.ntail; q++) {
            const TailDev &Td = x.tails[q];
            sl.tail_lk[q] = -1;
            sl.tail_root_len[q] = Td.root_len;
            sl.tail_len[q] = Td.L.len;
            sl.tail_npos[q] = Td.L.npos;
            if (Td.level == 1) {
                int j = 0;
                for (size_t i = 0; i < node.size(); i++) {
                    if ((int)i == cover_sub) continue;
                    if (node[i].atom == Td.atom) sl.tail_lk[q] = j;
                    j++;
                }
                if (sl.tail_lk[q] < 0) return fail(FJ_ERR_INTERNAL, "tail trie not reached by the first node");
            }
        }
    }
    sl.status = c->status_d;
    sl.count_stats = x.stats != nullptr;
    sl.node = 0;
    if (x.stats) x.stats->cover[0] += T;
    for (u64 t0 = 0; t0 < T; t0 += x.C) {
        uint32_t n = (uint32_t)std::min<u64>(x.C, T - t0);
        const u64 surv_base = c->status_h->survivors;
        sl.r0 = (uint32_t)t0;
        sl.n = n;
        sl.surv_base = surv_base;
        {
            Timer t(c, FJ_T_PROBE0, true);
            sl.t_start = t.a;
            sl.t_stop = t.b;
            FJ_HIP(fj::launch_scan_probe(sl, c->stream));
        }
        if (x.stats) x.stats->tiles++;
        if (sl.direct) continue;   // rows and count land on the device; no wait per tile
        if (sl.emit && x.out && !x.res && t0 + n >= T) {
            // the last tile's rows: emitted on the device without a wait for
            // its survivor count when the bindings are few (one workgroup);
            // the host finishes a larger emit after its final wait
            u64 *starts = c->emitbuf.as<u64>(align256(sizeof(u64) * x.C));
            Timer t(c, FJ_T_EMIT);
            FJ_HIP(fj::launch_emit_small_dev(x.emit_d, &c->status_d->survivors, surv_base, starts, c->status_d,
                                             x.cap, c->stream));
            x.emit_pending = true;
            x.emit_pending_base = surv_base;
            break;
        }
        FJ_TRY(sync_status(c));
        const uint32_t surv = (uint32_t)(c->status_h->survivors - surv_base);
        if (sl.emit) {
            FJ_TRY(emit_or_keep(x, surv));
        } else {
            if (x.stats) x.stats->survivors[0] += surv;
            if (surv) FJ_TRY(exec_node(x, 1, surv));
        }
    }
    return FJ_OK;
}

fj_status check_exec_args(const fj_ctx *c, const fj_query *q, const fj_plan *p, fj_colt *const *colts) {
    if (q->natoms != p->q.natoms || q->nvars != p->q.nvars) return fail(FJ_ERR_ARG, "query does not match the plan");
    for (int a = 0; a < q->natoms; a++) {
        if (q->atoms[a].arity != p->q.atoms[a].arity ||
            memcmp(q->atoms[a].vars, p->q.atoms[a].vars, sizeof(int32_t) * q->atoms[a].arity) != 0)
            return fail(FJ_ERR_ARG, "query does not match the plan");
        const fj_colt *t = colts[a];
        if (!t) return fail(FJ_ERR_ARG, "null COLT");
        if (t->atom != a || t->nlev != p->nlev[a]) return fail(FJ_ERR_ARG, "COLT was built for another atom or plan");
        for (int l = 0; l < t->nlev; l++) {
            if (t->lev_nk[l] != p->lev[a][l].nv) return fail(FJ_ERR_ARG, "COLT schema does not match the plan");
            for (int j = 0; j < t->lev_nk[l]; j++)
                if (t->lev_var[l][j] != p->lev[a][l].vars[j]) return fail(FJ_ERR_ARG, "COLT schema does not match the plan");
        }
        if (p->root_built[a] && !t->root_built) return fail(FJ_ERR_ARG, "COLT root rule does not match the plan");
        if (p->root_lazy[a] && !t->root_built && !t->root_lazy)
            return fail(FJ_ERR_ARG, "COLT root rule does not match the plan");
        if (t->root_built && !t->root_keys && root_needs_keys(c, p, a))
            return fail(FJ_ERR_ARG, "COLT was built for a plan that only probes its root; this plan iterates it");
    }
    std::string err;
    return fj::check_query(*q, err) == FJ_OK ? FJ_OK : fail(FJ_ERR_ARG, err);
}

}  // namespace

static fj_status execute_impl(fj_ctx *c, const fj_query *q, const fj_plan *p, fj_colt *const *colts,
                              uint64_t *count, int32_t *out, uint64_t cap, uint64_t *written, fj_stats *stats,
                              fj_result *res) {
    if (!c || !q || !p || !colts || !count) return fail(FJ_ERR_ARG, "null argument");
    FJ_TRY(check_exec_args(c, q, p, colts));
    FJ_HIP(hipSetDevice(c->device));
    if (stats) memset(stats, 0, sizeof(*stats));
    Exec x;
    x.c = c;
    x.p = p;
    x.colts = colts;
    x.out = cap ? out : nullptr;
    x.cap = out ? cap : 0;
    x.stats = stats;
    x.res = res;
    x.nnodes = (int)p->nodes.size();
    x.tail_from = c->opt.tail == 1 ? x.nnodes : p->tail_from;
    x.C = (u64)c->opt.tile;
    if (stats) { stats->tail_from = x.tail_from; stats->nnodes = x.nnodes; }

    // frontier buffers: F[0] is the single empty binding
    for (int k = 0; k <= x.tail_from; k++) {
        const auto &L = p->layout[k];
        FrontierDev &F = x.F[k];
        memset(&F, 0, sizeof(F));
        F.nvals = (int)L.in_var.size();
        F.nhdl = (int)L.in_hatom.size();
        F.cap = k == 0 ? 1 : x.C;
        if (k == 0) continue;
        size_t bv = align256(sizeof(int32_t) * F.cap * F.nvals);
        size_t bh = align256(sizeof(uint32_t) * F.cap * F.nhdl);
        size_t bm = align256(sizeof(u64) * F.cap);
        FJ_TRY(c->front[k].ensure(bv + bh + bm, c->stream));
        F.vals = c->front[k].as<int32_t>(0);
        F.hdl = c->front[k].as<uint32_t>(bv);
        F.mult = c->front[k].as<u64>(bv + bh);
    }
    for (int k = 0; k < x.tail_from; k++) {
        u64 E = k == 0 ? 1 : x.C;
        size_t b = align256(sizeof(u64) * (E + 1)) + align256(sizeof(u64) * E) + align256(E);
        b = std::max(b, align256(sizeof(u64) * (x.C + 1)) + align256(sizeof(u64) * x.C) + align256(x.C));
        FJ_TRY(c->nodebuf[k].ensure(b, c->stream));
    }
    size_t dl = align256(sizeof(uint32_t) * x.C);
    size_t dj = align256(x.C);
    FJ_TRY(c->defer.ensure(2 * (dl + dj), c->stream));
    x.dA = c->defer.as<uint32_t>(0);
    x.dB = c->defer.as<uint32_t>(dl);
    x.dA_j = c->defer.as<uint8_t>(2 * dl);
    x.dB_j = c->defer.as<uint8_t>(2 * dl + dj);
    if (x.out) FJ_TRY(c->emitbuf.ensure(align256(sizeof(u64) * x.C) + align256(sizeof(u64) * (x.C + 1)), c->stream));

    // tail nodes and head mapping
    const auto &LT = p->layout[x.tail_from];
    for (int k = x.tail_from; k < x.nnodes; k++) {
        const fj::Subatom &s = p->nodes[k][0];
        int a = s.atom;
        int l = p->sub_level[k][0];
        TailDev T;
        memset(&T, 0, sizeof(T));
        T.atom = a;
        T.level = l;
        T.nk = s.nv;
        for (int j = 0; j < s.nv; j++) {
            T.kvar[j] = s.vars[j];
            T.kcol[j] = colts[a]->lev[l].kcol[j];
        }
        for (int j = 0; j < FJ_MAX_COLS; j++) T.cols[j] = colts[a]->cols[j];
        T.root_len = colts[a]->nroot;
        T.L = colts[a]->lev[l];
        x.tails.push_back(T);
    }
    for (int j = 0; j < q->nhead; j++) {
        int v = q->head[j];
        int src = 0;
        bool found = false;
        for (size_t i = 0; i < LT.in_var.size(); i++)
            if (LT.in_var[i] == v) { src = (int)i; found = true; }
        for (size_t t = 0; t < x.tails.size() && !found; t++)
            for (int cc = 0; cc < x.tails[t].nk; cc++)
                if (x.tails[t].kvar[cc] == v) { src = -((int)t * FJ_MAX_COLS + cc) - 1; found = true; }
        if (!found) return fail(FJ_ERR_ARG, "head variable not bound by the plan");
        x.head_src.push_back(src);
    }

    if (res) {
        const fj::NodeLayout &LT0 = p->layout[x.tail_from];
        res->nvals = (int)LT0.in_var.size();
        res->nhdl = (int)LT0.in_hatom.size();
        res->in_var.assign(LT0.in_var.begin(), LT0.in_var.end());
        res->in_hatom.assign(LT0.in_hatom.begin(), LT0.in_hatom.end());
        res->head_src = x.head_src;
        res->tails = x.tails;
    }

    // node descriptors
    size_t nd_bytes = align256(sizeof(NodeDev) * std::max(x.tail_from, 1));
    size_t em_bytes = align256(fj::emit_dev_size());
    if (nd_bytes + em_bytes > c->desc.bytes) c->desc_last.clear();   // a new device buffer holds nothing yet
    FJ_TRY(c->desc.ensure(nd_bytes + em_bytes, c->stream));
    // the staging buffer mirrors the device layout (node descriptors, then
    // the emit descriptor) and goes over in one copy; only that copy of the
    // previous call must have finished before it is rewritten
    if (!c->desc_done) FJ_HIP(hipEventCreateWithFlags(&c->desc_done, hipEventDisableTiming));
    else FJ_HIP(hipEventSynchronize(c->desc_done));
    if (c->desc_h_bytes < nd_bytes + em_bytes) {
        if (c->desc_h) hipHostFree(c->desc_h);
        c->desc_h = nullptr;
        c->desc_h_bytes = 0;
        FJ_HIP(hipHostMalloc(&c->desc_h, nd_bytes + em_bytes, hipHostMallocDefault));
        c->desc_h_bytes = nd_bytes + em_bytes;
    }
    x.nd_d = c->desc.as<NodeDev>(0);
    x.emit_d = c->desc.as<char>(nd_bytes);
    NodeDev *ndh = (NodeDev *)c->desc_h;
    for (int k = 0; k < x.tail_from; k++) {
        NodeDev &nd = ndh[k];
        memset(&nd, 0, sizeof(nd));
        const auto &L = p->layout[k];
        const auto &LN = p->layout[k + 1];
        nd.k = k;
        nd.nsub = (int)p->nodes[k].size();
        nd.npure = (int)L.pure.size();
        for (int i = 0; i < nd.npure; i++) nd.pure[i] = L.pure[i];
        int slot_of[FJ_MAX_VARS];
        for (int v = 0; v < FJ_MAX_VARS; v++) slot_of[v] = -1;
        nd.nin = (int)L.in_var.size();
        for (int i = 0; i < nd.nin; i++) slot_of[L.in_var[i]] = i;
        nd.nnew = (int)L.new_vars.size();
        for (int i = 0; i < nd.nnew; i++) slot_of[L.new_vars[i]] = nd.nin + i;
        for (int i = 0; i < nd.nsub; i++) {
            const fj::Subatom &s = p->nodes[k][i];
            SubDev &S = nd.sub[i];
            int a = s.atom;
            int l = p->sub_level[k][i];
            S.atom = a;
            S.level = l;
            S.last = (l == p->nlev[a] - 1);
            S.child_leaf = (l + 1 == p->nlev[a]);
            S.nk = s.nv;
            S.fq_slot = a * fj::kMaxLevels + l;
            for (int j = 0; j < s.nv; j++) {
                S.kslot[j] = slot_of[s.vars[j]];
                S.kcol[j] = colts[a]->lev[l].kcol[j];
            }
            fill_level_sub(S, colts[a], l);
        }
        nd.nin_h = (int)L.in_hatom.size();
        for (int i = 0; i < nd.nin_h; i++) nd.in_h_atom[i] = L.in_hatom[i];
        nd.nout = (int)LN.in_var.size();
        for (int i = 0; i < nd.nout; i++) nd.out_slot[i] = slot_of[LN.in_var[i]];
        nd.nout_h = (int)LN.in_hatom.size();
        for (int i = 0; i < nd.nout_h; i++) nd.out_h_atom[i] = LN.in_hatom[i];
        nd.emit = (k == x.tail_from - 1);
        nd.materialize = nd.emit && (x.out != nullptr || x.res != nullptr);
        if (nd.emit) {
            nd.ntail = (int)x.tails.size();
            for (int i = 0; i < nd.ntail; i++) nd.tail[i] = x.tails[i];
        }
        nd.in = x.F[k];
        nd.out = x.F[k + 1];
    }
    if (x.out) {
        const fj::NodeLayout &LT0 = p->layout[x.tail_from];
        fj::emit_dev_fill((char *)c->desc_h + nd_bytes, x.F[x.tail_from], LT0.in_var.data(), LT0.in_var.size(),
                          LT0.in_hatom.data(), LT0.in_hatom.size(), x.tails.data(), (int)x.tails.size(),
                          x.head_src.data(), (int)x.head_src.size(), x.out, x.cap);
    }
    if (x.tail_from > 0 || x.out) {
        // kernels only read the descriptors: when they are the ones already
        // on the device (the same query run again), the copy is skipped
        const size_t bytes = x.out ? nd_bytes + fj::emit_dev_size() : sizeof(NodeDev) * x.tail_from;
        if (!(c->desc_last_dev == c->desc.p && c->desc_last.size() == bytes &&
              memcmp(c->desc_last.data(), c->desc_h, bytes) == 0)) {
            FJ_HIP(hipMemcpyAsync(c->desc.p, c->desc_h, bytes, hipMemcpyHostToDevice, c->stream));
            // (the staging buffer is rewritten only once this copy is done)
            FJ_HIP(hipEventRecord(c->desc_done, c->stream));
            c->desc_last.assign((const char *)c->desc_h, (const char *)c->desc_h + bytes);
            c->desc_last_dev = c->desc.p;
        }
    }

    // clear the counters but keep any error a build left for the next check;
    // the host copy mirrors the cleared counters (they are read as bases)
    FJ_HIP(hipMemsetAsync(c->status_d, 0, offsetof(StatusDev, err_line), c->stream));
    memset(c->status_h, 0, offsetof(StatusDev, err_line));
    fj_status st;
    if (x.tail_from == 0) {
        // every node is a product of base tables: one empty binding
        FJ_HIP(hipStreamSynchronize(c->stream));
        u64 total = 1;
        for (const auto &T : x.tails) total *= T.root_len;
        c->status_h->count = total;
        FJ_HIP(hipMemcpyAsync(c->status_d, c->status_h, sizeof(u64), hipMemcpyHostToDevice, c->stream));
        st = emit_or_keep(x, 1);
    } else {
        st = exec_node(x, 0, 1);
    }
    if (st != FJ_OK) return st;
    FJ_TRY(sync_status(c));
    if (x.emit_pending) {
        const u64 E = c->status_h->survivors - x.emit_pending_base;
        if (E > fj::emit_small_max()) {
            // too many bindings for the one-workgroup emit, which left the
            // status alone: the general path
            FJ_TRY(emit_rows(x, (uint32_t)E));
            FJ_TRY(sync_status(c));
        } else if (E > 0 && c->status_h->emit_rows > 0) {
            // placed, but too many rows to write in one workgroup
            const u64 *starts = c->emitbuf.as<u64>(align256(sizeof(u64) * x.C));
            {
                Timer t(c, FJ_T_EMIT);
                FJ_HIP(fj::launch_emit_rows(x.emit_d, (uint32_t)E, starts, c->status_h->emit_rows, c->status_d,
                                            c->stream));
            }
            FJ_TRY(sync_status(c));
        }
    }
    // a direct emit reserves every row it counts: what passed cap was not written
    x.written = std::min<u64>(c->status_h->written, x.cap);
    u64 total = c->status_h->count;
    for (int q = 0; q < fj::kCountParts; q++) total += c->status_h->count_part[q * fj::kPartStride];
    *count = total;
    if (written) *written = x.written;
    if (stats) {
        for (int k = 0; k < x.tail_from; k++) {
            stats->probe[k] = c->status_h->probe[k];
            stats->hit[k] = c->status_h->hit[k];
        }
        if (x.tail_from > 0) stats->survivors[x.tail_from - 1] = 0;
        stats->filtered = c->status_h->filtered;
    }
    return (x.out && *count > x.cap) ? FJ_TRUNCATED : FJ_OK;
}

extern "C" fj_status fj_execute(fj_ctx *c, const fj_query *q, const fj_plan *p, fj_colt *const *colts,
                                uint64_t *count, int32_t *out, uint64_t cap, uint64_t *written, fj_stats *stats) {
    return execute_impl(c, q, p, colts, count, out, cap, written, stats, nullptr);
}

// ------------------------------------------------------ factorized results

extern "C" fj_status fj_execute_factorized(fj_ctx *c, const fj_query *q, const fj_plan *p, fj_colt *const *colts,
                                           fj_result **out, uint64_t *count, uint64_t *bindings) {
    if (!out) return fail(FJ_ERR_ARG, "null argument");
    *out = nullptr;
    if (!c || !q || !count) return fail(FJ_ERR_ARG, "null argument");
    fj_result *r = new fj_result;
    r->device = c->device;
    fj_status st = execute_impl(c, q, p, colts, count, nullptr, 0, nullptr, nullptr, r);
    if (st != FJ_OK) {
        hipStreamSynchronize(c->stream);
        delete r;
        return st;
    }
    r->count = *count;
    if (bindings) *bindings = r->E;
    *out = r;
    return FJ_OK;
}

extern "C" fj_status fj_result_expand(fj_ctx *c, fj_result *r, uint64_t first, int32_t *out, uint64_t cap,
                                      uint64_t *written) {
    if (!c || !r || !written || (cap && !out)) return fail(FJ_ERR_ARG, "null argument");
    *written = 0;
    if (c->device != r->device) return fail(FJ_ERR_ARG, "the result is on another device than the context");
    if (first >= r->count || cap == 0) return FJ_OK;
    FJ_HIP(hipSetDevice(c->device));
    const u64 n = std::min<u64>(cap, r->count - first);
    FrontierDev F;
    memset(&F, 0, sizeof(F));
    F.vals = r->vals;
    F.hdl = r->hdl;
    F.mult = r->mult;
    F.cap = r->cap;
    F.nvals = r->nvals;
    F.nhdl = r->nhdl;
    // the emit descriptor names the caller's buffer, so it is written anew
    r->emit_h.resize(fj::emit_dev_size());
    fj::emit_dev_fill(r->emit_h.data(), F, r->in_var.data(), (int)r->in_var.size(), r->in_hatom.data(),
                      (int)r->in_hatom.size(), r->tails.data(), (int)r->tails.size(), r->head_src.data(),
                      (int)r->head_src.size(), out, n);
    if (!r->emit_d) FJ_TRY(fj::pool_alloc(r->device, fj::emit_dev_size(), &r->emit_d));
    FJ_HIP(hipMemcpyAsync(r->emit_d, r->emit_h.data(), fj::emit_dev_size(), hipMemcpyHostToDevice, c->stream));
    const uint32_t E = (uint32_t)r->E;
    if (!r->starts) {
        // every binding's row count and their scan, once per result
        r->starts_bytes = sizeof(u64) * (r->E + 1);
        FJ_TRY(fj::pool_alloc(r->device, r->starts_bytes, (void **)&r->starts));
        void *cnt = nullptr;
        FJ_TRY(fj::pool_alloc(r->device, sizeof(u64) * r->E, &cnt));
        fj_status st = FJ_OK;
        if (fj::launch_emit_count(r->emit_d, E, (u64 *)cnt, c->status_d, c->stream) != hipSuccess)
            st = fail(FJ_ERR_HIP, "emit count launch failed");
        if (st == FJ_OK) st = scan_u64(c, (const u64 *)cnt, r->starts, r->E);
        hipStreamSynchronize(c->stream);
        fj::pool_free(r->device, cnt, sizeof(u64) * r->E);
        if (st != FJ_OK) {
            fj::pool_free(r->device, r->starts, r->starts_bytes);
            r->starts = nullptr;
            return st;
        }
    }
    {
        Timer t(c, FJ_T_EMIT);
        FJ_HIP(fj::launch_emit_range(r->emit_d, E, r->starts, first, n, c->status_d, c->stream));
    }
    FJ_TRY(sync_status(c));
    *written = n;
    return FJ_OK;
}

extern "C" void fj_result_free(fj_result *r) {
    if (!r) return;
    hipSetDevice(r->device);
    hipDeviceSynchronize();
    delete r;
}

// ------------------------------------------------------------------ batches

struct fj_batch {
    fj_ctx *c = nullptr;
    int n = 0;
    fj_batch_options opt{};
    std::vector<const fj_query *> qs;
    std::vector<const fj_plan *> plans;
    std::vector<std::vector<fj_colt *>> colts;
    fj::BQuery *q_dev = nullptr;
    fj::BItem *items_dev = nullptr;
    uint32_t nitems = 0;
    u64 *counts_dev = nullptr;
    u64 *counts_h = nullptr;
    int grid = 0;
    int lv = 1, la = 1;             // largest variable and atom counts (lane state sizes)
    ColtGroup *group = nullptr;     // every COLT's root build, with its own scratch
    std::vector<fj_colt *> members;
    hipStream_t stream = nullptr;   // the batch's own stream (the null stream cannot be captured)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

fj_status batch_query(const fj_query *q, const fj_plan *p, fj_colt *const *colts, fj::BQuery &B) {
    memset(&B, 0, sizeof(B));
    if (q->nvars > fj::kBMaxVars) return fail(FJ_ERR_UNSUPPORTED, "batched queries have at most 16 variables");
    const int nexec = p->tail_from;
    if (nexec < 1 || nexec > fj::kBMaxNodes) return fail(FJ_ERR_UNSUPPORTED, "batched plans run 1..8 probing nodes");
    B.nexec = nexec;
    B.nvars = q->nvars;
    B.natoms = q->natoms;
    for (int k = 0; k < nexec; k++) {
        const auto &node = p->nodes[k];
        const auto &L = p->layout[k];
        // static cover: the node's first subatom when it is a pure cover (the
        // relation the binary plan iterates), else the first pure cover
        if (L.pure.empty()) return fail(FJ_ERR_UNSUPPORTED, "no pure cover");
        int ci = L.pure[0];
        for (int pc : L.pure)
            if (pc == 0) ci = 0;
        const int ca = node[ci].atom, cl = p->sub_level[k][ci];
        const fj_colt *ct = colts[ca];
        fj::BNode &N = B.node[k];
        N.catom = ca;
        if (k == 0) {
            if (p->root_built[ca] || p->nlev[ca] != 1)
                return fail(FJ_ERR_UNSUPPORTED, "batched plans iterate a base table first");
            N.offs = ct->sel;
            B.n0 = ct->nroot;
        } else {
            if (cl == 0 || cl != p->nlev[ca] - 1)
                return fail(FJ_ERR_UNSUPPORTED, "batched plans iterate the last level reached by a probe");
            N.offs = ct->lev[cl].offs;
            N.len = ct->lev[cl].len;
            N.kv = node[ci].nv == 1 ? ct->lev[cl].kv : nullptr;
        }
        N.npos = ct->lev[cl].npos;
        N.nrows = (uint32_t)ct->nrows;
        N.nk = node[ci].nv;
        for (int j = 0; j < N.nk; j++) {
            N.kslot[j] = node[ci].vars[j];
            N.kcol[j] = ct->cols[ct->lev[cl].kcol[j]];
        }
        for (int i = 0; i < (int)node.size(); i++) {
            if (i == ci) continue;
            const int a = node[i].atom;
            const fj_colt *t = colts[a];
            const LevelDev &R = t->lev[0];
            if (p->sub_level[k][i] != 0 || !p->root_built[a] ||
                !(R.mode == fj::KM_K32 || (R.mode == fj::KM_K64 && R.nk == 2)))
                return fail(FJ_ERR_UNSUPPORTED, "batched plans probe root maps keyed by one or two variables");
            if (N.nl >= fj::kBMaxLookups) return fail(FJ_ERR_UNSUPPORTED, "too many lookups in a node");
            fj::BLookup &BL = N.lk[N.nl++];
            BL.table = R.table;
            BL.mask = R.mask;
            BL.mode = R.mode;
            BL.kslot[0] = node[i].vars[0];
            BL.kslot[1] = node[i].nv > 1 ? node[i].vars[1] : node[i].vars[0];
            BL.atom = a;
            BL.child_leaf = p->nlev[a] == 1;
            BL.clen = t->lev[1].len;
            BL.cnpos = t->lev[1].npos;
        }
    }
    const int nn = (int)p->nodes.size();
    B.ntail = nn - nexec;
    for (int k = nexec; k < nn; k++) {
        const int q2 = k - nexec;
        const int a = p->nodes[k][0].atom, l = p->sub_level[k][0];
        B.tail_atom[q2] = a;
        B.tail_root[q2] = l == 0;
        B.tail_root_len[q2] = colts[a]->nroot;
        B.tail_len[q2] = colts[a]->lev[l].len;
        B.tail_npos[q2] = colts[a]->lev[l].npos;
    }
    return FJ_OK;
}

// The launches of one run (rebuilds, zeroed counts, the persistent kernel).
fj_status batch_launches(fj_batch *b) {
    fj_ctx *c = b->c;
    if (!b->opt.no_rebuild) FJ_TRY(group_launch(c, *b->group));
    FJ_HIP(fj::launch_zero_u64(b->counts_dev, (uint32_t)b->n, c->stream));
    FJ_HIP(fj::launch_batch_dfs(b->q_dev, b->items_dev, b->nitems, b->counts_dev, c->status_d, b->opt.block, b->grid,
                                b->lv, b->la, c->stream));
    return FJ_OK;
}

void batch_release(fj_batch *b) {
    if (!b) return;
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    if (b->q_dev) hipFree(b->q_dev);
    if (b->items_dev) hipFree(b->items_dev);
    if (b->counts_dev) hipFree(b->counts_dev);
    if (b->counts_h) hipHostFree(b->counts_h);
    if (b->stream) hipStreamDestroy(b->stream);
    destroy_group(b->group);
    delete b;
}

// Run f with the context's work on the batch stream, ordered after
// everything already queued on the context's own stream.
template <typename F> fj_status on_batch_stream(fj_batch *b, F f) {
    fj_ctx *c = b->c;
    hipStream_t orig = c->stream;
    FJ_HIP(hipStreamSynchronize(orig));
    c->stream = b->stream;
    fj_status st = f();
    c->stream = orig;
    return st;
}

}  // namespace

extern "C" fj_status fj_batch_create(fj_ctx *c, int32_t n, const fj_query *const *qs, const fj_plan *const *plans,
                                     fj_colt *const *const *colts, const fj_batch_options *opt, fj_batch **out) {
    if (!c || n < 1 || !qs || !plans || !colts || !out) return fail(FJ_ERR_ARG, "bad argument");
    *out = nullptr;
    if (c->opt.trie != 0) return fail(FJ_ERR_UNSUPPORTED, "batches run on COLTs (trie option 0)");
    FJ_HIP(hipSetDevice(c->device));
    fj_batch *b = new fj_batch();
    b->c = c;
    b->n = n;
    if (opt) b->opt = *opt;
    if (b->opt.chunk <= 0) b->opt.chunk = 1024;
    if (b->opt.block <= 0) b->opt.block = 256;
    if (b->opt.block % 64 || b->opt.block > 512) { batch_release(b); return fail(FJ_ERR_ARG, "bad block size"); }
    std::vector<fj::BQuery> hq(n);
    std::vector<fj::BItem> items;
    u64 max_rows = 0;
    for (int i = 0; i < n; i++) {
        if (!qs[i] || !plans[i] || !colts[i]) { batch_release(b); return fail(FJ_ERR_ARG, "null query"); }
        fj_status st = check_exec_args(c, qs[i], plans[i], colts[i]);
        if (st == FJ_OK) st = batch_query(qs[i], plans[i], colts[i], hq[i]);
        if (st != FJ_OK) {
            std::string m = g_err;
            batch_release(b);
            return fail(st, "query " + std::to_string(i) + ": " + m);
        }
        b->qs.push_back(qs[i]);
        b->plans.push_back(plans[i]);
        b->lv = std::max<int>(b->lv, qs[i]->nvars);
        b->la = std::max<int>(b->la, qs[i]->natoms);
        b->colts.emplace_back(colts[i], colts[i] + qs[i]->natoms);
        for (fj_colt *t : b->colts.back()) max_rows = std::max<u64>(max_rows, t->cap_rows);
        const uint32_t chunk =
            (uint32_t)((b->opt.query_chunk && b->opt.query_chunk[i] > 0) ? b->opt.query_chunk[i] : b->opt.chunk);
        for (uint32_t r0 = 0; r0 < hq[i].n0; r0 += chunk)
            items.push_back({(uint32_t)i, r0, std::min<uint32_t>(hq[i].n0, r0 + chunk)});
    }
    // largest items first; workgroups take items round robin
    std::stable_sort(items.begin(), items.end(),
                     [](const fj::BItem &x, const fj::BItem &y) { return x.r1 - x.r0 > y.r1 - y.r0; });
    b->nitems = (uint32_t)items.size();
    // workgroups that fit a CU's 160 KB of LDS at once
    const size_t lds_per = 2 * sizeof(uint32_t) * (size_t)(b->lv + b->la) * b->opt.block;
    const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(2048 / b->opt.block, (160 * 1024) / lds_per));
    b->grid = (int)std::max<u64>(1, std::min<u64>(b->nitems, (u64)c->num_cus * per_cu));
    fj_status st = FJ_OK;
    if (hipMalloc((void **)&b->q_dev, sizeof(fj::BQuery) * n) != hipSuccess ||
        hipMalloc((void **)&b->items_dev, sizeof(fj::BItem) * std::max<size_t>(items.size(), 1)) != hipSuccess ||
        hipMalloc((void **)&b->counts_dev, sizeof(u64) * n) != hipSuccess ||
        hipHostMalloc((void **)&b->counts_h, sizeof(u64) * n, hipHostMallocDefault) != hipSuccess) {
        batch_release(b);
        return fail(FJ_ERR_OOM, "batch buffers");
    }
    if (hipMemcpy(b->q_dev, hq.data(), sizeof(fj::BQuery) * n, hipMemcpyHostToDevice) != hipSuccess ||
        (!items.empty() && hipMemcpy(b->items_dev, items.data(), sizeof(fj::BItem) * items.size(),
                                     hipMemcpyHostToDevice) != hipSuccess)) {
        batch_release(b);
        return fail(FJ_ERR_HIP, "batch upload");
    }
    // the grouped root build of every distinct COLT, with descriptors and
    // scratch owned by the batch (the captured graph keeps their addresses)
    if (!b->opt.no_rebuild) {
        u64 wcap = 0;
        for (int i = 0; i < n; i++)
            for (fj_colt *t : b->colts[i])
                if (std::find(b->members.begin(), b->members.end(), t) == b->members.end()) {
                    b->members.push_back(t);
                    if (t->root_built) wcap += t->cap_rows;
                }
        b->group = new ColtGroup();
        st = group_prepare(c, *b->group, b->members.data(), (int)b->members.size(), wcap);
        if (st == FJ_OK) st = sync_status(c);
        if (st != FJ_OK) { batch_release(b); return st; }
    }
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
        batch_release(b);
        return fail(FJ_ERR_HIP, "stream creation failed");
    }
    if (!b->opt.no_graph) {
        const int timing = c->opt.timing;
        c->opt.timing = 0;   // no event nodes in the graph
        st = on_batch_stream(b, [&]() -> fj_status {
            hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess) return fail(FJ_ERR_HIP, std::string("stream capture failed: ") + hipGetErrorString(e));
            fj_status s1 = batch_launches(b);
            hipGraph_t g = nullptr;
            hipError_t e2 = hipStreamEndCapture(c->stream, &g);
            b->graph = g;
            if (s1 != FJ_OK) return s1;
            if (e2 != hipSuccess) return fail(FJ_ERR_HIP, "graph capture failed");
            if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
                return fail(FJ_ERR_HIP, "graph instantiation failed");
            return FJ_OK;
        });
        c->opt.timing = timing;
        if (st != FJ_OK) { batch_release(b); return st; }
    }
    *out = b;
    return FJ_OK;
}

extern "C" fj_status fj_batch_run(fj_batch *b, uint64_t *counts) {
    if (!b || !counts) return fail(FJ_ERR_ARG, "null argument");
    fj_ctx *c = b->c;
    FJ_HIP(hipSetDevice(c->device));
    FJ_TRY(on_batch_stream(b, [&]() -> fj_status {
        {
            Timer t(c, FJ_T_PROBE);
            if (b->exec) FJ_HIP(hipGraphLaunch(b->exec, c->stream));
            else FJ_TRY(batch_launches(b));
        }
        FJ_HIP(hipMemcpyAsync(b->counts_h, b->counts_dev, sizeof(u64) * b->n, hipMemcpyDeviceToHost, c->stream));
        return sync_status(c);
    }));
    // the run rebuilt every root: inner levels need initialising again
    for (fj_colt *t : b->members)
        for (int l = 0; l < t->nlev; l++) t->lev_ready[l] = false;
    memcpy(counts, b->counts_h, sizeof(u64) * b->n);
    return FJ_OK;
}

extern "C" void fj_batch_free(fj_batch *b) {
    if (!b) return;
    hipSetDevice(b->c->device);
    hipStreamSynchronize(b->c->stream);
    batch_release(b);
}
