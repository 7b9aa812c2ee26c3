// Device-side data layout of COLT levels, plan nodes and frontiers, shared by
// the HIP kernels and the host orchestration in libfj.  Internal header.
//
// Position space.  Every level of one atom's COLT uses the same positions
// [0, nroot): the root handle owns [0, nroot); when a handle owning
// [p, p + len) at level l is forced, its children at level l + 1 own disjoint
// sub-ranges of [p, p + len) holding the same row offsets regrouped by key.
// A handle is therefore identified by the start position of its range, and
// per-handle metadata lives in position-indexed arrays of each level.
#pragma once

#include <cstdint>

#include "fj.h"

namespace fj {

constexpr int kMaxLevels = FJ_MAX_NODES;   // schema levels per atom
constexpr uint32_t kQueued = 0xFFFFFFFFu;  // state word: force requested
constexpr uint32_t kEmpty32 = 0xFFFFFFFFu;
constexpr unsigned long long kEmpty64 = ~0ull;

// Hash-map layouts of one level, chosen by key width.
enum KeyMode : int {
    KM_K32 = 0,   // root level, one key column: u32 key and u32 val per
                  // slot, in split buckets (below)
    KM_K64 = 1,   // packed 64-bit key (root with two key columns, or
                  // (handle, value) below the root): slot {u64 key, u32 val, pad}
    KM_REP = 2,   // wider keys: slot {u32 handle, u32 representative row, u32 val, pad},
                  // compared column by column against the representative row
    KM_ZERO = 3   // a level with no variables: one key, no table
};

// KM_K32 maps hold buckets of four slots as four keys followed by their four
// values (32 bytes), so one 16-byte load compares a probe against a whole
// bucket and the value is read only on a hit.  Slot i's key is 32-bit word
// k32_key_word(i) of the table and its value the word four after it; the
// reserved slot (index capacity) starts a bucket of its own.
constexpr int kK32Bucket = 4;
__host__ __device__ inline unsigned long long k32_key_word(unsigned long long i) {
    return ((i >> 2) << 3) + (i & 3);
}
__host__ __device__ inline unsigned long long k32_table_words(unsigned long long cap) { return 2 * cap + 8; }
// A KM_K32 map is probed within ranges of kK32Part slots (the whole map when
// it is smaller): a key's walk starts at its bucket and wraps at the end of
// the bucket's range.  So the keys of one range can be placed by one
// workgroup in LDS (the grouped root build) and found by the same walk.
constexpr unsigned long long kK32Part = 2048;
__host__ __device__ inline unsigned long long k32_part_mask(unsigned long long mask) {
    return mask < kK32Part ? mask : kK32Part - 1;
}
__host__ __device__ inline unsigned long long k32_next(unsigned long long b, unsigned long long mask) {
    const unsigned long long pm = k32_part_mask(mask);
    return (b & ~pm) | ((b + kK32Bucket) & pm);
}
// A KM_K32 root built range by range also gets a membership filter of its
// keys: each key sets two bits (from its hash's top ten bits) of one 32-bit
// word, the word being its home bucket shifted right by the filter's shift,
// so the keys of one build range set bits of that range's words only.  At
// most kBloomWords words (64 KB), the size one workgroup keeps in LDS.
constexpr uint32_t kBloomWords = 16384;
struct alignas(16) Slot64 { unsigned long long key; uint32_t val; uint32_t pad; };
struct alignas(16) SlotRep { unsigned long long hr; uint32_t val; uint32_t pad; };  // hr = row << 32 | handle

// One level of one atom's COLT.  The leaf level (index nlev) only uses offs/len.
struct LevelDev {
    uint32_t *offs;      // row offsets by position (root: selection, or null = identity)
    uint32_t *len;       // len[p] of the handle starting at p
    uint32_t *st;        // 0 = unforced, kQueued, else (number of keys + 1)
    uint32_t *kl;        // kl[p + r] = start of the child with rank r of handle p
    void *table;         // hash slots, mask + 2 entries (the last is the reserved slot)
    unsigned long long mask;
    uint32_t *rank_ctr;  // per handle: distinct keys seen while forcing
    uint32_t *cnt;       // per child rank position: offsets while forcing (returns to 0)
    uint32_t *fq;        // force queue: handle starts
    // Keys kept beside the offsets (levels keyed by one variable only):
    int32_t *kv;         // kv[p]: the level's key value of the row at offs[p] (below the root)
    int32_t *kk;         // kk[p + r]: the key of rank r of the forced handle at p
    uint32_t *kn;        // kn[p + r]: the number of offsets under that key
    int mode;
    int nk;
    int kcol[FJ_MAX_COLS];
    uint32_t npos;       // entries of every position-indexed array (>= 1)
    uint32_t nrows;      // rows of the relation's columns
    unsigned long long nslots;  // hash slots including the reserved one (0: no map)
    int local;           // per-trie maps (levels below the root, KM_K64 / KM_REP): the trie at
                         // position p with len[p] offsets owns slots [2p, 2p + 2 len[p])
    uint32_t *bloom;     // KM_K32 root built range by range: its keys' filter (written by the
                         // build), or null
    uint32_t bloom_shift;   // filter word of a key = its home bucket >> bloom_shift
};

struct SubDev {
    int atom;
    int level;
    int last;        // level == nlev - 1
    int child_leaf;  // level + 1 == nlev: a get reaches an offset vector (a multiplicity)
    int nk;
    int fq_slot;     // index of this (atom, level) in the status block's queue counters
    int kslot[FJ_MAX_COLS];   // thread value slot of each key variable
    int kcol[FJ_MAX_COLS];    // atom column of each key variable
    const int32_t *cols[FJ_MAX_COLS];  // the atom's columns
    uint32_t root_len;        // level 0: number of root offsets
    LevelDev L;               // this level
    LevelDev C;               // the child level
};

struct TailDev {
    int atom;
    int level;
    int nk;
    int kcol[FJ_MAX_COLS];
    int kvar[FJ_MAX_COLS];
    const int32_t *cols[FJ_MAX_COLS];
    uint32_t root_len;
    LevelDev L;
};

// A frontier: values of the bound variables and current handles of the
// atoms part-way through their schemas, structure of arrays, `cap` rows.
struct FrontierDev {
    int32_t *vals;     // nvals columns of cap
    uint32_t *hdl;     // nhdl columns of cap
    unsigned long long *mult;
    unsigned long long cap;
    int nvals;
    int nhdl;
};

struct NodeDev {
    int k;
    int nsub;
    int npure;
    int pure[FJ_MAX_ATOMS];
    SubDev sub[FJ_MAX_ATOMS];
    int nin;                       // input value columns -> slots [0, nin)
    int nnew;                      // new variables -> slots [nin, nin + nnew)
    int nin_h;
    int in_h_atom[FJ_MAX_ATOMS];   // input handle column j -> atom
    int nout;
    int out_slot[FJ_MAX_VARS];     // output value column j <- slot
    int nout_h;
    int out_h_atom[FJ_MAX_ATOMS];  // output handle column j <- atom
    int emit;                      // survivors are results (this is the last probed node)
    int materialize;               // emit: also write survivors to the output frontier
    int ntail;
    TailDev tail[FJ_MAX_NODES];
    FrontierDev in;
    FrontierDev out;
};

// A root-map probe of the specialised first-node kernel.
struct ScanLookup {
    const void *table;
    unsigned long long mask;
    int mode;              // KM_K32 or KM_K64 (root keys of one or two columns)
    int kc[2];             // cover columns of the key variables
    int child_leaf;
    const uint32_t *clen;  // child level lengths
    uint32_t cnpos;        // child level positions
    int hcol;              // output handle column of this atom, or -1
    const uint32_t *bloom; // the map's key filter, used by the first lookup, or null
    uint32_t bloom_shift;
    uint32_t bloom_words;  // words of the filter in use
};

// Batched counting of plans that probe only root maps (see fj_batch_create).
constexpr int kBMaxNodes = 8;
constexpr int kBMaxLookups = 8;
constexpr int kBMaxVars = 16;

struct BLookup {
    const void *table;
    unsigned long long mask;
    int mode;                 // KM_K32 or KM_K64
    int kslot[2];             // variables of the key
    int atom;
    int child_leaf;           // the child is an offset vector (a multiplicity)
    const uint32_t *clen;     // child level lengths
    uint32_t cnpos;
};

struct BNode {
    int catom;                // atom whose trie the node iterates (by offset)
    int nk;
    int kslot[FJ_MAX_COLS];   // variables the cover binds
    const int32_t *kcol[FJ_MAX_COLS];  // their columns
    const uint32_t *offs;     // offsets of the cover's level (node 0: selection or null)
    const int32_t *kv;        // the cover's key values beside its offsets (one key variable), or null
    const uint32_t *len;      // lengths of the cover's level (unused at node 0)
    uint32_t npos;
    uint32_t nrows;
    int nl;
    BLookup lk[kBMaxLookups];
};

struct BQuery {
    int nexec;                // nodes run tuple by tuple; the rest are products
    int ntail;
    int nvars, natoms;
    uint32_t n0;              // rows of the first node's cover
    BNode node[kBMaxNodes];
    int tail_atom[kBMaxNodes];
    int tail_root[kBMaxNodes];         // the tail iterates a root (its length is root_len)
    const uint32_t *tail_len[kBMaxNodes];
    uint32_t tail_npos[kBMaxNodes];
    uint32_t tail_root_len[kBMaxNodes];
};

struct BItem {
    uint32_t q;               // query
    uint32_t r0, r1;          // first-node rows [r0, r1)
};

// Regions a COLT (re)build initialises in one launch.
struct FillRegion {
    uint32_t *p;
    unsigned long long nwords;
    uint32_t pat[8];
    int period;   // 1, 2, 4 or 8 words
};
constexpr int kMaxFill = 6 * kMaxLevels + 4;
struct FillList {
    int n;
    FillRegion r[kMaxFill];
};

// One force: the handles queued on level L regrouped into child level C.
// Per-item scratch (wslot, cntv, ex) is indexed by the item's position among
// the queued handles' offsets.
struct ForceArgs {
    LevelDev L;
    LevelDev C;
    const int32_t *cols[FJ_MAX_COLS];
    const uint32_t *fq;     // queued handle starts
    uint32_t nh;            // number of queued handles
    const uint32_t *pre;    // exclusive scan of their lengths (nh + 1)
    uint32_t W;             // total offsets
    uint32_t wcap;          // capacity of the per-item scratch arrays
    uint32_t *wslot;        // per item: slot index | kClaim for the item that inserted the key
    unsigned long long *cntv;  // per item: (1 << 32 | offsets of the key) for claimers, else 0
    unsigned long long *ex;    // exclusive scan of cntv (W + 1)
    struct StatusDev *status;
};

// Grouped root builds: a chunk of a fill region, and a COLT's root words.
struct FillBlock {
    uint32_t *p;
    unsigned long long start, n;   // words [start, start + n) of the region at p (start % 8 == 0)
    uint32_t pat[8];
    int period;
};
struct GroupRoot {
    uint32_t *len, *st, *fq, *pre;
    uint32_t nroot;
    int built;
};

// Grouped root builds by key range (KM_K32 roots): a member COLT whose map
// of np ranges (kK32Part slots each, or the whole map when smaller) is
// built range by range, each range by one workgroup in LDS.
constexpr uint32_t kMaxParts = 4096;       // ranges per map on this path
constexpr uint32_t kPlaceChunk = 1024;     // items a block of the place pass holds at once (4 a thread)
constexpr uint32_t kMaxPlaceBlocks = 1024; // place blocks per member (one per build thread)
struct PartMember {
    int desc;                 // the member's ForceArgs in the group
    uint32_t np;              // ranges of its map
    uint32_t plog;            // log2 of the slots per range
    uint32_t part_base;       // its first range in the group's range space
    uint32_t block_base;      // its first block of the place pass
    uint32_t nb;              // its blocks of the place pass
    uint32_t ipb;             // items per place block (a multiple of kPlaceChunk; the last takes the rest)
    uint32_t item_base;       // its first item in the group's item space
    uint32_t W;               // its root rows
    int clear_cst;            // the build clears level 1's state words of the member's positions
    int keys;                 // its root's keys are listed (the rank pass); else only probed
    unsigned long long slot_base;  // its first slot in the group's slot space (scnt)
    unsigned long long off_base;   // its (np + 1) x nb offset matrix in poff
};
struct PartArgs {
    const ForceArgs *descs;
    const PartMember *mem;
    const uint32_t *mop;      // nparts: each range's member
    const uint32_t *mob;      // nblocks: each place block's member
    int n;
    uint32_t nblocks;         // blocks of the place pass
    uint32_t nparts;          // ranges of every member
    uint32_t items;           // items of every member (the length of prow, pkey, pkv)
    int inline_scan;          // few ranges: the rank pass sums the distinct counts it needs itself
    uint32_t *poff;           // per member: poff[p * nb + b] = block b's items in ranges before p
    uint32_t *prow, *pkey, *pkv;   // the items' row, key and child key: each place block's slice
                                   // of ipb items, grouped by range within the slice
    uint32_t *scnt;           // per slot of every range (ranges at slot_base): its key's offset count
    uint32_t *pdist;          // per range: distinct keys
    uint32_t *rstart;         // nparts + 1: exclusive scan of pdist (ranks)
    const GroupRoot *roots;   // nroots > 0: the group's root words, written by blocks after the place blocks
    int nroots;
    struct StatusDev *status;
};

// Result counts are added to kCountParts partial counters, each on its own
// 128-byte line, so that many workgroups adding at once do not queue on one
// address; the host sums them.
constexpr int kCountParts = 16;
constexpr int kPartStride = 16;   // 64-bit words between partial counters

// Host <-> device status block, one per context.
struct StatusDev {
    unsigned long long count;      // result tuples so far
    unsigned long long survivors;  // rows written to the output frontier by the last launch
    unsigned long long deferred;   // tuples waiting for a lazy force
    unsigned long long total;      // scan totals
    unsigned long long written;    // result rows materialized so far
    unsigned long long emit_base;  // the current emit's first output row
    unsigned long long emit_rows;  // the current emit's rows (within the output capacity)
    unsigned long long probe[FJ_MAX_NODES];
    unsigned long long hit[FJ_MAX_NODES];
    unsigned long long filtered;   // first-lookup probes the key filter settled
    uint32_t fq_n[FJ_MAX_ATOMS * kMaxLevels];  // force-queue lengths per (atom, level)
    uint32_t pending;              // entries whose cover had to be forced first
    uint32_t total32;              // 32-bit scan totals
    alignas(128) unsigned long long count_part[kCountParts * kPartStride];  // more result tuples
    uint32_t err_line;             // first failed device bounds check (source line)
    uint32_t err_count;            // failed device bounds checks
};

}  // namespace fj
