// Kernel launchers of libfj (host-callable, stream-ordered).  Internal header.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "fj_dev.h"

namespace fj {

struct ForceLaunch {
    LevelDev L;            // level being forced
    LevelDev C;            // its child level
    const int32_t *cols[FJ_MAX_COLS];
    const uint32_t *fq;    // queued handle starts (device)
    uint32_t nh;
    const uint32_t *pre;   // exclusive scan of their lengths (device, nh + 1)
    uint32_t W;            // total offsets of the queued handles
    uint32_t *wslot;       // scratch, W entries
    unsigned long long *cntv, *ex;  // scratch, W and W + 1 entries
    uint32_t wcap;         // entries of each scratch array
    StatusDev *status;
};

struct ProbeLaunch {
    const NodeDev *nd;
    const unsigned long long *starts;
    const uint8_t *cov;
    uint32_t E;
    unsigned long long t0;
    uint32_t n;
    const uint32_t *din;
    const uint8_t *din_j;
    uint32_t *dout;
    uint8_t *dout_j;
    StatusDev *status;
    int count_stats;
    int block;
    uint32_t dcap;         // capacity of the deferral lists
    unsigned long long surv_base, def_base;  // counter values before the launch
    uint32_t *chunk_buf;   // scratch for the per-block binding bounds (chunk_cap entries), or null
    unsigned long long chunk_cap;
    int max_slots;         // variable slots of a binding (<= FJ_MAX_VARS)
    int max_atoms;         // atoms of the query (<= FJ_MAX_ATOMS)
};

struct ScanLaunch {
    const int32_t *cols[FJ_MAX_COLS];
    int ncols;
    const uint32_t *sel;
    uint32_t nrows;
    uint32_t r0;
    uint32_t n;
    int nl;
    ScanLookup lk[FJ_MAX_ATOMS];
    int nout;
    int out_col[FJ_MAX_VARS];
    FrontierDev out;
    int emit, materialize;
    int ntail;
    int tail_lk[FJ_MAX_NODES];
    const uint32_t *tail_len[FJ_MAX_NODES];
    uint32_t tail_npos[FJ_MAX_NODES];
    uint32_t tail_root_len[FJ_MAX_NODES];
    StatusDev *status;
    int count_stats;
    int node;
    unsigned long long surv_base;
    int direct;                // the kernel writes result rows itself (the first node emits)
    const void *ed;            // the execution's device emit descriptor (direct)
    unsigned long long cap;    // output capacity in rows (direct)
    // list of the first lookup's hits for a two-launch node (lk[0].bloom):
    // l0_cap entries of rows and of keys, kScanListGroups x kScanListWaves
    // counters; null: one launch without the filter
    uint32_t *l0_row, *l0_key, *l0_cnt;
    unsigned long long l0_cap;
    // the node's timing, or null: events the launches record themselves,
    // at the start of its first kernel and the end of its last
    hipEvent_t t_start, t_stop;
};

// The most filter-pass workgroups of a two-launch first node, the list's
// counters per workgroup (one per wave), and the list entries one over n
// cover positions needs.
constexpr uint32_t kScanListGroups = 4096;
constexpr uint32_t kScanListWaves = 16;
unsigned long long scan_list_entries(unsigned long long n);

hipError_t launch_scan_probe(const ScanLaunch &l, hipStream_t s);
int scan_max_lookups();
hipError_t launch_batch_dfs(const BQuery *qs, const BItem *items, uint32_t nitems, unsigned long long *counts,
                            StatusDev *status, int block, int grid, int lv, int la, hipStream_t s);
hipError_t launch_zero_u64(unsigned long long *p, uint32_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, unsigned long long n, uint32_t v, hipStream_t s);
hipError_t launch_fill_list(const FillList *fl_dev, unsigned long long total_words, const LevelDev &root,
                            uint32_t nroot, uint32_t *pre, hipStream_t s);
hipError_t launch_scan_u64(const unsigned long long *in, unsigned long long *out, unsigned long long n,
                           unsigned long long *bsum, unsigned long long *total, hipStream_t s);
hipError_t launch_scan_u32(const uint32_t *in, uint32_t *out, unsigned long long n, uint32_t *bsum,
                           uint32_t *total, hipStream_t s);
hipError_t launch_filter_lt(const int32_t *col, unsigned long long n, int32_t bound, uint32_t *out,
                            uint32_t *bsum, uint32_t *total, hipStream_t s);
// Block sums (32-bit words of bsum) launch_filter_lt uses for n rows.
unsigned long long filter_lt_blocks(unsigned long long n);
// Selections of n columns (each with its own bound, output and block-sum
// scratch of rows / 1024 + 1 words) in three launches; totals[i] receives
// selection i's row count.
// Queue every child trie of level L's forced tries on level C's force
// queue, counting them in *fq_n: root: the keys [0, nq) of L's one trie;
// otherwise the tries starting at positions [0, nq).
hipError_t launch_enqueue_children(const LevelDev &L, const LevelDev &C, uint32_t nq, int root, uint32_t *fq_n,
                                   StatusDev *st, hipStream_t s);
// Row-major rows (n x m int32, m <= FJ_MAX_COLS) to m column arrays of n.
hipError_t launch_rows_to_cols(const int32_t *rows, unsigned long long n, int m, int32_t *const *cols,
                               hipStream_t s);
hipError_t launch_filter_lt_group(int n, const int32_t *const *cols, const unsigned long long *rows,
                                  const int32_t *bounds, uint32_t *const *outs, uint32_t *const *bsums,
                                  uint32_t *const *totals, hipStream_t s);
hipError_t launch_fq_lens(const LevelDev &L, const uint32_t *fq, uint32_t nh, uint32_t *lens, StatusDev *st,
                          hipStream_t s);
hipError_t launch_force_phase(int phase, const ForceLaunch &f, hipStream_t s);
// Grouped builds of KM_K32 roots by key range, phase 0: place each slice of
// items grouped by range; 1: build each range; 2: rank the keys (after a
// scan of the distinct counts).
hipError_t launch_part_phase(int phase, const PartArgs &a, hipStream_t s);
// Exclusive scan of n u32 values in one workgroup (small n), out[n] = total.
hipError_t launch_scan_small_u32(const uint32_t *in, uint32_t *out, uint32_t n, hipStream_t s);
hipError_t launch_group_fill(const FillBlock *fb, uint32_t nblocks, const GroupRoot *roots, int n, hipStream_t s);
hipError_t launch_group_force(int phase, const ForceArgs *descs, const unsigned long long *wpre, int n,
                              unsigned long long wtot, hipStream_t s);
hipError_t launch_cover_choose(const NodeDev *nd, uint32_t E, uint8_t *cov, unsigned long long *cnt,
                               StatusDev *st, hipStream_t s);
hipError_t launch_cover_fill(const NodeDev *nd, uint32_t E, const uint8_t *cov, unsigned long long *cnt,
                             StatusDev *st, hipStream_t s);
hipError_t launch_probe(const ProbeLaunch &p, hipStream_t s);
// Counts, scan and output placement of E <= emit_small_max() bindings in
// one workgroup (starts has E + 1 entries).
hipError_t launch_emit_small_dev(const void *emit_dev, const unsigned long long *surv, unsigned long long surv_base,
                                 unsigned long long *starts, StatusDev *st, unsigned long long cap, hipStream_t s);
hipError_t launch_emit_count_small(const void *emit_dev, uint32_t E, unsigned long long *starts, StatusDev *st,
                                   unsigned long long cap, hipStream_t s);
uint32_t emit_small_max();
hipError_t launch_emit_count(const void *emit_dev, uint32_t E, unsigned long long *cnt, StatusDev *st,
                             hipStream_t s);
// Rows of the current emit (placed on the device by launch_scan_u64_emit),
// grid-stride over at most max_rows.
hipError_t launch_emit_rows(const void *emit_dev, uint32_t E, const unsigned long long *starts,
                            unsigned long long max_rows, StatusDev *st, hipStream_t s);
// Rows [first, first + n) of E bindings laid out by starts, to output rows
// [0, n) of the emit descriptor's output.
hipError_t launch_emit_range(const void *emit_dev, uint32_t E, const unsigned long long *starts,
                             unsigned long long first, unsigned long long n, StatusDev *st, hipStream_t s);
// Exclusive scan of an emit's n > 0 row counts that also places the emit in
// the output: st->emit_base = st->written, st->emit_rows = the total cut to
// cap rows, st->written advanced.
hipError_t launch_scan_u64_emit(const unsigned long long *in, unsigned long long *out, unsigned long long n,
                                unsigned long long *bsum, StatusDev *st, unsigned long long cap, hipStream_t s);
size_t emit_dev_size();
void emit_dev_fill(void *host_buf, const FrontierDev &F, const int *in_var, int nin, const int *in_h_atom,
                   int nin_h, const TailDev *tails, int ntail, const int *head_src, int nhead, int32_t *out,
                   unsigned long long out_rows);

// ---- learned plan chooser: column sketch and perceptron

constexpr int kSketchTop = 8;         // largest frequencies kept per column
constexpr int kSkDistinct = 0;        // result slots (u64) of a sketch
constexpr int kSkOther = 1;
constexpr int kSkTop = 2;
constexpr int kSketchRes = kSkTop + kSketchTop;

struct SketchLaunch {
    const int32_t *col;
    const uint32_t *sel;   // nullable: rows are sel[0..n) instead of 0..n
    uint32_t n;
    uint32_t *keys, *cnt;  // table of mask + 1 slots
    uint32_t mask;
    uint32_t *part;        // max_blocks * kSketchTop
    uint32_t max_blocks;
    unsigned long long *res;  // kSketchRes
};

hipError_t launch_sketch(const SketchLaunch &a, hipStream_t s);

hipError_t mlp_gemm(const float *A, const float *B, const float *bias, float *C, int M, int N, int K, bool ta,
                    bool tb, bool relu, bool accumulate, hipStream_t s);
hipError_t mlp_rows(const float *x, int B, int D, int H, const float *w, const int64_t off[6], float *y,
                    hipStream_t s);
hipError_t mlp_mse_grad(const float *y, const float *t, float *dy, float *sq, int B, hipStream_t s);
hipError_t mlp_relu_back(const float *h, float *dz, int n, hipStream_t s);
hipError_t mlp_colsum(const float *dz, float *db, int B, int N, hipStream_t s);
hipError_t mlp_sum(const float *x, int n, float *out, hipStream_t s);
hipError_t mlp_adam(float *w, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t s);

}  // namespace fj
