/*
 * fj.h -- C-ABI of the MI355X Free Join executor (libfj.so).
 *
 * The library runs Free Join plans over COLT indexes on one gfx950 GPU.
 * Its calls follow the paper's problem statement (Section 5 opening): a
 * full conjunctive query over column-stored relations plus a left-deep
 * binary plan, which is converted to a Free Join plan (Section 4.1), whose
 * COLT indexes are built (Section 3.3 build phase, Section 4.2), and which
 * is executed (Section 3.3 join phase, Section 4.3 vectorized batches,
 * Section 4.4 dynamic covers).
 *
 * Conventions for every call:
 *   - Device pointers are HIP device addresses on the context's device.
 *     Host pointers are ordinary process memory.  Each argument says which.
 *   - Relation columns and selection vectors are borrowed: the caller keeps
 *     them alive and unchanged for the lifetime of every COLT built on them
 *     (a COLT stores row offsets into the base relation, Section 4.2).
 *   - Plans, COLTs and contexts are owned by the library; free them with
 *     the matching *_free / *_destroy call.  Output buffers are the caller's.
 *   - Calls return an fj_status and never abort.  On a non-OK status,
 *     fj_last_error() returns a thread-local description.
 *   - Work is ordered on the context's HIP stream.  Calls that return host
 *     results synchronize that stream before returning.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef FJ_H
#define FJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FJ_OK = 0,
    FJ_TRUNCATED = 1,               /* count exact, output rows capped at cap */
    FJ_ERR_ARG = -1,                /* bad argument (null, size, range)      */
    FJ_ERR_PLAN_INVALID = -2,       /* Section 3.2 validity (a)/(b) fails    */
    FJ_ERR_PLAN_NO_PURE_COVER = -3, /* a node has no cover free of bound vars */
    FJ_ERR_OOM = -4,                /* device or host allocation failed      */
    FJ_ERR_HIP = -5,                /* a HIP runtime call failed             */
    FJ_ERR_UNSUPPORTED = -6,        /* outside the documented limits         */
    FJ_ERR_INTERNAL = -7            /* a device bounds check or an internal
                                       consistency check failed (a library bug) */
} fj_status;

#define FJ_MAX_COLS 8     /* columns per relation / variables per subatom */
#define FJ_MAX_ATOMS 16   /* atoms per query */
#define FJ_MAX_VARS 32    /* variables per query */
#define FJ_MAX_NODES 16   /* nodes per plan */

/* A (possibly filtered) column-stored relation.  cols[j] is a device array
   of nrows int32 values.  When sel is non-null it is a device array of nsel
   row offsets (each < nrows): the atom ranges over those rows only, which is
   how a pushed-down selection reaches the join (Section 2.1). */
typedef struct {
    int32_t ncols;
    int64_t nrows;                       /* < 2^31 */
    const int32_t *cols[FJ_MAX_COLS];    /* device, borrowed */
    const uint32_t *sel;                 /* device, borrowed, nullable */
    int64_t nsel;
} fj_relation;

/* One atom R_i(x_i) of Section 2.1, eq. "cq": vars[j] is the variable of
   column j.  The variables of one atom are distinct (selections such as
   R(x,x) are pushed down before the join, Section 2.1). */
typedef struct {
    int32_t arity;
    int32_t vars[FJ_MAX_COLS];
} fj_atom;

/* A full conjunctive query.  head lists every variable once, in the column
   order of materialized output rows.  Self-joins are separate atoms (the
   paper renames them, Section 2.1); they may share one relation's buffers. */
typedef struct {
    int32_t natoms;
    fj_atom atoms[FJ_MAX_ATOMS];
    int32_t nvars;
    int32_t nhead;
    int32_t head[FJ_MAX_VARS];
} fj_query;

typedef struct fj_ctx fj_ctx;
typedef struct fj_plan fj_plan;
typedef struct fj_colt fj_colt;

/* Execution options; zero fields take the defaults in brackets. */
typedef struct {
    int64_t tile;        /* max cover tuples per probe launch = frontier capacity [1<<24] */
    int32_t block;       /* threads per workgroup for probe kernels, 64..1024 [256] */
    int32_t timing;      /* time kernel classes with hipEvents: 0 off [default];
                            2: the node-0 probe (FJ_T_PROBE0) alone, two event
                            records per launch of it and none elsewhere; any
                            other nonzero value: every class */
    int32_t tail;        /* 0: multiply trailing single-cover nodes (default);
                            1: run every node through the probe kernel */
    int32_t generic;     /* 1: never use the specialised first-node scan kernel [0] */
    int32_t trie;        /* tries, for the paper's ablation (Section 5): 0: COLT [default]:
                            lazy, and a base table that is its node's only cover is
                            iterated directly; 1: simple lazy trie: every root map is
                            built ahead, inner levels lazily; 2: simple trie: every
                            level of every COLT is built when it is (re)built.
                            Batches take 0 only. */
    int32_t no_filter;   /* 1: the first-node scan never uses a root map's key filter
                            (the membership filter a range-by-range root build
                            writes beside its map) [0] */
    int32_t reserved[1];
} fj_options;

/* Per-execution counters (fj_execute fills them when stats is non-null).
   Index k is plan node k.  Counting lookups costs a few percent. */
typedef struct {
    uint64_t cover[FJ_MAX_NODES];        /* cover tuples iterated */
    uint64_t probe[FJ_MAX_NODES];        /* get() calls */
    uint64_t hit[FJ_MAX_NODES];          /* successful get() calls */
    uint64_t survivors[FJ_MAX_NODES];    /* tuples passing every lookup */
    uint64_t forced[FJ_MAX_NODES];       /* tries forced while running node k */
    uint64_t forced_offsets[FJ_MAX_NODES];
    int32_t tail_from;                   /* first node handled as a product */
    int32_t nnodes;
    uint64_t tiles;                      /* probe launches */
    uint64_t deferred;                   /* tuples re-run after a lazy force */
    uint64_t filtered;                   /* first-node probes settled as misses by the
                                            first lookup's key filter (counted in probe) */
} fj_stats;

/* Kernel-class timings accumulated since the last fj_timings_reset. */
typedef enum {
    FJ_T_FILTER = 0, FJ_T_BUILD, FJ_T_COVER, FJ_T_PROBE, FJ_T_PROBE0,
    FJ_T_FORCE, FJ_T_EMIT, FJ_T_SCAN, FJ_T_COUNT
} fj_timer;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  `stream` is a hipStream_t (or
   NULL for the default stream); the context does not own it.  opt may be
   NULL.  Returns FJ_ERR_HIP if the device cannot be selected. */
fj_status fj_ctx_create(int device, void *stream, const fj_options *opt, fj_ctx **out);
void fj_ctx_destroy(fj_ctx *ctx);

/* Thread-local message for the last non-OK status of this thread. */
const char *fj_last_error(void);

/* Accumulated milliseconds and launch counts per fj_timer class (host
   arrays of FJ_T_COUNT entries); timing must be enabled in the options.
   Synchronizes the stream. */
fj_status fj_timings(fj_ctx *ctx, double *ms, uint64_t *launches);
fj_status fj_timings_reset(fj_ctx *ctx);

/* Change the context's timing mode (the values of fj_options.timing) for
   the calls that follow; timings already taken are kept.  FJ_ERR_ARG for a
   null context or a mode other than 0, 1 or 2.  Host only. */
fj_status fj_set_timing(fj_ctx *ctx, int32_t mode);

/* -------------------------------------------------------------------- plans */

#define FJ_FACTOR 1u   /* apply conservative factoring (Section 4.1) */

/* Convert the left-deep binary plan [R_order[0], ..., R_order[n-1]] (atom
   indices, each atom once) into a Free Join plan (Section 4.1, figure
   "bj2fj"), then factor it when flags has FJ_FACTOR (figure
   "factorize-plan").  The result is validated (Section 3.2).  q and order
   are host memory. */
fj_status fj_plan_from_binary(const fj_query *q, const int32_t *order, int32_t n,
                              uint32_t flags, fj_plan **out);

/* Build a plan from explicit nodes (Section 3.2 definition): node k has
   node_nsub[k] subatoms, listed flat in node order; subatom i belongs to
   atom sub_atom[i] and has sub_nvars[i] variables sub_vars[i*FJ_MAX_COLS+j].
   Returns FJ_ERR_PLAN_INVALID when the nodes do not partition every atom
   or validity (a)/(b) fails, FJ_ERR_PLAN_NO_PURE_COVER when some node has
   no cover whose variables are all new.  All arrays are host memory. */
fj_status fj_plan_from_nodes(const fj_query *q, int32_t nnodes, const int32_t *node_nsub,
                             const int32_t *sub_atom, const int32_t *sub_nvars,
                             const int32_t *sub_vars, fj_plan **out);

/* Read a plan back in the fj_plan_from_nodes layout (host arrays with room
   for cap_sub subatoms; node_nsub needs FJ_MAX_NODES entries). */
fj_status fj_plan_get(const fj_plan *p, int32_t *nnodes, int32_t *node_nsub, int32_t *sub_atom,
                      int32_t *sub_nvars, int32_t *sub_vars, int32_t cap_sub);
void fj_plan_free(fj_plan *p);

/* ---------------------------------------------------------------- selection */

/* Pushed-down selection sigma_{col < bound} (Section 2.1): writes the row
   offsets r with col[r] < bound into out_sel (device, capacity nrows) in
   row order and their number to *out_n (host).  col is device. */
fj_status fj_filter_lt(fj_ctx *ctx, const int32_t *col, int64_t nrows, int32_t bound,
                       uint32_t *out_sel, int64_t *out_n);

/* fj_filter_lt for callers that cannot allocate device memory (code under
   stream capture, tight serving loops, harnesses that forbid hipMalloc):
   the same selection, same arguments and same result, but its block sums
   live in a fixed 256 KiB device array that the library holds on each GPU
   until the process ends (its address is looked up when a context is
   created on that GPU), and the call makes no allocation.  nrows is at
   most 67,108,864 (65,536 blocks of 1,024 rows); larger inputs return
   FJ_ERR_UNSUPPORTED before any device work.  Every call on one GPU shares
   that GPU's array: calls that overlap on one GPU (other threads or
   streams) race and must be serialized by the caller.  Synchronizes the
   context's stream. */
fj_status fj_filter_lt_noalloc(fj_ctx *ctx, const int32_t *col, int64_t nrows, int32_t bound,
                               uint32_t *out_sel, int64_t *out_n);

/* Several selections with one synchronization: selection i keeps the rows
   r < nrows[i] of device column cols[i] with cols[i][r] < bounds[i], writing
   their offsets to outs[i] (device, capacity nrows[i]) in row order and
   their number to counts[i] (host).  n <= FJ_MAX_ATOMS. */
fj_status fj_filter_lt_batch(fj_ctx *ctx, int32_t n, const int32_t *const *cols, const int64_t *nrows,
                             const int32_t *bounds, uint32_t *const *outs, int64_t *counts);

/* -------------------------------------------------------------------- COLTs */

/* Build phase (Section 3.3) for atom `atom` of q under plan p: the COLT's
   schema is the atom's subatom variable lists in plan order (Section 4.2).
   Its root map is built now, on the GPU, unless the atom's first subatom is
   both its only level and the only pure cover of its node; then the base
   table (or rel->sel) is iterated directly (Section 4.2).  Deeper levels are
   forced lazily during fj_execute.  rel describes the relation; its column
   pointers are borrowed.  Device memory for the index is allocated here. */
fj_status fj_build_colt(fj_ctx *ctx, const fj_query *q, const fj_plan *p, int32_t atom,
                        const fj_relation *rel, fj_colt **out);

/* Return a COLT to its just-built state (root rebuilt, inner levels
   unforced) without reallocating; rel may change its row count only
   downward and must keep its arity. */
fj_status fj_colt_rebuild(fj_ctx *ctx, fj_colt *colt, const fj_relation *rel);
/* Rebuild n COLTs at once (as fj_colt_rebuild for each colts[k] with
   rels[k], host arrays): every root build runs in the same few launches.
   No COLT may appear twice.  Device scratch for the combined root rows is
   owned by the context and grows when needed. */
fj_status fj_colt_rebuild_many(fj_ctx *ctx, int32_t n, fj_colt *const *colts, const fj_relation *rels);
/* Pushed-down selections (Section 2.1) and then the build phase (Section 3.3)
   over the selected rows, in one call with one host wait between: the
   selections' counts size the maps.  Selection i keeps the rows
   r < rels[atoms[i]].nrows of column rels[atoms[i]].cols[cols[i]] whose value
   is below bounds[i], writing their offsets in row order to
   rels[atoms[i]].sel (a device buffer of nrows entries, which must be
   non-null; it is written although the field is const) and their number to
   rels[atoms[i]].nsel; then as fj_colt_rebuild_many(ctx, n, colts, rels).
   nsel <= FJ_MAX_ATOMS, each atoms[i] in [0, n) and listed once.  On an error
   after the selections ran, their counts are already in rels. */
fj_status fj_select_rebuild(fj_ctx *ctx, int32_t nsel, const int32_t *atoms, const int32_t *cols,
                            const int32_t *bounds, int32_t n, fj_colt *const *colts, fj_relation *rels);
void fj_colt_free(fj_colt *colt);

/* --------------------------------------------------------------------- join */

/* Join phase (Section 3.3, figure "fj-algo"; Section 4.3; Section 4.4).
   colts: host array of q->natoms COLTs built for this q and p.  *count
   (host) receives the exact number of result tuples under bag semantics.
   If out (device, row-major cap x q->nhead int32) is non-null, min(count,
   cap) result rows in head order are written to out[0 .. *written) in
   unspecified order; FJ_TRUNCATED is returned when count > cap.  stats
   (host) is optional. */
fj_status fj_execute(fj_ctx *ctx, const fj_query *q, const fj_plan *p, fj_colt *const *colts,
                     uint64_t *count, int32_t *out, uint64_t cap, uint64_t *written,
                     fj_stats *stats);

/* ------------------------------------------------------- factorized results */

typedef struct fj_result fj_result;

/* Join phase that keeps the result factorized (Section 4.4's view of a trie
   as a factorized relation, used in Section 5.2 to avoid building large
   outputs): the final bindings of the plan's last enumerated node are
   kept, each standing for its multiplicity times the product of its
   trailing tries' lengths, instead of being expanded into rows.  *count
   (host) receives the exact result count and *bindings (host, nullable)
   the number of bindings kept.  The result reads the COLTs' tries and
   their relations' columns when it is expanded: the COLTs and the columns
   must stay alive, and the COLTs must not be rebuilt, until fj_result_free.
   Device memory for the bindings is owned by the result (pooled).  Errors:
   FJ_ERR_ARG for null arguments or those fj_execute refuses,
   FJ_ERR_UNSUPPORTED for 2^32 bindings or more; *out is then null. */
fj_status fj_execute_factorized(fj_ctx *ctx, const fj_query *q, const fj_plan *p, fj_colt *const *colts,
                                fj_result **out, uint64_t *count, uint64_t *bindings);

/* Rows [first, first + n) of a factorized result, in head order, written
   row-major to out (device, cap x q->nhead int32) with n = min(cap, count -
   first); *written (host) receives n, 0 when first >= count.  Rows keep
   one fixed order across calls, so pages of consecutive ranges cover the
   result exactly once.  The first call also counts every binding's rows
   (device memory of 8 bytes per binding, kept with the result).  ctx must
   be on the result's device (FJ_ERR_ARG otherwise); calls on one result
   must not overlap. */
fj_status fj_result_expand(fj_ctx *ctx, fj_result *r, uint64_t first, int32_t *out, uint64_t cap,
                           uint64_t *written);
/* Frees the result and its device memory (null is a no-op). */
void fj_result_free(fj_result *r);

/* ------------------------------------------------------------- bushy plans */

#define FJ_MAX_BUSHY (2 * FJ_MAX_ATOMS - 1)   /* nodes of a binary join tree */

/* A binary join plan over a query's atoms (Section 2.2), bushy or not.
   Node i is a leaf when atom[i] >= 0 (that atom of the query) and otherwise
   the join of nodes left[i] and right[i], both below i.  root is the whole
   plan.  Every node but the root is the child of exactly one join and
   every atom of the query is exactly one leaf. */
typedef struct {
    int32_t n;
    int32_t root;
    int32_t atom[FJ_MAX_BUSHY];
    int32_t left[FJ_MAX_BUSHY];
    int32_t right[FJ_MAX_BUSHY];
} fj_bushy;

/* Split a binary plan into left-deep plans (Section 2.2).  A join whose
   result feeds its parent from the right, with the subtree under it, is
   run as a plan of its own, ahead of the plan that consumes it, and its
   result is materialized as a relation; what remains of each tree along
   its left edge, read from the bottom, is that plan's left-deep order.  Writes the plans in evaluation order (the whole plan
   last) to *nplans (host) and, for plan k, its inputs in left-deep order to
   inputs[k * FJ_MAX_ATOMS + i] (host, FJ_MAX_BUSHY * FJ_MAX_ATOMS entries)
   with their number in ninputs[k] (host, FJ_MAX_BUSHY entries): an input
   is an atom index (>= 0) or -(j + 1) for the result of plan j < k.
   Returns FJ_ERR_ARG when b is not a tree of the form above.  Host only. */
fj_status fj_bushy_decompose(const fj_bushy *b, int32_t *nplans, int32_t *ninputs, int32_t *inputs);

/* Run a binary plan by its decomposition.  Every plan is converted (and
   factored when flags has FJ_FACTOR) as by fj_plan_from_binary, its COLTs
   are built, and it is executed; each plan but the last has its result
   materialized on the device as a relation over all its variables (columns
   in increasing variable order, as the paper keeps every attribute of an
   intermediate), which the later plans join as an atom.  The last plan's
   result is the query's: count, out, cap and written as for fj_execute.
   rels: host array of q->natoms relations (device columns).  Intermediates
   are allocated and freed inside the call.  FJ_ERR_UNSUPPORTED when an
   intermediate has more than FJ_MAX_COLS variables or 2^31 rows or more. */
fj_status fj_execute_bushy(fj_ctx *ctx, const fj_query *q, const fj_bushy *b, const fj_relation *rels,
                           uint32_t flags, uint64_t *count, int32_t *out, uint64_t cap, uint64_t *written);

/* ------------------------------------------------------------------ batches */

typedef struct fj_batch fj_batch;

/* Batch options; zero fields take the defaults in brackets. */
typedef struct {
    int32_t chunk;       /* first-node rows per work item [1024] */
    int32_t block;       /* threads per workgroup, a multiple of 64, <= 512 [256] */
    int32_t no_graph;    /* nonzero: launch directly instead of replaying a hipGraph [0] */
    int32_t no_rebuild;  /* nonzero: runs reuse the COLTs as built instead of rebuilding [0] */
    int32_t reserved[3];
    const int32_t *query_chunk;  /* optional host array of n per-query chunks (0: use chunk) */
} fj_batch_options;

/* Prepare n independent queries for counting together.  qs[i], plans[i]
   and colts[i] (a host array of qs[i]->natoms COLTs) are as for
   fj_execute and must stay alive for the batch's lifetime.  Every plan must
   probe only root maps keyed by one or two variables, with each later node
   iterating the sub-trie a previous node reached (the shape of plans
   converted from left-deep binary plans, Section 4.1); other plans give
   FJ_ERR_UNSUPPORTED.  The whole run (optional COLT rebuilds and one
   persistent kernel draining a static queue of (query, row chunk) work
   items, largest first) is captured once in a hipGraph.  Each node iterates
   a fixed cover (its first subatom when that is a pure cover, as in the
   binary plan it came from) instead of choosing one per binding. */
fj_status fj_batch_create(fj_ctx *ctx, int32_t n, const fj_query *const *qs, const fj_plan *const *plans,
                          fj_colt *const *const *colts, const fj_batch_options *opt, fj_batch **out);

/* Run the batch: counts (host, n entries) receive each query's exact result
   count.  Synchronizes the context's stream. */
fj_status fj_batch_run(fj_batch *b, uint64_t *counts);
void fj_batch_free(fj_batch *b);

/* ------------------------------------------------------- column statistics */

#define FJ_SKETCH_TOPK 8

/* Exact statistics of the rows an atom ranges over: the learned plan
   chooser's inputs and the cardinality estimates of the greedy left-deep
   optimizer below.  top[j] holds the FJ_SKETCH_TOPK largest frequencies of
   the values of column j in descending order (zero-padded when the column
   has fewer distinct values). */
typedef struct {
    int64_t rows;                                /* rel->nsel when sel is set, else nrows */
    int32_t ncols;
    int64_t distinct[FJ_MAX_COLS];
    int64_t top[FJ_MAX_COLS][FJ_SKETCH_TOPK];
} fj_sketch;

/* Count, on the GPU, the distinct values of every column of rel (over
   rel->sel when set) and their largest frequencies into *out (host).  Uses
   a hash table of at least 2 x rows slots of 8 bytes in device scratch owned
   by the context.  Synchronizes the stream. */
fj_status fj_sketch_relation(fj_ctx *ctx, const fj_relation *rel, fj_sketch *out);

/* ----------------------------------------------------------- plan choosing */

/* Greedy left-deep join order from textbook estimates, the stand-in for the
   cost-based optimizer that produces the binary plans Section 4.1 converts.
   The order starts at atom `first`, or at the atom with the most rows when
   first < 0 (a traditional binary plan iterates its largest relation,
   Section 4.4); then it repeatedly appends the remaining atom sharing a
   variable with those already placed that minimizes the estimate
   |J| |R| / prod over shared v of max(V(J,v), V(R,v)), where V is a
   distinct count and V(J,v) is the smallest V over placed atoms holding v;
   an atom sharing nothing is taken only when nothing connected is left, the
   smallest first.  Ties go to the lower atom index.  sk: host array of
   q->natoms sketches; order: host array receiving q->natoms atom indices. */
fj_status fj_greedy_order(const fj_query *q, const fj_sketch *sk, int32_t first, int32_t *order);

#define FJ_CAND_MAX 32
#define FJ_FEATURES 128
#define FJ_CAND_BINARY 0   /* left-deep order, converted and factored (Section 4.1) */
#define FJ_CAND_GJ 1       /* Generic Join plan: one variable per node (Section 3.2, eq. "gj") */

typedef struct {
    int32_t kind;                /* FJ_CAND_BINARY or FJ_CAND_GJ */
    int32_t n;                   /* entries of order */
    int32_t order[FJ_MAX_VARS];  /* atom order (binary) or variable order (GJ) */
} fj_candidate;

/* Enumerate candidate Free Join plans for q and describe each by a row of
   FJ_FEATURES floats.  Candidate 0 is always the plain plan: the greedy
   order from the largest atom, converted and factored.  Then, for every
   start atom, the greedy order from it (converted and factored), and the
   Generic Join plan over the variable order that order induces (variables
   by first appearance); duplicates are dropped and at most cap (<=
   FJ_CAND_MAX) are kept.  The features hold the plan's shape, per-atom
   statistics in plan order (rows, distinct counts, top frequencies, whether
   the root map is built, trie depth) and per-node textbook estimates of
   frontier and cover sizes.  All arrays are host memory; features has room
   for cap x FJ_FEATURES floats. */
fj_status fj_plan_candidates(const fj_query *q, const fj_sketch *sk, int32_t cap, fj_candidate *out, int32_t *n,
                             float *features);

/* The plan of a candidate (as fj_plan_from_binary / fj_plan_from_nodes). */
fj_status fj_candidate_plan(const fj_query *q, const fj_candidate *c, fj_plan **out);

/* ------------------------------------------------------------ perceptron */

typedef struct fj_mlp fj_mlp;

/* A three-layer FP32 perceptron y = W3 relu(W2 relu(W1 x + b1) + b2) + b3
   (in_dim -> hidden -> hidden -> 1) trained on the GPU by the library's own
   kernels, here to predict the run time of a candidate plan from its
   features.  Parameters are one host-visible vector in the order W1 (in_dim
   x hidden, row-major), b1, W2 (hidden x hidden), b2, W3 (hidden), b3;
   they start at zero.  in_dim and hidden are 1..1024.  Device buffers grow
   with the largest batch seen. */
fj_status fj_mlp_create(fj_ctx *ctx, int32_t in_dim, int32_t hidden, fj_mlp **out);
int64_t fj_mlp_param_count(const fj_mlp *m);
/* Copy n = fj_mlp_param_count(m) host floats in / out.  Setting parameters
   also clears the optimizer state. */
fj_status fj_mlp_set_params(fj_mlp *m, const float *params, int64_t n);
fj_status fj_mlp_get_params(fj_mlp *m, float *params, int64_t n);
/* y[i] = f(x[i]) for batch rows: x is device batch x in_dim row-major, y is
   device batch floats.  Stream-ordered, no synchronization. */
fj_status fj_mlp_forward(fj_mlp *m, const float *x, int32_t batch, float *y);
/* Gradient of the mean squared error (1/batch) sum_i (f(x[i]) - t[i])^2
   with respect to every parameter, in parameter order, into grad (host,
   param_count floats), and the loss into *loss (host).  x and t are device.
   Synchronizes the stream. */
fj_status fj_mlp_gradient(fj_mlp *m, const float *x, const float *t, int32_t batch, float *grad, float *loss);
/* One Adam step (beta1 0.9, beta2 0.999, epsilon 1e-8, bias-corrected)
   with learning rate lr on that loss.  *loss (host, nullable) receives the
   loss before the step, which synchronizes the stream; without it the call
   only enqueues work. */
fj_status fj_mlp_train_step(fj_mlp *m, const float *x, const float *t, int32_t batch, float lr, float *loss);
void fj_mlp_free(fj_mlp *m);

/* Learned choice: enumerate the candidates of q (fj_plan_candidates),
   score them with m on the GPU and return in *out the plan with the lowest
   predicted time, unless it beats the plain plan (candidate 0) by less than
   `margin` in the model's output units, or q has more atoms than the
   features describe (6), or m is NULL: then the plain converted plan is
   returned.  A query whose atoms hold fewer than gate_rows rows in all (by
   the sketches) gets the plain plan without enumeration or scoring: where
   every plan is fast, choosing costs more than it can gain (0: no gate).
   *chosen (host, nullable) receives the candidate index (0 when gated),
   scores (host, nullable, FJ_CAND_MAX floats) the predictions (untouched
   when gated).  Synchronizes when it scores. */
fj_status fj_choose_plan(fj_ctx *ctx, fj_mlp *m, const fj_query *q, const fj_sketch *sk, float margin,
                         uint64_t gate_rows, fj_plan **out, int32_t *chosen, float *scores);

#ifdef __cplusplus
}
#endif

#endif /* FJ_H */
