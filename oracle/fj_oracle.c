/*
 * fj_oracle.c -- plain C Free Join over COLT (oracle; TEST INFRASTRUCTURE ONLY).
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load this file's library.  It shares no code with the HIP executor.
 *
 * What it follows, in the paper's order:
 *   - COLT (Section 4.2, figure "colt-impl"): a trie whose leaves are vectors
 *     of row offsets into the base relation and whose inner nodes are hash
 *     maps from a key tuple to a child.  force() replaces a vector by a map
 *     keyed on the node's level variables, children being offset vectors.
 *     get() forces first; iter() on a vector iterates its offsets when the
 *     node is at the last level of its schema, and otherwise forces and
 *     iterates the keys.
 *   - The build phase (Section 3.3): every atom gets a COLT whose schema is
 *     the list of its subatoms' variable lists in plan order.  The root map
 *     is built up front except when the atom has a single level and that
 *     subatom is a pure cover of its node.  Such a root stays the base table
 *     (or its pushed-down selection): iterated directly when it is the
 *     cover, forced by its first get() when another cover wins (Section
 *     4.2: no auxiliary structure on a table nobody probes).  Every other
 *     root is forced before the join starts, which changes no result and
 *     differs from forcing it at its first get() (or non-suffix iter())
 *     only when no binding ever reaches that call.
 *   - The join phase (Section 3.3, figure "fj-algo") with vectorized batches
 *     of at most B cover tuples (Section 4.3): all lookups of one trie are
 *     done for the batch before the next trie, misses are dropped, then the
 *     survivors recurse one by one.
 *   - Dynamic covers (Section 4.4): among the node's pure covers, iterate the
 *     one whose current trie has the fewest keys (a forced map's key count,
 *     an unforced vector's length); ties go to the first in node order.
 *   - Bag semantics (Section 2.3 footnotes): multiplicities multiply.  A get
 *     that reaches a leaf offset vector multiplies the tuple's multiplicity
 *     by the vector's length; iterating a leaf-level map's keys multiplies by
 *     the child's length; iterating offsets contributes 1 per offset.
 *
 * Counters per node (OFJ_NCTR words): cover tuples, lookups (get calls),
 * hits, survivors, tries forced, offsets forced.  Forces done by the build
 * phase are charged to a separate slot after the last node.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OFJ_MAXC 8     /* columns per atom */
#define OFJ_MAXA 16    /* atoms per query  */
#define OFJ_MAXV 32    /* variables        */
#define OFJ_MAXN 32    /* plan nodes       */
#define OFJ_NCTR 6

enum { C_COVER = 0, C_PROBE, C_HIT, C_SURV, C_FORCED, C_FORCED_OFFS };

typedef struct Trie Trie;
struct Trie {
    int level;           /* schema level of this node's keys (or leaf) */
    int forced;
    /* vector form */
    uint32_t *offs;      /* NULL with iota != 0 for an unfiltered root */
    uint64_t len, cap_offs;
    int iota;
    /* map form */
    uint64_t nkeys, cap;
    int32_t *keys;       /* cap * kw values */
    Trie **slot_child;   /* cap; NULL = empty */
    uint64_t *order;     /* slot indices in insertion order, nkeys of them */
};

typedef struct {
    int natoms, nvars, nnodes, batch;
    int arity[OFJ_MAXA];
    int var_col[OFJ_MAXA][OFJ_MAXV];   /* column of variable v in atom a, or -1 */
    const int32_t *cols[OFJ_MAXA][OFJ_MAXC];
    /* schema: per atom, per level, the columns of its key */
    int nlev[OFJ_MAXA];
    int lev_nk[OFJ_MAXA][OFJ_MAXN];
    int lev_col[OFJ_MAXA][OFJ_MAXN][OFJ_MAXC];
    int lev_var[OFJ_MAXA][OFJ_MAXN][OFJ_MAXC];
    /* plan */
    int nsub[OFJ_MAXN];
    int sub_atom[OFJ_MAXN][OFJ_MAXA];
    int sub_level[OFJ_MAXN][OFJ_MAXA];
    int npure[OFJ_MAXN];
    int pure[OFJ_MAXN][OFJ_MAXA];      /* subatom indices within the node */
    /* output */
    int nhead;
    int head[OFJ_MAXV];
    uint64_t count, written, cap_out;
    int32_t *out;
    uint64_t *ctr;                     /* (nnodes + 1) * OFJ_NCTR or NULL */
    int oom;
} Ctx;

/* ------------------------------------------------------------------ tries */

static Trie *trie_new(int level) {
    Trie *t = (Trie *)calloc(1, sizeof(Trie));
    if (t) t->level = level;
    return t;
}

static void trie_free(Trie *t) {
    if (!t) return;
    if (t->forced) {
        for (uint64_t i = 0; i < t->cap; i++)
            if (t->slot_child[i]) trie_free(t->slot_child[i]);
        free(t->keys);
        free(t->slot_child);
        free(t->order);
    }
    free(t->offs);
    free(t);
}

static int push_offset(Trie *t, uint32_t off) {
    if (t->len == t->cap_offs) {
        uint64_t nc = t->cap_offs ? 2 * t->cap_offs : 4;
        uint32_t *p = (uint32_t *)realloc(t->offs, nc * sizeof(uint32_t));
        if (!p) return -1;
        t->offs = p;
        t->cap_offs = nc;
    }
    t->offs[t->len++] = off;
    return 0;
}

static uint64_t key_hash(const int32_t *k, int kw) {
    uint64_t h = 1469598103934665603ULL;          /* FNV-1a over the bytes */
    for (int i = 0; i < kw; i++) {
        uint32_t v = (uint32_t)k[i];
        for (int b = 0; b < 4; b++) {
            h ^= (v >> (8 * b)) & 0xFFu;
            h *= 1099511628211ULL;
        }
    }
    return h;
}

/* find the slot of key k (kw values) in map t; insert an empty child when
   absent and insert != 0.  Returns slot index or UINT64_MAX. */
static uint64_t map_find(Ctx *c, Trie *t, const int32_t *k, int kw, int insert);

static int map_grow(Ctx *c, Trie *t, int kw) {
    uint64_t ncap = t->cap ? 2 * t->cap : 8;
    int32_t *okeys = t->keys;
    Trie **ochild = t->slot_child;
    uint64_t *oorder = t->order;
    uint64_t onk = t->nkeys;
    t->keys = (int32_t *)malloc((ncap * (uint64_t)(kw ? kw : 1)) * sizeof(int32_t));
    t->slot_child = (Trie **)calloc(ncap, sizeof(Trie *));
    t->order = (uint64_t *)malloc(ncap * sizeof(uint64_t));
    if (!t->keys || !t->slot_child || !t->order) return -1;
    t->cap = ncap;
    t->nkeys = 0;
    for (uint64_t j = 0; j < onk; j++) {
        uint64_t s = oorder[j];
        uint64_t ns = map_find(c, t, okeys + s * (uint64_t)kw, kw, 1);
        t->slot_child[ns] = ochild[s];
    }
    free(okeys);
    free(ochild);
    free(oorder);
    return 0;
}

static uint64_t map_find(Ctx *c, Trie *t, const int32_t *k, int kw, int insert) {
    if (insert && 2 * (t->nkeys + 1) > t->cap) {
        if (map_grow(c, t, kw)) { c->oom = 1; return UINT64_MAX; }
    }
    if (t->cap == 0) return UINT64_MAX;
    uint64_t mask = t->cap - 1;
    uint64_t s = key_hash(k, kw) & mask;
    for (;;) {
        if (t->slot_child[s] == NULL) {
            if (!insert) return UINT64_MAX;
            memcpy(t->keys + s * (uint64_t)kw, k, sizeof(int32_t) * (size_t)kw);
            t->slot_child[s] = (Trie *)1;   /* placeholder, replaced by caller */
            t->order[t->nkeys++] = s;
            return s;
        }
        if (memcmp(t->keys + s * (uint64_t)kw, k, sizeof(int32_t) * (size_t)kw) == 0) return s;
        s = (s + 1) & mask;
    }
}

static uint32_t trie_offset(const Trie *t, uint64_t i) {
    return t->iota ? (uint32_t)i : t->offs[i];
}

static void load_key(Ctx *c, int a, int level, uint32_t row, int32_t *k) {
    for (int j = 0; j < c->lev_nk[a][level]; j++)
        k[j] = c->cols[a][c->lev_col[a][level][j]][row];
}

/* force(): replace the offset vector by a map on this level's key, whose
   children are offset vectors of the next level (Section 4.2). */
static void force(Ctx *c, int a, Trie *t, uint64_t *ctr) {
    if (t->forced) return;
    int kw = c->lev_nk[a][t->level];
    int32_t k[OFJ_MAXC];
    t->nkeys = 0;
    t->cap = 0;
    t->keys = NULL;
    t->slot_child = NULL;
    t->order = NULL;
    if (map_grow(c, t, kw)) { c->oom = 1; return; }
    for (uint64_t i = 0; i < t->len; i++) {
        uint32_t row = trie_offset(t, i);
        load_key(c, a, t->level, row, k);
        uint64_t before = t->nkeys;
        uint64_t s = map_find(c, t, k, kw, 1);
        if (s == UINT64_MAX) { c->oom = 1; return; }
        if (t->nkeys != before) {
            t->slot_child[s] = trie_new(t->level + 1);
            if (!t->slot_child[s]) { c->oom = 1; return; }
        }
        if (push_offset(t->slot_child[s], row)) { c->oom = 1; return; }
    }
    if (ctr) {
        ctr[C_FORCED] += 1;
        ctr[C_FORCED_OFFS] += t->len;
    }
    free(t->offs);
    t->offs = NULL;
    t->iota = 0;
    t->forced = 1;
}

static Trie *get(Ctx *c, int a, Trie *t, const int32_t *k, uint64_t *ctr) {
    force(c, a, t, ctr);
    if (c->oom) return NULL;
    uint64_t s = map_find(c, t, k, c->lev_nk[a][t->level], 0);
    return s == UINT64_MAX ? NULL : t->slot_child[s];
}

static uint64_t estimate(const Trie *t) {
    return t->forced ? t->nkeys : t->len;
}

/* --------------------------------------------------------------- join */

static void emit(Ctx *c, const int32_t *vals, uint64_t mult) {
    c->count += mult;
    while (mult-- && c->written < c->cap_out) {
        int32_t *row = c->out + c->written * (uint64_t)c->nhead;
        for (int j = 0; j < c->nhead; j++) row[j] = vals[c->head[j]];
        c->written++;
    }
}

typedef struct {
    int32_t vals[OFJ_MAXV];
    Trie *tries[OFJ_MAXA];
    uint64_t mult;
} Tup;

static void join(Ctx *c, int k, Trie **tries, const int32_t *vals, uint64_t mult);

static void run_batch(Ctx *c, int k, Tup *batch, int nb, int cover_sub) {
    uint64_t *ctr = c->ctr ? c->ctr + (uint64_t)k * OFJ_NCTR : NULL;
    int live[4096];
    int nlive = 0;
    for (int i = 0; i < nb; i++) live[nlive++] = i;
    /* probe trie by trie over the whole batch, dropping misses */
    for (int s = 0; s < c->nsub[k]; s++) {
        if (s == cover_sub) continue;
        int a = c->sub_atom[k][s];
        int lev = c->sub_level[k][s];
        int keep = 0;
        for (int ii = 0; ii < nlive; ii++) {
            Tup *tp = &batch[live[ii]];
            int32_t key[OFJ_MAXC];
            for (int j = 0; j < c->lev_nk[a][lev]; j++) key[j] = tp->vals[c->lev_var[a][lev][j]];
            if (ctr) ctr[C_PROBE]++;
            Trie *sub = get(c, a, tp->tries[a], key, ctr);
            if (c->oom) return;
            if (!sub) continue;
            if (ctr) ctr[C_HIT]++;
            if (sub->level == c->nlev[a]) {       /* leaf vector: a multiplicity */
                tp->mult *= sub->len;
                tp->tries[a] = NULL;
            } else {
                tp->tries[a] = sub;
            }
            live[keep++] = live[ii];
        }
        nlive = keep;
    }
    if (ctr) ctr[C_SURV] += (uint64_t)nlive;
    for (int ii = 0; ii < nlive; ii++) {
        Tup *tp = &batch[live[ii]];
        join(c, k + 1, tp->tries, tp->vals, tp->mult);
        if (c->oom) return;
    }
}

static void join(Ctx *c, int k, Trie **tries, const int32_t *vals, uint64_t mult) {
    if (k == c->nnodes) {
        emit(c, vals, mult);
        return;
    }
    uint64_t *ctr = c->ctr ? c->ctr + (uint64_t)k * OFJ_NCTR : NULL;
    /* dynamic cover: fewest keys among the pure covers, first on ties */
    int cover_sub = c->pure[k][0];
    uint64_t best = estimate(tries[c->sub_atom[k][cover_sub]]);
    for (int i = 1; i < c->npure[k]; i++) {
        int s = c->pure[k][i];
        uint64_t e = estimate(tries[c->sub_atom[k][s]]);
        if (e < best) { best = e; cover_sub = s; }
    }
    int ca = c->sub_atom[k][cover_sub];
    int clev = c->sub_level[k][cover_sub];
    Trie *ct = tries[ca];
    int by_offset = (!ct->forced && clev == c->nlev[ca] - 1);
    if (!by_offset) {
        force(c, ca, ct, ctr);
        if (c->oom) return;
    }
    uint64_t n = by_offset ? ct->len : ct->nkeys;
    if (n == 0) return;
    int B = c->batch;
    if ((uint64_t)B > n) B = (int)n;
    Tup *batch = (Tup *)malloc(sizeof(Tup) * (size_t)B);
    if (!batch) { c->oom = 1; return; }
    int nb = 0;
    for (uint64_t i = 0; i < n; i++) {
        Tup *tp = &batch[nb];
        memcpy(tp->vals, vals, sizeof(int32_t) * (size_t)c->nvars);
        memcpy(tp->tries, tries, sizeof(Trie *) * (size_t)c->natoms);
        tp->mult = mult;
        if (by_offset) {
            uint32_t row = trie_offset(ct, i);
            for (int j = 0; j < c->lev_nk[ca][clev]; j++)
                tp->vals[c->lev_var[ca][clev][j]] = c->cols[ca][c->lev_col[ca][clev][j]][row];
            tp->tries[ca] = NULL;                  /* consumed: last level */
        } else {
            uint64_t s = ct->order[i];
            const int32_t *key = ct->keys + s * (uint64_t)c->lev_nk[ca][clev];
            for (int j = 0; j < c->lev_nk[ca][clev]; j++) tp->vals[c->lev_var[ca][clev][j]] = key[j];
            Trie *child = ct->slot_child[s];
            if (child->level == c->nlev[ca]) {
                tp->mult *= child->len;
                tp->tries[ca] = NULL;
            } else {
                tp->tries[ca] = child;
            }
        }
        if (ctr) ctr[C_COVER]++;
        if (++nb == B) {
            run_batch(c, k, batch, nb, cover_sub);
            nb = 0;
            if (c->oom) { free(batch); return; }
        }
    }
    if (nb) run_batch(c, k, batch, nb, cover_sub);
    free(batch);
}

/* ----------------------------------------------------------------- API */

/*
 * Run a Free Join plan.  Plan subatoms are given flat in node order:
 * node_nsub[k] subatoms for node k; each has sub_atom, sub_nvars and
 * OFJ_MAXC entries of sub_vars.  Selection offsets (atom_sel[a]) replace the
 * root vector [0..nrows) when non-NULL.  Returns 0, or -1 on bad input, -2
 * when out of memory.  ``out`` receives min(count, cap) head-ordered rows.
 */
int ofj_execute(int natoms, const int32_t *atom_arity, const int32_t *atom_vars,
                const int32_t *const *atom_cols, const int64_t *atom_nrows,
                const uint32_t *const *atom_sel, const int64_t *atom_nsel,
                int nvars, int nnodes, const int32_t *node_nsub,
                const int32_t *sub_atom, const int32_t *sub_nvars, const int32_t *sub_vars,
                int batch, int nhead, const int32_t *head,
                uint64_t *count, int32_t *out, uint64_t cap, uint64_t *written,
                uint64_t *counters) {
    if (natoms < 1 || natoms > OFJ_MAXA || nvars < 1 || nvars > OFJ_MAXV ||
        nnodes < 1 || nnodes > OFJ_MAXN || batch < 1 || batch > 4096 ||
        nhead < 0 || nhead > OFJ_MAXV)
        return -1;
    Ctx *c = (Ctx *)calloc(1, sizeof(Ctx));
    if (!c) return -2;
    c->natoms = natoms; c->nvars = nvars; c->nnodes = nnodes; c->batch = batch;
    for (int a = 0; a < natoms; a++) {
        c->arity[a] = atom_arity[a];
        if (c->arity[a] < 0 || c->arity[a] > OFJ_MAXC) { free(c); return -1; }
        for (int v = 0; v < OFJ_MAXV; v++) c->var_col[a][v] = -1;
        for (int j = 0; j < c->arity[a]; j++) {
            int v = atom_vars[a * OFJ_MAXC + j];
            if (v < 0 || v >= nvars) { free(c); return -1; }
            c->var_col[a][v] = j;
            c->cols[a][j] = atom_cols[a * OFJ_MAXC + j];
        }
    }
    /* plan -> per-node subatoms and per-atom schema levels */
    int idx = 0;
    int bound[OFJ_MAXV] = {0};
    for (int k = 0; k < nnodes; k++) {
        c->nsub[k] = node_nsub[k];
        if (c->nsub[k] < 1 || c->nsub[k] > OFJ_MAXA) { free(c); return -1; }
        int isnew[OFJ_MAXV] = {0};
        for (int s = 0; s < c->nsub[k]; s++, idx++) {
            int a = sub_atom[idx];
            if (a < 0 || a >= natoms) { free(c); return -1; }
            int l = c->nlev[a]++;
            c->sub_atom[k][s] = a;
            c->sub_level[k][s] = l;
            c->lev_nk[a][l] = sub_nvars[idx];
            for (int j = 0; j < sub_nvars[idx]; j++) {
                int v = sub_vars[idx * OFJ_MAXC + j];
                if (v < 0 || v >= nvars || c->var_col[a][v] < 0) { free(c); return -1; }
                c->lev_var[a][l][j] = v;
                c->lev_col[a][l][j] = c->var_col[a][v];
                if (!bound[v]) isnew[v] = 1;
            }
        }
        /* pure covers: variables exactly the node's new variables */
        c->npure[k] = 0;
        for (int s = 0; s < c->nsub[k]; s++) {
            int a = c->sub_atom[k][s], l = c->sub_level[k][s];
            int has_bound = 0, nnew = 0, tot = 0;
            for (int v = 0; v < nvars; v++) tot += isnew[v];
            for (int j = 0; j < c->lev_nk[a][l]; j++) {
                int v = c->lev_var[a][l][j];
                if (bound[v]) has_bound = 1; else nnew++;
            }
            if (!has_bound && nnew == tot) c->pure[k][c->npure[k]++] = s;
        }
        if (c->npure[k] == 0) { free(c); return -1; }
        for (int v = 0; v < nvars; v++) if (isnew[v]) bound[v] = 1;
    }
    c->nhead = nhead;
    for (int j = 0; j < nhead; j++) c->head[j] = head[j];
    c->out = out;
    c->cap_out = out ? cap : 0;
    c->ctr = counters;
    if (counters) memset(counters, 0, sizeof(uint64_t) * (size_t)(nnodes + 1) * OFJ_NCTR);

    /* build phase: roots */
    Trie *roots[OFJ_MAXA] = {0};
    int rc = 0;
    for (int a = 0; a < natoms; a++) {
        Trie *t = trie_new(0);
        if (!t) { rc = -2; goto done; }
        roots[a] = t;
        if (atom_sel && atom_sel[a]) {
            t->len = (uint64_t)atom_nsel[a];
            t->offs = (uint32_t *)malloc(sizeof(uint32_t) * (t->len ? t->len : 1));
            if (!t->offs) { rc = -2; goto done; }
            memcpy(t->offs, atom_sel[a], sizeof(uint32_t) * t->len);
            t->cap_offs = t->len;
        } else {
            t->len = (uint64_t)atom_nrows[a];
            t->iota = 1;
        }
    }
    for (int a = 0; a < natoms; a++) {
        /* find the node holding the atom's first subatom */
        int built = 1;
        for (int k = 0; k < nnodes; k++) {
            int found = -1;
            for (int s = 0; s < c->nsub[k]; s++)
                if (c->sub_atom[k][s] == a && c->sub_level[k][s] == 0) found = s;
            if (found >= 0) {
                for (int i = 0; i < c->npure[k]; i++)
                    if (c->nlev[a] == 1 && c->pure[k][i] == found) built = 0;
                break;
            }
        }
        if (built) {
            force(c, a, roots[a], counters ? counters + (uint64_t)nnodes * OFJ_NCTR : NULL);
            if (c->oom) { rc = -2; goto done; }
        }
    }
    {
        int32_t vals[OFJ_MAXV] = {0};
        join(c, 0, roots, vals, 1);
        if (c->oom) rc = -2;
    }
done:
    if (count) *count = c->count;
    if (written) *written = c->written;
    for (int a = 0; a < natoms; a++) trie_free(roots[a]);
    free(c);
    return rc;
}
