// Bushy binary plans as a series of left-deep plans (Section 2.2): every
// join that is a right child is evaluated first and its result materialized
// as a relation over all its variables; the parent plan joins it as an atom.
// Each left-deep plan then goes through the usual conversion to Free Join
// (Section 4.1), COLT builds and execution.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "fj.h"
#include "fj_host.h"
#include "fj_launch.h"

namespace {

using u64 = unsigned long long;

struct Decomposed {
    std::vector<std::vector<int32_t>> plans;   // inputs: atom >= 0, or -(j + 1) for plan j
};

// Checks that b is a binary tree over distinct leaves and decomposes it.
fj_status decompose(const fj_bushy *b, Decomposed &d) {
    if (!b) return fj::set_error(FJ_ERR_ARG, "null plan");
    const int n = b->n;
    if (n < 1 || n > FJ_MAX_BUSHY || b->root < 0 || b->root >= n)
        return fj::set_error(FJ_ERR_ARG, "bushy plan size or root out of range");
    std::vector<int> parents(n, 0);
    std::vector<int> seen_atom;
    for (int i = 0; i < n; i++) {
        if (b->atom[i] >= 0) {
            if (b->atom[i] >= FJ_MAX_ATOMS) return fj::set_error(FJ_ERR_ARG, "leaf atom out of range");
            if (std::find(seen_atom.begin(), seen_atom.end(), b->atom[i]) != seen_atom.end())
                return fj::set_error(FJ_ERR_ARG, "an atom is a leaf twice");
            seen_atom.push_back(b->atom[i]);
        } else {
            const int l = b->left[i], r = b->right[i];
            if (l < 0 || l >= i || r < 0 || r >= i || l == r)
                return fj::set_error(FJ_ERR_ARG, "a join's children must be two earlier nodes");
            parents[l]++;
            parents[r]++;
        }
    }
    for (int i = 0; i < n; i++) {
        const int want = i == b->root ? 0 : 1;
        if (parents[i] != want) return fj::set_error(FJ_ERR_ARG, "the nodes do not form one tree under root");
    }
    if ((int)seen_atom.size() * 2 - 1 != n) return fj::set_error(FJ_ERR_ARG, "the nodes do not form one tree");
    // plan of node v: its left spine down to the first leaf, then every right
    // child on the way back up, a join child becoming a plan of its own first
    std::vector<std::vector<int32_t>> &plans = d.plans;
    auto build = [&](auto &&self, int v) -> int {
        std::vector<int> rights;   // the right children along the left spine, bottom-up
        int u = v;
        while (b->atom[u] < 0) {
            rights.push_back(b->right[u]);
            u = b->left[u];
        }
        std::vector<int32_t> inputs{b->atom[u]};
        for (int k = (int)rights.size() - 1; k >= 0; k--) {
            const int r = rights[k];
            if (b->atom[r] >= 0) inputs.push_back(b->atom[r]);
            else inputs.push_back(-(self(self, r) + 1));
        }
        plans.push_back(inputs);
        return (int)plans.size() - 1;
    };
    build(build, b->root);
    return FJ_OK;
}

// Device buffers returned to the pool on scope exit, once the context's
// stream has finished with them.
struct DevBufs {
    int device = 0;
    hipStream_t stream = nullptr;
    std::vector<std::pair<void *, size_t>> p;
    ~DevBufs() {
        if (!p.empty()) hipStreamSynchronize(stream);
        for (const auto &x : p) fj::pool_free(device, x.first, x.second);
    }
    fj_status alloc(void **out, size_t bytes) {
        bytes = std::max<size_t>(bytes, 4);
        fj_status st = fj::pool_alloc(device, bytes, out);
        if (st != FJ_OK) return st;
        p.push_back({*out, bytes});
        return FJ_OK;
    }
};

// A factorized intermediate, freed (before its plan's COLTs) on scope exit.
struct ResultGuard {
    fj_result *r = nullptr;
    ~ResultGuard() { fj_result_free(r); }
};

struct PlanColts {
    fj_plan *plan = nullptr;
    std::vector<fj_colt *> colts;
    ~PlanColts() {
        for (fj_colt *t : colts) fj_colt_free(t);
        if (plan) fj_plan_free(plan);
    }
};

}  // namespace

extern "C" fj_status fj_bushy_decompose(const fj_bushy *b, int32_t *nplans, int32_t *ninputs, int32_t *inputs) {
    if (!nplans || !ninputs || !inputs) return fj::set_error(FJ_ERR_ARG, "null argument");
    Decomposed d;
    fj_status st = decompose(b, d);
    if (st != FJ_OK) return st;
    *nplans = (int32_t)d.plans.size();
    for (size_t k = 0; k < d.plans.size(); k++) {
        ninputs[k] = (int32_t)d.plans[k].size();
        for (size_t i = 0; i < d.plans[k].size(); i++) inputs[k * FJ_MAX_ATOMS + i] = d.plans[k][i];
    }
    return FJ_OK;
}

extern "C" fj_status fj_execute_bushy(fj_ctx *ctx, const fj_query *q, const fj_bushy *b, const fj_relation *rels,
                                      uint32_t flags, uint64_t *count, int32_t *out, uint64_t cap,
                                      uint64_t *written) {
    if (!ctx || !q || !rels || !count) return fj::set_error(FJ_ERR_ARG, "null argument");
    if (q->natoms < 1 || q->natoms > FJ_MAX_ATOMS || q->nvars < 1 || q->nvars > FJ_MAX_VARS)
        return fj::set_error(FJ_ERR_ARG, "query size out of range");
    Decomposed d;
    fj_status st = decompose(b, d);
    if (st != FJ_OK) return st;
    for (int i = 0; i < b->n; i++)
        if (b->atom[i] >= q->natoms) return fj::set_error(FJ_ERR_ARG, "leaf atom out of range");
    if ((b->n + 1) / 2 != q->natoms) return fj::set_error(FJ_ERR_ARG, "the plan's leaves are not the query's atoms");
    if (hipSetDevice(fj::ctx_device(ctx)) != hipSuccess) return fj::set_error(FJ_ERR_HIP, "hipSetDevice failed");
    const hipStream_t s = fj::ctx_stream(ctx);
    DevBufs mem;
    mem.device = fj::ctx_device(ctx);
    mem.stream = s;
    const int np = (int)d.plans.size();
    // per plan: its variables (increasing original ids) and, once run, its
    // result as a relation
    std::vector<std::vector<int32_t>> pvars(np);
    std::vector<fj_relation> prel(np);
    for (int k = 0; k < np; k++) {
        const std::vector<int32_t> &in = d.plans[k];
        std::vector<int32_t> vars;
        for (int32_t x : in) {
            if (x >= 0) {
                for (int j = 0; j < q->atoms[x].arity; j++) vars.push_back(q->atoms[x].vars[j]);
            } else {
                const std::vector<int32_t> &v = pvars[-x - 1];
                vars.insert(vars.end(), v.begin(), v.end());
            }
        }
        std::sort(vars.begin(), vars.end());
        vars.erase(std::unique(vars.begin(), vars.end()), vars.end());
        pvars[k] = vars;
        const bool last = k == np - 1;
        if (!last && (int)vars.size() > FJ_MAX_COLS)
            return fj::set_error(FJ_ERR_UNSUPPORTED, "an intermediate would hold more than FJ_MAX_COLS variables");
        // the plan's own query over dense variable ids
        auto dense = [&](int32_t v) {
            return (int32_t)(std::lower_bound(vars.begin(), vars.end(), v) - vars.begin());
        };
        fj_query qk;
        memset(&qk, 0, sizeof(qk));
        qk.natoms = (int32_t)in.size();
        qk.nvars = (int32_t)vars.size();
        std::vector<fj_relation> rk(in.size());
        for (size_t i = 0; i < in.size(); i++) {
            fj_atom &A = qk.atoms[i];
            if (in[i] >= 0) {
                A.arity = q->atoms[in[i]].arity;
                for (int j = 0; j < A.arity; j++) A.vars[j] = dense(q->atoms[in[i]].vars[j]);
                rk[i] = rels[in[i]];
            } else {
                const int j0 = -in[i] - 1;
                A.arity = (int32_t)pvars[j0].size();
                for (int j = 0; j < A.arity; j++) A.vars[j] = dense(pvars[j0][j]);
                rk[i] = prel[j0];
            }
        }
        if (last) {
            if (q->nhead != q->nvars || (int)vars.size() != q->nvars)
                return fj::set_error(FJ_ERR_ARG, "the query's head must list every variable once");
            qk.nhead = q->nhead;
            for (int j = 0; j < q->nhead; j++) qk.head[j] = dense(q->head[j]);
        } else {
            qk.nhead = qk.nvars;
            for (int j = 0; j < qk.nvars; j++) qk.head[j] = j;
        }
        PlanColts pc;
        std::vector<int32_t> order(in.size());
        for (size_t i = 0; i < in.size(); i++) order[i] = (int32_t)i;
        st = fj_plan_from_binary(&qk, order.data(), (int32_t)order.size(), flags, &pc.plan);
        if (st != FJ_OK) return st;
        pc.colts.assign(in.size(), nullptr);
        for (size_t i = 0; i < in.size(); i++) {
            st = fj_build_colt(ctx, &qk, pc.plan, (int32_t)i, &rk[i], &pc.colts[i]);
            if (st != FJ_OK) return st;
        }
        if (last) return fj_execute(ctx, &qk, pc.plan, pc.colts.data(), count, out, cap, written, nullptr);
        // an intermediate: one run that keeps its result factorized (its
        // exact count known), then its rows expanded into a row-major
        // buffer and laid out as columns
        uint64_t n = 0, nbind = 0;
        ResultGuard rg;
        st = fj_execute_factorized(ctx, &qk, pc.plan, pc.colts.data(), &rg.r, &n, &nbind);
        if (st != FJ_OK) return st;
        if (n >= (uint64_t(1) << 31)) return fj::set_error(FJ_ERR_UNSUPPORTED, "an intermediate has 2^31 rows or more");
        const int m = qk.nvars;
        fj_relation &R = prel[k];
        memset(&R, 0, sizeof(R));
        R.ncols = m;
        R.nrows = (int64_t)n;
        int32_t *colp[FJ_MAX_COLS] = {nullptr};
        for (int j = 0; j < m; j++) {
            void *p = nullptr;
            st = mem.alloc(&p, n * sizeof(int32_t));
            if (st != FJ_OK) return st;
            colp[j] = (int32_t *)p;
            R.cols[j] = colp[j];
        }
        if (n == 0) continue;
        void *rows = nullptr;
        st = mem.alloc(&rows, n * (size_t)m * sizeof(int32_t));
        if (st != FJ_OK) return st;
        uint64_t w = 0;
        st = fj_result_expand(ctx, rg.r, 0, (int32_t *)rows, n, &w);
        if (st != FJ_OK) return st;
        if (w != n) return fj::set_error(FJ_ERR_INTERNAL, "an intermediate's expansion wrote fewer rows than its count");
        if (fj::launch_rows_to_cols((const int32_t *)rows, n, m, colp, s) != hipSuccess)
            return fj::set_error(FJ_ERR_HIP, "row to column launch failed");
        // the rows buffer is freed with the others when the call returns;
        // the stream keeps the transpose ahead of any later use
    }
    return FJ_OK;   // not reached: the last plan returns above
}
