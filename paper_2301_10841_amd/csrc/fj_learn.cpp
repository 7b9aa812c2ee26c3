// libfj: the learned plan chooser.  A greedy left-deep optimizer over
// textbook estimates (the source of the plain binary plan that Section 4.1
// converts), the enumeration of candidate Free Join plans with their feature
// rows, the perceptron that scores them (trained and run on the GPU by the
// kernels in fj_learn.hip), and the choice itself with the plain converted
// plan as its fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <limits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "fj.h"
#include "fj_host.h"
#include "fj_launch.h"
#include "fj_plan.h"

using fj::set_error;

#define FJ_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return set_error(e_ == hipErrorOutOfMemory ? FJ_ERR_OOM : FJ_ERR_HIP,              \
                             std::string(#call) + ": " + hipGetErrorString(e_));               \
    } while (0)

#define FJ_TRY(expr)                         \
    do {                                     \
        fj_status s_ = (expr);               \
        if (s_ != FJ_OK) return s_;          \
    } while (0)

namespace {

constexpr int kSlots = 6;        // atoms described in a feature row
constexpr int kSlotF = 12;       // features per atom
constexpr int kNodeSlots = 8;    // nodes described in a feature row
constexpr int kNodeF = 4;        // features per node
constexpr int kAtomBase = 16;
constexpr int kNodeBase = kAtomBase + kSlots * kSlotF;   // 88
constexpr int kTailBase = kNodeBase + kNodeSlots * kNodeF;  // 120
static_assert(kTailBase + 8 == FJ_FEATURES, "feature layout");

// log2(1 + x) / 32: counts up to 2^32 map into [0, 1]
inline float lg(double x) { return (float)(std::log2(1.0 + std::max(x, 0.0)) / 32.0); }

int col_of(const fj_query &q, int a, int v) {
    for (int j = 0; j < q.atoms[a].arity; j++)
        if (q.atoms[a].vars[j] == v) return j;
    return -1;
}

double rows_of(const fj_sketch *sk, int a) { return std::max<double>(1.0, (double)sk[a].rows); }

// distinct values of variable v's column in atom a (at least 1)
double dist_of(const fj_query &q, const fj_sketch *sk, int a, int v) {
    const int j = col_of(q, a, v);
    if (j < 0) return 1.0;
    return std::max<double>(1.0, (double)sk[a].distinct[j]);
}

// distinct combinations of a set of variables of atom a under independence,
// capped at the atom's rows
double dist_set(const fj_query &q, const fj_sketch *sk, int a, const int *vars, int nv) {
    double p = 1.0;
    for (int i = 0; i < nv; i++) p *= dist_of(q, sk, a, vars[i]);
    return std::min(p, rows_of(sk, a));
}

fj_status check_sketches(const fj_query *q, const fj_sketch *sk) {
    if (!q || !sk) return set_error(FJ_ERR_ARG, "null argument");
    if (q->natoms < 1 || q->natoms > FJ_MAX_ATOMS) return set_error(FJ_ERR_ARG, "natoms out of range");
    for (int a = 0; a < q->natoms; a++) {
        if (sk[a].ncols != q->atoms[a].arity) return set_error(FJ_ERR_ARG, "sketch arity differs from the atom's");
        if (sk[a].rows < 0) return set_error(FJ_ERR_ARG, "negative rows in a sketch");
    }
    return FJ_OK;
}

// The greedy left-deep order (the estimate is evaluated as (|J| |R|) / P,
// with P multiplied over the atom's columns in column order).
void greedy(const fj_query &q, const fj_sketch *sk, int first, std::vector<int> &order) {
    const int n = q.natoms;
    std::vector<char> used(n, 0);
    std::vector<double> vj(FJ_MAX_VARS, 0.0);  // 0: variable not yet bound
    double J = 0.0;
    order.clear();
    auto place = [&](int a, double est) {
        const bool firstp = order.empty();
        J = firstp ? rows_of(sk, a) : est;
        for (int j = 0; j < q.atoms[a].arity; j++) {
            const int v = q.atoms[a].vars[j];
            const double d = dist_of(q, sk, a, v);
            vj[v] = vj[v] > 0.0 ? std::min(vj[v], d) : d;
        }
        for (int v = 0; v < FJ_MAX_VARS; v++)
            if (vj[v] > 0.0) vj[v] = std::max(1.0, std::min(vj[v], J));
        used[a] = 1;
        order.push_back(a);
    };
    if (first < 0) {
        first = 0;
        for (int a = 1; a < n; a++)
            if (sk[a].rows > sk[first].rows) first = a;
    }
    place(first, 0.0);
    while ((int)order.size() < n) {
        int best = -1;
        double best_est = 0.0;
        for (int a = 0; a < n; a++) {
            if (used[a]) continue;
            bool shared = false;
            double P = 1.0;
            for (int j = 0; j < q.atoms[a].arity; j++) {
                const int v = q.atoms[a].vars[j];
                if (vj[v] > 0.0) {
                    shared = true;
                    P *= std::max(vj[v], dist_of(q, sk, a, v));
                }
            }
            if (!shared) continue;
            const double est = (J * rows_of(sk, a)) / P;
            if (best < 0 || est < best_est) { best = a; best_est = est; }
        }
        if (best < 0) {  // nothing connected: the smallest remaining atom
            for (int a = 0; a < n; a++) {
                if (used[a]) continue;
                if (best < 0 || sk[a].rows < sk[best].rows) best = a;
            }
            best_est = J * rows_of(sk, best);
        }
        place(best, best_est);
    }
}

// GYO reduction: true when the query's hypergraph is cyclic
bool cyclic(const fj_query &q) {
    std::vector<std::vector<int>> e(q.natoms);
    for (int a = 0; a < q.natoms; a++) e[a].assign(q.atoms[a].vars, q.atoms[a].vars + q.atoms[a].arity);
    std::vector<char> alive(q.natoms, 1);
    bool changed = true;
    while (changed) {
        changed = false;
        // drop variables that occur in one live edge only
        for (int a = 0; a < q.natoms; a++) {
            if (!alive[a]) continue;
            std::vector<int> keep;
            for (int v : e[a]) {
                int occ = 0;
                for (int b = 0; b < q.natoms; b++)
                    if (alive[b] && std::find(e[b].begin(), e[b].end(), v) != e[b].end()) occ++;
                if (occ > 1) keep.push_back(v);
            }
            if (keep.size() != e[a].size()) { e[a] = keep; changed = true; }
        }
        // drop edges contained in another live edge
        for (int a = 0; a < q.natoms; a++) {
            if (!alive[a]) continue;
            for (int b = 0; b < q.natoms; b++) {
                if (b == a || !alive[b]) continue;
                bool sub = true;
                for (int v : e[a])
                    if (std::find(e[b].begin(), e[b].end(), v) == e[b].end()) { sub = false; break; }
                if (sub) { alive[a] = 0; changed = true; break; }
            }
        }
    }
    int left = 0;
    for (int a = 0; a < q.natoms; a++) left += alive[a];
    return left > 1;
}

struct Est {
    double ein[FJ_MAX_NODES], cov[FJ_MAX_NODES], eout[FJ_MAX_NODES];
    double cover_tuples = 0, probes = 0, emax = 0;
};

// Textbook estimates along the plan: each node multiplies the incoming
// bindings by the smallest pure cover's expected size per binding and by the
// match probability of every other subatom.
Est estimate(const fj_query &q, const fj_sketch *sk, const fj_plan &p) {
    Est E{};
    double bound_v[FJ_MAX_VARS] = {0};  // distinct count of the atom that bound v
    double e = 1.0;
    for (size_t k = 0; k < p.nodes.size(); k++) {
        const auto &node = p.nodes[k];
        auto size_of = [&](size_t i) {
            const fj::Subatom &s = node[i];
            const int a = s.atom, l = p.sub_level[k][i];
            if (l == 0) return p.root_built[a] ? dist_set(q, sk, a, s.vars, s.nv) : rows_of(sk, a);
            int prev[FJ_MAX_COLS * fj::kMaxLev], np = 0;
            for (int ll = 0; ll < l; ll++)
                for (int j = 0; j < p.lev[a][ll].nv && np < FJ_MAX_COLS; j++) prev[np++] = p.lev[a][ll].vars[j];
            double f = rows_of(sk, a) / dist_set(q, sk, a, prev, np);
            if (l < p.nlev[a] - 1) f = std::min(f, dist_set(q, sk, a, s.vars, s.nv));
            return std::max(1.0, f);
        };
        const auto &pure = p.layout[k].pure;
        int cov_i = pure.empty() ? 0 : pure[0];
        double c = size_of(cov_i);
        for (int i : pure) {
            const double z = size_of(i);
            if (z < c) { c = z; cov_i = i; }
        }
        const int ca = node[cov_i].atom;
        double sel = 1.0;
        for (size_t i = 0; i < node.size(); i++) {
            if ((int)i == cov_i) continue;
            const fj::Subatom &s = node[i];
            for (int j = 0; j < s.nv; j++) {
                const int v = s.vars[j];
                const double db = dist_of(q, sk, s.atom, v);
                const double dc = col_of(q, ca, v) >= 0 ? dist_of(q, sk, ca, v) : std::max(1.0, bound_v[v]);
                sel *= std::min(1.0, db / dc);
            }
        }
        for (int j = 0; j < node[cov_i].nv; j++) {
            const int v = node[cov_i].vars[j];
            if (bound_v[v] == 0.0) bound_v[v] = dist_of(q, sk, ca, v);
        }
        E.ein[k] = e;
        E.cov[k] = c;
        E.cover_tuples += e * c;
        E.probes += e * c * (double)(node.size() - 1);
        e = e * c * sel;
        E.eout[k] = e;
        E.emax = std::max(E.emax, e);
    }
    return E;
}

void featurize(const fj_query &q, const fj_sketch *sk, const fj_plan &p, int kind, bool is_cyclic, float *f) {
    std::fill(f, f + FJ_FEATURES, 0.0f);
    const int nn = (int)p.nodes.size();
    double sum_rows = 0, max_rows = 0, min_rows = 1e300, built_rows = 0;
    int nbuilt = 0, arity2 = 0, max_ar = 0;
    double skew = 0;
    for (int a = 0; a < q.natoms; a++) {
        const double r = (double)sk[a].rows;
        sum_rows += r;
        max_rows = std::max(max_rows, r);
        min_rows = std::min(min_rows, r);
        if (p.root_built[a]) { built_rows += r; nbuilt++; }
        arity2 += q.atoms[a].arity == 2;
        max_ar = std::max(max_ar, (int)q.atoms[a].arity);
        skew += (double)sk[a].top[0][0] / rows_of(sk, a);
    }
    const Est E = estimate(q, sk, p);
    f[0] = kind == FJ_CAND_BINARY;
    f[1] = kind == FJ_CAND_GJ;
    f[2] = nn / 16.0f;
    f[3] = q.natoms / 16.0f;
    f[4] = q.nvars / 32.0f;
    f[5] = is_cyclic;
    f[6] = lg(sum_rows);
    f[7] = lg(max_rows);
    f[8] = lg(min_rows);
    f[9] = p.tail_from / 16.0f;
    f[10] = lg(E.cover_tuples);
    f[11] = lg(E.probes);
    f[12] = lg(E.eout[nn - 1]);
    f[13] = lg(E.emax);
    f[14] = lg(built_rows);
    f[15] = nbuilt / 16.0f;
    // atoms in plan order (first appearance of a subatom)
    int seen[FJ_MAX_ATOMS], nseen = 0;
    int first_node[FJ_MAX_ATOMS];
    char first_pure[FJ_MAX_ATOMS] = {0};
    std::fill(first_node, first_node + FJ_MAX_ATOMS, -1);
    for (int k = 0; k < nn; k++)
        for (size_t i = 0; i < p.nodes[k].size(); i++) {
            const int a = p.nodes[k][i].atom;
            if (first_node[a] >= 0) continue;
            first_node[a] = k;
            const auto &pure = p.layout[k].pure;
            first_pure[a] = !pure.empty() && pure[0] == (int)i;
            seen[nseen++] = a;
        }
    for (int sl = 0; sl < kSlots && sl < nseen; sl++) {
        const int a = seen[sl];
        float *g = f + kAtomBase + sl * kSlotF;
        const fj::Subatom &root = p.lev[a][0];
        const int c0 = col_of(q, a, root.vars[0]);
        int c1 = -1;
        for (int j = 0; j < q.atoms[a].arity && c1 < 0; j++) {
            bool in_root = false;
            for (int t = 0; t < root.nv; t++) in_root |= root.vars[t] == q.atoms[a].vars[j];
            if (!in_root) c1 = j;
        }
        const double r = rows_of(sk, a);
        const double vroot = dist_set(q, sk, a, root.vars, root.nv);
        g[0] = 1.0f;
        g[1] = lg((double)sk[a].rows);
        g[2] = lg(vroot);
        if (c0 >= 0) {
            double t8 = 0;
            for (int t = 0; t < FJ_SKETCH_TOPK; t++) t8 += (double)sk[a].top[c0][t];
            g[3] = (float)((double)sk[a].top[c0][0] / r);
            g[4] = (float)(t8 / r);
        }
        g[5] = p.root_built[a];
        g[6] = p.nlev[a] / 8.0f;
        g[7] = first_node[a] / 16.0f;
        g[8] = first_pure[a];
        g[9] = lg(r / vroot);
        if (c1 >= 0) {
            g[10] = lg((double)sk[a].distinct[c1]);
            g[11] = (float)((double)sk[a].top[c1][0] / r);
        }
    }
    for (int k = 0; k < kNodeSlots && k < nn; k++) {
        float *g = f + kNodeBase + k * kNodeF;
        g[0] = lg(E.ein[k]);
        g[1] = lg(E.cov[k]);
        g[2] = p.nodes[k].size() / 8.0f;
        g[3] = lg(E.eout[k]);
    }
    f[kTailBase + 0] = max_ar / 8.0f;
    f[kTailBase + 1] = (float)arity2 / (float)q.natoms;
    f[kTailBase + 2] = (float)(skew / q.natoms);
    f[kTailBase + 3] = lg(built_rows / std::max(1.0, sum_rows) * 1e6);
}

fj_status make_plan(const fj_query &q, const fj_candidate &c, fj_plan *p) {
    std::string err;
    fj_status st;
    if (c.kind == FJ_CAND_BINARY) {
        st = fj::plan_from_binary(q, c.order, c.n, true, p, err);
    } else if (c.kind == FJ_CAND_GJ) {
        if (c.n < 1 || c.n > FJ_MAX_NODES) return set_error(FJ_ERR_UNSUPPORTED, "too many variables for a GJ plan");
        std::vector<std::vector<fj::Subatom>> nodes;
        for (int i = 0; i < c.n; i++) {
            const int v = c.order[i];
            std::vector<fj::Subatom> node;
            for (int a = 0; a < q.natoms; a++) {
                if (col_of(q, a, v) < 0) continue;
                fj::Subatom s;
                s.atom = a;
                s.nv = 1;
                s.vars[0] = v;
                node.push_back(s);
            }
            nodes.push_back(node);
        }
        st = fj::plan_from_nodes(q, nodes, p, err);
    } else {
        return set_error(FJ_ERR_ARG, "unknown candidate kind");
    }
    if (st != FJ_OK) return set_error(st, err);
    return FJ_OK;
}

struct Candidates {
    std::vector<fj_candidate> c;
    std::vector<float> feat;
};

fj_status enumerate(const fj_query &q, const fj_sketch *sk, int cap, Candidates &out) {
    std::string err;
    FJ_TRY(fj::check_query(q, err) == FJ_OK ? FJ_OK : set_error(FJ_ERR_ARG, err));
    out.c.clear();
    out.feat.clear();
    const bool is_cyclic = cyclic(q);
    std::vector<std::vector<int>> orders;
    std::vector<int> ord;
    greedy(q, sk, -1, ord);
    orders.push_back(ord);
    for (int s = 0; s < q.natoms; s++) {
        greedy(q, sk, s, ord);
        if (std::find(orders.begin(), orders.end(), ord) == orders.end()) orders.push_back(ord);
    }
    std::vector<fj_candidate> cands;
    for (const auto &o : orders) {
        fj_candidate c{};
        c.kind = FJ_CAND_BINARY;
        c.n = (int)o.size();
        std::copy(o.begin(), o.end(), c.order);
        cands.push_back(c);
    }
    std::vector<std::vector<int>> vorders;
    for (const auto &o : orders) {
        std::vector<int> vo;
        for (int a : o)
            for (int j = 0; j < q.atoms[a].arity; j++) {
                const int v = q.atoms[a].vars[j];
                if (std::find(vo.begin(), vo.end(), v) == vo.end()) vo.push_back(v);
            }
        if ((int)vo.size() > FJ_MAX_NODES) continue;
        if (std::find(vorders.begin(), vorders.end(), vo) != vorders.end()) continue;
        vorders.push_back(vo);
        fj_candidate c{};
        c.kind = FJ_CAND_GJ;
        c.n = (int)vo.size();
        std::copy(vo.begin(), vo.end(), c.order);
        cands.push_back(c);
    }
    // one plan object serves every candidate (its vectors keep their
    // storage); the caller builds the chosen candidate's plan again
    fj_plan scratch;
    for (const auto &c : cands) {
        if ((int)out.c.size() >= cap) break;
        fj_status st = make_plan(q, c, &scratch);
        if (st != FJ_OK) {
            if (out.c.empty()) return st;  // the plain plan must exist
            continue;
        }
        out.c.push_back(c);
        out.feat.resize(out.c.size() * FJ_FEATURES);
        featurize(q, sk, scratch, c.kind, is_cyclic, out.feat.data() + (out.c.size() - 1) * FJ_FEATURES);
    }
    return FJ_OK;
}

}  // namespace

// --------------------------------------------------------------- perceptron

struct fj_mlp {
    fj_ctx *ctx = nullptr;
    hipStream_t s = nullptr;
    int dev = 0;
    int D = 0, H = 0;
    int64_t np = 0, oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // np floats each
    float *act = nullptr;  // h1 | h2 | dz1 | dz2 (cap x H each) | y | dy | sq (cap each) | loss
    int cap = 0;
    float *loss_h = nullptr;  // pinned
    int64_t step = 0;
    // chooser staging (pinned, mapped, coherent)
    float *feat_h = nullptr, *score_h = nullptr;
    float *h1() const { return act; }
    float *h2() const { return act + (size_t)cap * H; }
    float *dz1() const { return act + 2 * (size_t)cap * H; }
    float *dz2() const { return act + 3 * (size_t)cap * H; }
    float *y() const { return act + 4 * (size_t)cap * H; }
    float *dy() const { return y() + cap; }
    float *sq() const { return dy() + cap; }
    float *loss_d() const { return sq() + cap; }
};

namespace {

fj_status mlp_ensure(fj_mlp *m, int B) {
    if (B <= m->cap) return FJ_OK;
    int cap = std::max(B, 256);
    if (m->act) {
        FJ_HIP(hipStreamSynchronize(m->s));
        hipFree(m->act);
        m->act = nullptr;
        m->cap = 0;
    }
    const size_t n = 4 * (size_t)cap * m->H + 3 * (size_t)cap + 64;
    FJ_HIP(hipMalloc((void **)&m->act, n * sizeof(float)));
    m->cap = cap;
    return FJ_OK;
}

fj_status mlp_check(fj_mlp *m, const float *x, int B) {
    if (!m || !x) return set_error(FJ_ERR_ARG, "null argument");
    if (B < 1) return set_error(FJ_ERR_ARG, "batch must be positive");
    FJ_HIP(hipSetDevice(m->dev));
    return mlp_ensure(m, B);
}

fj_status mlp_fwd(fj_mlp *m, const float *x, int B, float *y) {
    const int D = m->D, H = m->H;
    FJ_HIP(fj::mlp_gemm(x, m->w + m->oW1, m->w + m->ob1, m->h1(), B, H, D, false, false, true, false, m->s));
    FJ_HIP(fj::mlp_gemm(m->h1(), m->w + m->oW2, m->w + m->ob2, m->h2(), B, H, H, false, false, true, false, m->s));
    FJ_HIP(fj::mlp_gemm(m->h2(), m->w + m->oW3, m->w + m->ob3, y, B, 1, H, false, false, false, false, m->s));
    return FJ_OK;
}

// forward, loss and the full gradient into m->g; the loss sum into loss_d
fj_status mlp_bwd(fj_mlp *m, const float *x, const float *t, int B) {
    const int D = m->D, H = m->H;
    FJ_TRY(mlp_fwd(m, x, B, m->y()));
    FJ_HIP(fj::mlp_mse_grad(m->y(), t, m->dy(), m->sq(), B, m->s));
    float *g = m->g;
    // output layer
    FJ_HIP(fj::mlp_gemm(m->h2(), m->dy(), nullptr, g + m->oW3, H, 1, B, true, false, false, false, m->s));
    FJ_HIP(fj::mlp_colsum(m->dy(), g + m->ob3, B, 1, m->s));
    FJ_HIP(fj::mlp_gemm(m->dy(), m->w + m->oW3, nullptr, m->dz2(), B, H, 1, false, true, false, false, m->s));
    FJ_HIP(fj::mlp_relu_back(m->h2(), m->dz2(), B * H, m->s));
    // second layer
    FJ_HIP(fj::mlp_gemm(m->h1(), m->dz2(), nullptr, g + m->oW2, H, H, B, true, false, false, false, m->s));
    FJ_HIP(fj::mlp_colsum(m->dz2(), g + m->ob2, B, H, m->s));
    FJ_HIP(fj::mlp_gemm(m->dz2(), m->w + m->oW2, nullptr, m->dz1(), B, H, H, false, true, false, false, m->s));
    FJ_HIP(fj::mlp_relu_back(m->h1(), m->dz1(), B * H, m->s));
    // first layer
    FJ_HIP(fj::mlp_gemm(x, m->dz1(), nullptr, g + m->oW1, D, H, B, true, false, false, false, m->s));
    FJ_HIP(fj::mlp_colsum(m->dz1(), g + m->ob1, B, H, m->s));
    FJ_HIP(fj::mlp_sum(m->sq(), B, m->loss_d(), m->s));
    return FJ_OK;
}

}  // namespace

extern "C" {

fj_status fj_mlp_create(fj_ctx *ctx, int32_t in_dim, int32_t hidden, fj_mlp **out) {
    if (!ctx || !out) return set_error(FJ_ERR_ARG, "null argument");
    *out = nullptr;
    if (in_dim < 1 || in_dim > 1024 || hidden < 1 || hidden > 1024)
        return set_error(FJ_ERR_ARG, "in_dim and hidden must be 1..1024");
    fj_mlp *m = new fj_mlp();
    m->ctx = ctx;
    m->s = fj::ctx_stream(ctx);
    m->dev = fj::ctx_device(ctx);
    m->D = in_dim;
    m->H = hidden;
    const int64_t D = in_dim, H = hidden;
    m->oW1 = 0;
    m->ob1 = D * H;
    m->oW2 = m->ob1 + H;
    m->ob2 = m->oW2 + H * H;
    m->oW3 = m->ob2 + H;
    m->ob3 = m->oW3 + H;
    m->np = m->ob3 + 1;
    auto cleanup = [&](fj_status st, const char *msg) {
        fj_mlp_free(m);
        return set_error(st, msg);
    };
    if (hipSetDevice(m->dev) != hipSuccess) return cleanup(FJ_ERR_HIP, "hipSetDevice");
    float **bufs[4] = {&m->w, &m->g, &m->m, &m->v};
    for (auto b : bufs)
        if (hipMalloc((void **)b, m->np * sizeof(float)) != hipSuccess) return cleanup(FJ_ERR_OOM, "parameters");
    // the chooser's staging is read and written by the GPU directly
    const unsigned coh = hipHostMallocMapped | hipHostMallocCoherent;
    if (hipHostMalloc((void **)&m->feat_h, FJ_CAND_MAX * FJ_FEATURES * sizeof(float), coh) != hipSuccess ||
        hipHostMalloc((void **)&m->score_h, FJ_CAND_MAX * sizeof(float), coh) != hipSuccess ||
        hipHostMalloc((void **)&m->loss_h, sizeof(float), hipHostMallocDefault) != hipSuccess)
        return cleanup(FJ_ERR_OOM, "pinned buffers");
    std::vector<float> zero(m->np, 0.0f);
    fj_status st = fj_mlp_set_params(m, zero.data(), m->np);
    if (st != FJ_OK) { fj_mlp_free(m); return st; }
    *out = m;
    return FJ_OK;
}

int64_t fj_mlp_param_count(const fj_mlp *m) { return m ? m->np : 0; }

fj_status fj_mlp_set_params(fj_mlp *m, const float *params, int64_t n) {
    if (!m || !params) return set_error(FJ_ERR_ARG, "null argument");
    if (n != m->np) return set_error(FJ_ERR_ARG, "parameter count mismatch");
    FJ_HIP(hipSetDevice(m->dev));
    FJ_HIP(hipMemcpyAsync(m->w, params, n * sizeof(float), hipMemcpyHostToDevice, m->s));
    FJ_HIP(hipMemsetAsync(m->m, 0, n * sizeof(float), m->s));
    FJ_HIP(hipMemsetAsync(m->v, 0, n * sizeof(float), m->s));
    FJ_HIP(hipStreamSynchronize(m->s));
    m->step = 0;
    return FJ_OK;
}

fj_status fj_mlp_get_params(fj_mlp *m, float *params, int64_t n) {
    if (!m || !params) return set_error(FJ_ERR_ARG, "null argument");
    if (n != m->np) return set_error(FJ_ERR_ARG, "parameter count mismatch");
    FJ_HIP(hipSetDevice(m->dev));
    FJ_HIP(hipMemcpyAsync(params, m->w, n * sizeof(float), hipMemcpyDeviceToHost, m->s));
    FJ_HIP(hipStreamSynchronize(m->s));
    return FJ_OK;
}

fj_status fj_mlp_forward(fj_mlp *m, const float *x, int32_t batch, float *y) {
    if (!y) return set_error(FJ_ERR_ARG, "null output");
    FJ_TRY(mlp_check(m, x, batch));
    return mlp_fwd(m, x, batch, y);
}

fj_status fj_mlp_gradient(fj_mlp *m, const float *x, const float *t, int32_t batch, float *grad, float *loss) {
    if (!t || !grad || !loss) return set_error(FJ_ERR_ARG, "null argument");
    FJ_TRY(mlp_check(m, x, batch));
    FJ_TRY(mlp_bwd(m, x, t, batch));
    FJ_HIP(hipMemcpyAsync(grad, m->g, m->np * sizeof(float), hipMemcpyDeviceToHost, m->s));
    FJ_HIP(hipMemcpyAsync(m->loss_h, m->loss_d(), sizeof(float), hipMemcpyDeviceToHost, m->s));
    FJ_HIP(hipStreamSynchronize(m->s));
    *loss = *m->loss_h / (float)batch;
    return FJ_OK;
}

fj_status fj_mlp_train_step(fj_mlp *m, const float *x, const float *t, int32_t batch, float lr, float *loss) {
    if (!t) return set_error(FJ_ERR_ARG, "null targets");
    if (!(lr > 0.0f)) return set_error(FJ_ERR_ARG, "learning rate must be positive");
    FJ_TRY(mlp_check(m, x, batch));
    FJ_TRY(mlp_bwd(m, x, t, batch));
    if (loss) FJ_HIP(hipMemcpyAsync(m->loss_h, m->loss_d(), sizeof(float), hipMemcpyDeviceToHost, m->s));
    m->step++;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(b1, (double)m->step));
    const float c2 = (float)(1.0 - std::pow(b2, (double)m->step));
    FJ_HIP(fj::mlp_adam(m->w, m->g, m->m, m->v, (int)m->np, lr, (float)b1, (float)b2, 1e-8f, c1, c2, m->s));
    if (loss) {
        FJ_HIP(hipStreamSynchronize(m->s));
        *loss = *m->loss_h / (float)batch;
    }
    return FJ_OK;
}

void fj_mlp_free(fj_mlp *m) {
    if (!m) return;
    hipSetDevice(m->dev);
    hipStreamSynchronize(m->s);
    for (float *p : {m->w, m->g, m->m, m->v, m->act})
        if (p) hipFree(p);
    for (float *p : {m->feat_h, m->score_h, m->loss_h})
        if (p) hipHostFree(p);
    delete m;
}

// ------------------------------------------------------------ plan choice

fj_status fj_greedy_order(const fj_query *q, const fj_sketch *sk, int32_t first, int32_t *order) {
    FJ_TRY(check_sketches(q, sk));
    if (!order) return set_error(FJ_ERR_ARG, "null order");
    if (first >= q->natoms) return set_error(FJ_ERR_ARG, "first out of range");
    std::vector<int> o;
    greedy(*q, sk, first, o);
    std::copy(o.begin(), o.end(), order);
    return FJ_OK;
}

fj_status fj_plan_candidates(const fj_query *q, const fj_sketch *sk, int32_t cap, fj_candidate *out, int32_t *n,
                             float *features) {
    FJ_TRY(check_sketches(q, sk));
    if (!out || !n || !features) return set_error(FJ_ERR_ARG, "null argument");
    if (cap < 1 || cap > FJ_CAND_MAX) return set_error(FJ_ERR_ARG, "cap must be 1..FJ_CAND_MAX");
    Candidates C;
    FJ_TRY(enumerate(*q, sk, cap, C));
    *n = (int32_t)C.c.size();
    std::copy(C.c.begin(), C.c.end(), out);
    std::copy(C.feat.begin(), C.feat.end(), features);
    return FJ_OK;
}

fj_status fj_candidate_plan(const fj_query *q, const fj_candidate *c, fj_plan **out) {
    if (!q || !c || !out) return set_error(FJ_ERR_ARG, "null argument");
    *out = nullptr;
    fj_plan *p = new fj_plan();
    fj_status st = make_plan(*q, *c, p);
    if (st != FJ_OK) { delete p; return st; }
    *out = p;
    return FJ_OK;
}

fj_status fj_choose_plan(fj_ctx *ctx, fj_mlp *m, const fj_query *q, const fj_sketch *sk, float margin,
                         uint64_t gate_rows, fj_plan **out, int32_t *chosen, float *scores) {
    if (!ctx || !out) return set_error(FJ_ERR_ARG, "null argument");
    FJ_TRY(check_sketches(q, sk));
    *out = nullptr;
    if (m && m->D != FJ_FEATURES) return set_error(FJ_ERR_ARG, "the perceptron's input is not FJ_FEATURES wide");
    uint64_t rows = 0;
    for (int a = 0; a < q->natoms; a++) rows += (uint64_t)std::max<int64_t>(sk[a].rows, 0);
    if (rows < gate_rows) {
        // the plain plan alone: the greedy order, converted and factored
        std::string err;
        FJ_TRY(fj::check_query(*q, err) == FJ_OK ? FJ_OK : set_error(FJ_ERR_ARG, err));
        std::vector<int> ord;
        greedy(*q, sk, -1, ord);
        fj_plan *p = new fj_plan();
        fj_status st = fj::plan_from_binary(*q, ord.data(), (int)ord.size(), true, p, err);
        if (st != FJ_OK) {
            delete p;
            return set_error(st, err);
        }
        if (chosen) *chosen = 0;
        *out = p;
        return FJ_OK;
    }
    Candidates C;
    FJ_TRY(enumerate(*q, sk, FJ_CAND_MAX, C));
    const int nc = (int)C.c.size();
    int pick = 0;
    if (m && q->natoms <= kSlots && nc > 1) {
        // one launch reads the features from and writes the scores to
        // pinned host memory; the scores start as NaN and the host spins
        // until every one is written, which skips the runtime's completion
        // wait (a spin that runs out falls back to a stream synchronize,
        // which also reports a failed kernel)
        FJ_HIP(hipSetDevice(m->dev));
        std::copy(C.feat.begin(), C.feat.end(), m->feat_h);
        volatile float *sc = m->score_h;
        for (int i = 0; i < nc; i++) sc[i] = std::numeric_limits<float>::quiet_NaN();
        const int64_t off[6] = {m->oW1, m->ob1, m->oW2, m->ob2, m->oW3, m->ob3};
        FJ_HIP(fj::mlp_rows(m->feat_h, nc, m->D, m->H, m->w, off, m->score_h, m->s));
        auto written = [&]() {
            for (int i = 0; i < nc; i++)
                if (std::isnan(sc[i])) return false;
            return true;
        };
        const auto t0 = std::chrono::steady_clock::now();
        while (!written() && std::chrono::steady_clock::now() - t0 < std::chrono::milliseconds(2)) {
        }
        if (!written()) FJ_HIP(hipStreamSynchronize(m->s));
        int best = 0;
        for (int i = 1; i < nc; i++)
            if (sc[i] < sc[best]) best = i;
        if (sc[0] - sc[best] >= margin) pick = best;
        if (scores)
            for (int i = 0; i < nc; i++) scores[i] = sc[i];
    }
    if (chosen) *chosen = pick;
    fj_plan *p = new fj_plan();
    fj_status st = make_plan(*q, C.c[pick], p);
    if (st != FJ_OK) {
        delete p;
        return st;
    }
    *out = p;
    return FJ_OK;
}

}  // extern "C"
