// Free Join plan pipeline on the host: binary-plan conversion and
// conservative factoring (Section 4.1), validity and covers (Section 3.2),
// COLT schemas (Section 3.3 build phase) and the executor's per-node layout.
#include "fj_plan.h"

#include <algorithm>
#include <cstring>

namespace fj {

namespace {

using VarSet = uint64_t;  // FJ_MAX_VARS <= 64

VarSet vset(const Subatom &s) {
    VarSet m = 0;
    for (int j = 0; j < s.nv; j++) m |= VarSet(1) << s.vars[j];
    return m;
}

VarSet node_vset(const std::vector<Subatom> &node) {
    VarSet m = 0;
    for (const auto &s : node) m |= vset(s);
    return m;
}

Subatom make_sub(const fj_query &q, int atom, VarSet keep) {
    // the atom's variables that are in `keep`, in column order
    Subatom s;
    s.atom = atom;
    const fj_atom &a = q.atoms[atom];
    for (int j = 0; j < a.arity; j++)
        if (keep & (VarSet(1) << a.vars[j])) s.vars[s.nv++] = a.vars[j];
    return s;
}

VarSet atom_vset(const fj_query &q, int a) {
    VarSet m = 0;
    for (int j = 0; j < q.atoms[a].arity; j++) m |= VarSet(1) << q.atoms[a].vars[j];
    return m;
}

}  // namespace

fj_status check_query(const fj_query &q, std::string &err) {
    if (q.natoms < 1 || q.natoms > FJ_MAX_ATOMS) { err = "natoms out of range"; return FJ_ERR_ARG; }
    if (q.nvars < 1 || q.nvars > FJ_MAX_VARS) { err = "nvars out of range"; return FJ_ERR_ARG; }
    VarSet all = 0;
    for (int a = 0; a < q.natoms; a++) {
        const fj_atom &at = q.atoms[a];
        if (at.arity < 0 || at.arity > FJ_MAX_COLS) { err = "atom arity out of range"; return FJ_ERR_ARG; }
        VarSet m = 0;
        for (int j = 0; j < at.arity; j++) {
            int v = at.vars[j];
            if (v < 0 || v >= q.nvars) { err = "atom variable out of range"; return FJ_ERR_ARG; }
            if (m & (VarSet(1) << v)) { err = "variables of one atom must be distinct"; return FJ_ERR_ARG; }
            m |= VarSet(1) << v;
        }
        all |= m;
    }
    if (all != ((q.nvars == 64) ? ~VarSet(0) : ((VarSet(1) << q.nvars) - 1))) {
        err = "every variable must occur in some atom";
        return FJ_ERR_ARG;
    }
    if (q.nhead != q.nvars) { err = "the query is full: the head lists every variable once"; return FJ_ERR_ARG; }
    VarSet h = 0;
    for (int j = 0; j < q.nhead; j++) {
        int v = q.head[j];
        if (v < 0 || v >= q.nvars || (h & (VarSet(1) << v))) { err = "bad head"; return FJ_ERR_ARG; }
        h |= VarSet(1) << v;
    }
    return FJ_OK;
}

// Section 4.1: a left-deep binary plan R_1 ... R_m becomes one node per
// relation.  Node i iterates the variables R_i adds to those of R_1..R_{i-1}
// and, unless it is the last node, looks R_{i+1} up on the variables it
// shares with R_1..R_i (reading A2: the current relation's variables count
// as available).
static std::vector<std::vector<Subatom>> binary_to_fj(const fj_query &q, const int32_t *order, int n) {
    std::vector<VarSet> bound(n + 1, 0);   // bound[i]: variables of the first i relations
    for (int i = 0; i < n; i++) bound[i + 1] = bound[i] | atom_vset(q, order[i]);
    std::vector<std::vector<Subatom>> plan(n);
    for (int i = 0; i < n; i++) {
        plan[i].push_back(make_sub(q, order[i], atom_vset(q, order[i]) & ~bound[i]));
        if (i + 1 < n) plan[i].push_back(make_sub(q, order[i + 1], atom_vset(q, order[i + 1]) & bound[i + 1]));
    }
    return plan;
}

// Section 4.1, figure "factorize-plan": walk nodes from the last to the
// second; move the node's lookups (subatoms after the first, in order) to the
// previous node while their variables are bound before this node and the
// previous node holds no subatom of the same atom; stop at the first that
// cannot move, so the optimizer's lookup order is kept.
static void factor_plan(std::vector<std::vector<Subatom>> &plan) {
    int n = (int)plan.size();
    for (int i = n - 1; i >= 1; i--) {
        VarSet before = 0;
        for (int j = 0; j < i; j++) before |= node_vset(plan[j]);
        auto &phi = plan[i];
        auto &prev = plan[i - 1];
        while (phi.size() > 1) {
            const Subatom cand = phi[1];
            bool avail = (vset(cand) & ~before) == 0;
            bool clash = false;
            for (const auto &p : prev) clash |= (p.atom == cand.atom);
            if (!avail || clash) break;
            prev.push_back(cand);
            phi.erase(phi.begin() + 1);
        }
    }
}

static fj_status finish_plan(const fj_query &q, const std::vector<std::vector<Subatom>> &nodes,
                             fj_plan *out, std::string &err) {
    int nn = (int)nodes.size();
    if (nn < 1 || nn > FJ_MAX_NODES) { err = "plan must have 1..FJ_MAX_NODES nodes"; return FJ_ERR_UNSUPPORTED; }
    out->q = q;
    out->nodes = nodes;
    for (int a = 0; a < FJ_MAX_ATOMS; a++) {
        out->nlev[a] = 0;
        out->root_built[a] = false;
    }
    out->tail_from = 0;
    // partition check and schemas
    VarSet seen[FJ_MAX_ATOMS] = {0};
    for (int k = 0; k < nn; k++) {
        if (nodes[k].empty()) { err = "empty plan node"; return FJ_ERR_PLAN_INVALID; }
        if ((int)nodes[k].size() > FJ_MAX_ATOMS) { err = "validity (a): an atom occurs twice in a node"; return FJ_ERR_PLAN_INVALID; }
        uint32_t atoms_here = 0;
        int si = 0;
        for (const auto &s : nodes[k]) {
            if (s.atom < 0 || s.atom >= q.natoms) { err = "subatom names an unknown atom"; return FJ_ERR_PLAN_INVALID; }
            if (atoms_here & (1u << s.atom)) { err = "validity (a): an atom occurs twice in a node"; return FJ_ERR_PLAN_INVALID; }
            atoms_here |= 1u << s.atom;
            VarSet sv = vset(s);
            if (s.nv < 0 || s.nv > FJ_MAX_COLS || (sv & ~atom_vset(q, s.atom))) {
                err = "subatom variables are not the atom's"; return FJ_ERR_PLAN_INVALID;
            }
            if (__builtin_popcountll(sv) != s.nv) { err = "repeated variable in a subatom"; return FJ_ERR_PLAN_INVALID; }
            if (seen[s.atom] & sv) { err = "the nodes do not partition an atom"; return FJ_ERR_PLAN_INVALID; }
            seen[s.atom] |= sv;
            int l = out->nlev[s.atom]++;
            if (l >= kMaxLev) { err = "an atom has more levels than nodes"; return FJ_ERR_PLAN_INVALID; }
            out->lev[s.atom][l] = s;
            out->sub_level[k][si++] = l;
        }
    }
    for (int a = 0; a < q.natoms; a++) {
        if (seen[a] != atom_vset(q, a) || out->nlev[a] == 0) { err = "the nodes do not partition an atom"; return FJ_ERR_PLAN_INVALID; }
    }
    // covers (validity (b)) and pure covers; per-node frontier layout
    for (int k = 0; k <= nn; k++) {
        out->layout[k].in_var.clear();
        out->layout[k].in_hatom.clear();
        out->layout[k].new_vars.clear();
        out->layout[k].pure.clear();
    }
    VarSet bound = 0;
    int lev_at[FJ_MAX_ATOMS] = {0};  // current level of each atom before node k
    for (int k = 0; k <= nn; k++) {
        fj::NodeLayout &L = out->layout[k];
        for (int v = 0; v < q.nvars; v++)
            if (bound & (VarSet(1) << v)) L.in_var.push_back(v);
        for (int a = 0; a < q.natoms; a++)
            if (lev_at[a] > 0 && lev_at[a] < out->nlev[a]) L.in_hatom.push_back(a);
        if (k == nn) break;
        VarSet nv = node_vset(nodes[k]) & ~bound;
        bool any_cover = false;
        for (int i = 0; i < (int)nodes[k].size(); i++) {
            VarSet sv = vset(nodes[k][i]);
            if ((nv & ~sv) == 0) {
                any_cover = true;
                if ((sv & bound) == 0) L.pure.push_back(i);
            }
        }
        if (!any_cover) { err = "validity (b): a node has no cover"; return FJ_ERR_PLAN_INVALID; }
        if (L.pure.empty()) { err = "no cover of a node is free of bound variables"; return FJ_ERR_PLAN_NO_PURE_COVER; }
        for (int v = 0; v < q.nvars; v++)
            if (nv & (VarSet(1) << v)) L.new_vars.push_back(v);
        for (const auto &s : nodes[k]) lev_at[s.atom]++;
        bound |= nv;
    }
    // build-phase rule for roots (Section 4.2: no auxiliary structure on a
    // table nobody probes): a single-level atom whose subatom is a pure
    // cover of its node keeps its base table.  When it is the node's only
    // pure cover it is always iterated directly; when other covers compete
    // for some bindings it is forced by the first probe that reaches it.
    for (int a = 0; a < q.natoms; a++) {
        out->root_built[a] = true;
        out->root_lazy[a] = false;
        for (int k = 0; k < nn; k++) {
            for (int i = 0; i < (int)nodes[k].size(); i++) {
                if (nodes[k][i].atom != a || out->sub_level[k][i] != 0 || out->nlev[a] != 1) continue;
                const auto &pc = out->layout[k].pure;
                for (int j = 0; j < (int)pc.size(); j++) {
                    if (pc[j] != i) continue;
                    out->root_built[a] = false;
                    out->root_lazy[a] = pc.size() > 1;
                }
            }
        }
    }
    // trailing nodes whose only subatom is the last level of its atom need
    // no probing: each input binding contributes the product of their sizes.
    int t = nn;
    while (t > 0) {
        const auto &node = nodes[t - 1];
        if (node.size() != 1) break;
        int a = node[0].atom;
        if (out->sub_level[t - 1][0] != out->nlev[a] - 1) break;
        t--;
    }
    out->tail_from = t;
    return FJ_OK;
}

fj_status plan_from_binary(const fj_query &q, const int32_t *order, int n, bool do_factor,
                           fj_plan *out, std::string &err) {
    fj_status st = check_query(q, err);
    if (st != FJ_OK) return st;
    if (!order || n != q.natoms) { err = "the left-deep order must list every atom once"; return FJ_ERR_ARG; }
    uint32_t used = 0;
    for (int i = 0; i < n; i++) {
        if (order[i] < 0 || order[i] >= q.natoms || (used & (1u << order[i]))) {
            err = "the left-deep order must list every atom once"; return FJ_ERR_ARG;
        }
        used |= 1u << order[i];
    }
    auto plan = binary_to_fj(q, order, n);
    if (do_factor) factor_plan(plan);
    return finish_plan(q, plan, out, err);
}

fj_status plan_from_nodes(const fj_query &q, const std::vector<std::vector<Subatom>> &nodes,
                          fj_plan *out, std::string &err) {
    fj_status st = check_query(q, err);
    if (st != FJ_OK) return st;
    return finish_plan(q, nodes, out, err);
}

}  // namespace fj
