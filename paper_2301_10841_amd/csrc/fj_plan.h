// Host-side Free Join plan model (Section 3.2) and its derived per-node
// execution layout.  Internal to libfj.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fj.h"

namespace fj {

constexpr int kMaxLev = FJ_MAX_NODES;  // a schema has at most one level per node

// A vector of at most N elements stored inline (plans are built per
// candidate while choosing, so they avoid heap allocations).
template <typename T, int N>
struct SmallVec {
    T v[N];
    int n = 0;
    void push_back(const T &x) { v[n++] = x; }
    int size() const { return n; }
    bool empty() const { return n == 0; }
    void clear() { n = 0; }
    const T &operator[](int i) const { return v[i]; }
    T &operator[](int i) { return v[i]; }
    const T *data() const { return v; }
    const T *begin() const { return v; }
    const T *end() const { return v + n; }
};

struct Subatom {
    int atom = -1;
    int nv = 0;
    int vars[FJ_MAX_COLS] = {0};
};

// Per-node layout used by the executor.  A node's input frontier holds the
// values of the variables bound by earlier nodes (in_var) and, for every atom
// that is part-way through its schema, the start position of its current
// sub-trie at that level (in_hatom).
struct NodeLayout {
    SmallVec<int, FJ_MAX_VARS> in_var;     // variable ids stored in the input frontier
    SmallVec<int, FJ_MAX_ATOMS> in_hatom;  // atoms whose inner handle the frontier carries
    SmallVec<int, FJ_MAX_VARS> new_vars;   // variables bound by this node's cover
    SmallVec<int, FJ_MAX_ATOMS> pure;      // subatom indices (within node) of pure covers
};

}  // namespace fj

struct fj_plan {
    fj_query q{};
    std::vector<std::vector<fj::Subatom>> nodes;
    // schema per atom: level l of atom a is subatom lev[a][l]
    int nlev[FJ_MAX_ATOMS] = {0};
    fj::Subatom lev[FJ_MAX_ATOMS][fj::kMaxLev];
    int sub_level[FJ_MAX_NODES][FJ_MAX_ATOMS] = {};  // [node][subatom] -> level in its atom
    fj::NodeLayout layout[FJ_MAX_NODES + 1];          // nnodes + 1 used (last = final)
    bool root_built[FJ_MAX_ATOMS] = {false};
    // an unbuilt root that another cover of its node may win: forced by the
    // first probe that reaches it, so its map is allocated but not filled
    bool root_lazy[FJ_MAX_ATOMS] = {false};
    int tail_from = 0;                        // nodes >= tail_from are single-cover products
};

namespace fj {

// Returns FJ_OK or an error status and sets `err`.
fj_status plan_from_binary(const fj_query &q, const int32_t *order, int n, bool do_factor,
                           fj_plan *out, std::string &err);
fj_status plan_from_nodes(const fj_query &q, const std::vector<std::vector<Subatom>> &nodes,
                          fj_plan *out, std::string &err);
fj_status check_query(const fj_query &q, std::string &err);

}  // namespace fj
