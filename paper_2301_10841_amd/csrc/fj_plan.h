// Host-side Free Join plan model (Section 3.2) and its derived per-node
// execution layout.  Internal to libfj.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fj.h"

namespace fj {

constexpr int kMaxLev = FJ_MAX_NODES;  // a schema has at most one level per node

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
    std::vector<int> in_var;      // variable ids stored in the input frontier
    std::vector<int> in_hatom;    // atoms whose inner handle the frontier carries
    std::vector<int> new_vars;    // variables bound by this node's cover
    std::vector<int> pure;        // subatom indices (within node) of pure covers
};

}  // namespace fj

struct fj_plan {
    fj_query q{};
    std::vector<std::vector<fj::Subatom>> nodes;
    // schema per atom: level l of atom a is subatom lev[a][l]
    int nlev[FJ_MAX_ATOMS] = {0};
    fj::Subatom lev[FJ_MAX_ATOMS][fj::kMaxLev];
    std::vector<std::vector<int>> sub_level;  // [node][subatom] -> level in its atom
    std::vector<fj::NodeLayout> layout;       // nnodes + 1 entries (last = final)
    bool root_built[FJ_MAX_ATOMS] = {false};
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
