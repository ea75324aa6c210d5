// Host-side search plans (pattern analyzer).
#pragma once

#include <array>
#include <string>
#include <utility>
#include <vector>

#include "../../include/gpm.h"
#include "gpm_internal.h"

namespace gpm {

struct HostPlan {
  int k = 0;
  int mode = GPM_VERTEX_INDUCED;
  bool clique = false;
  int aut = 1;                                  // |Aut(P)|
  int order[kMaxK] = {};                        // pattern vertex matched at each depth
  std::vector<std::pair<int, int>> restrictions;  // (a, b): v_a > v_b (pattern ids)
  int n_buffers = 0;                            // stored frontier levels (X)
  int choose_r = 0;                             // counting-only leaf: vertices it stands for
  Plan plan{};                                  // device plan, depth-indexed
};

int validate_pattern(const gpm_pattern& p, std::string* err);
bool is_clique(const gpm_pattern& p);

// Build the plan for `p` in `mode`.  on_dag: cliques on an oriented DAG.
// count_only: the plan may end in a counting-only leaf (edge-induced mode:
// the last r >= 2 pattern vertices pairwise non-adjacent twins, chosen as
// r-subsets of one candidate set; Plan::leaf_choose), never for listing.
int build_plan(const gpm_pattern& p, int mode, bool on_dag, HostPlan* out, std::string* err,
               bool count_only = false);

}  // namespace gpm
