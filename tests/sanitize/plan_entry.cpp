// Host-only entry point for the sanitizer build of the hierarchy analysis (tests only):
// the same two analysis parts the library runs inside rsd_analyze and rsd_setup, compiled
// with g++ -fsanitize=address,undefined and driven by the host tests' invalid inputs.
#include <cstdio>
#include <string>

#include "plan.hpp"

extern "C" int plan_check(int32_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                          int32_t num_nodes, const int32_t* parent, const int32_t* dof_node,
                          char* msg, int msg_len) {
  rsd::Plan plan;
  std::string m;
  rsd::PlanError e =
      rsd::build_plan(n, nnz, row_ptr, col_idx, num_nodes, parent, dof_node, &plan, &m);
  if (e == rsd::PlanError::kOk) e = rsd::build_plan_couplings(row_ptr, col_idx, &plan, &m);
  std::snprintf(msg, size_t(msg_len), "%s", m.c_str());
  return int(e);
}
