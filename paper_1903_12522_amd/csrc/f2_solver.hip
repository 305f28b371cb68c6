// Second-order (nodal, 3D) solver: not built yet.
#include "solver.h"

namespace cmcg {

cmcg_status make_f2_solver(const cmcg_problem *, const SolverConfig &, Solver **out) {
  *out = nullptr;
  set_error("second-order formulation not built yet");
  return CMCG_EUNSUPPORTED;
}

}  // namespace cmcg
