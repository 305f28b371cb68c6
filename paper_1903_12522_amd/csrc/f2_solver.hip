// Second-order (nodal, 3D) solver: placeholder until the nodal kernels land.
#include "f2_runtime.h"

namespace cmcg {

struct F2Solver {};

cmcg_status f2_create(F2Solver **out, const F2Params &, const cmcg_problem *, hipStream_t) {
  *out = nullptr;
  set_error("second-order formulation not built yet");
  return CMCG_EUNSUPPORTED;
}
void f2_destroy(F2Solver *S) { delete S; }
size_t f2_device_bytes(const F2Solver *) { return 0; }
cmcg_status f2_begin(F2Solver *) { return CMCG_EUNSUPPORTED; }
cmcg_status f2_iterate(F2Solver *, int, int *) { return CMCG_EUNSUPPORTED; }
cmcg_status f2_finish(F2Solver *, double *, double *) { return CMCG_EUNSUPPORTED; }
cmcg_status f2_solve(F2Solver *, double *, double *) { return CMCG_EUNSUPPORTED; }
cmcg_status f2_apply(F2Solver *, int, const double *, double *) { return CMCG_EUNSUPPORTED; }
cmcg_status f2_filter(F2Solver *, const double *, double *, double *) { return CMCG_EUNSUPPORTED; }
cmcg_status f2_get_state(F2Solver *, int, double *) { return CMCG_EUNSUPPORTED; }
void f2_report(const F2Solver *, cmcg_report *) {}

}  // namespace cmcg
