// Weighted join and its adjoint -- not implemented yet.
#include "plan.h"

using namespace gjh;

struct gj_wstate {
  int dummy;
};

extern "C" {

gj_status gj_weighted_forward(gj_ctx*, const gj_factors*, const void* const*, int32_t, double*, gj_wstate**) {
  set_error("gj_weighted_forward: not implemented");
  return GJ_E_INVALID;
}
gj_status gj_weighted_backward(gj_ctx*, const gj_wstate*, const double*, void* const*) {
  set_error("gj_weighted_backward: not implemented");
  return GJ_E_INVALID;
}
void gj_free_wstate(gj_wstate* st) { delete st; }

gj_status gj_unroll_gfjs(gj_ctx*, const gj_summary*, int64_t, int64_t, int32_t* const*, int64_t* const*, int64_t*) {
  set_error("gj_unroll_gfjs: not implemented");
  return GJ_E_INVALID;
}

}  // extern "C"
