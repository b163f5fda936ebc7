// Batched many-q plan (placeholder entry points).
#include "common.h"

extern "C" {
gw_status gw_plan_create(gw_ctx* c, gw_plan** plan, const int*, int, gw_dtype, gw_prec, int,
                         const double*, double, int, const gw_q_desc*) {
  if (plan) *plan = nullptr;
  return gw::fail(c, GW_EUNSUPPORTED, "batched plan not built yet");
}
gw_status gw_plan_compile(gw_plan*) { return GW_EUNSUPPORTED; }
gw_status gw_plan_launch(gw_plan*) { return GW_EUNSUPPORTED; }
gw_status gw_plan_destroy(gw_plan*) { return GW_EUNSUPPORTED; }
const char* gw_plan_describe(const gw_plan*) { return ""; }
}
