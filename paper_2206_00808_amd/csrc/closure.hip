// Learned closure of the truncated conduction-band sum (placeholder entry points).
#include "common.h"

extern "C" {
gw_status gw_mlp_create(gw_ctx* c, gw_mlp** net, int, int, int, int, uint64_t) {
  if (net) *net = nullptr;
  return gw::fail(c, GW_EUNSUPPORTED, "closure network not built yet");
}
gw_status gw_mlp_destroy(gw_mlp*) { return GW_EUNSUPPORTED; }
gw_status gw_mlp_save(const gw_mlp*, void*, size_t*) { return GW_EUNSUPPORTED; }
gw_status gw_mlp_load(gw_mlp*, const void*, size_t) { return GW_EUNSUPPORTED; }
gw_status gw_chi0_closure(gw_ctx* c, gw_mlp*, int, int, const double*, const double*, double,
                          double, const double*, float, float*, double*) {
  return gw::fail(c, GW_EUNSUPPORTED, "closure network not built yet");
}
}
