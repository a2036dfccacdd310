// Serving engine (continuous batching) - placeholder until implemented.
#include "bhx_runtime.h"

extern "C" {
int bhx_engine_create(bhx_engine** e, int, size_t, int, const bhx_opts*) {
  if (e) *e = nullptr;
  return BHX_ERR_ARG;
}
int bhx_engine_submit(bhx_engine*, const double*, double*, int, int, double, int, double,
                      uint64_t*) { return BHX_ERR_ARG; }
int bhx_engine_poll(bhx_engine*, uint64_t*, bhx_stats*, int, int* n) {
  if (n) *n = 0;
  return BHX_ERR_ARG;
}
int bhx_engine_inflight(bhx_engine*) { return 0; }
void bhx_engine_destroy(bhx_engine*) {}
}
