// server.cpp -- placeholder, replaced by the continuous-batching runtime.
#include "hom.h"

extern "C" {
hom_status hom_server_create(size_t, const hom_options*, hom_server** out) {
  if (out) *out = nullptr;
  return HOM_EINVAL;
}
hom_status hom_server_submit(hom_server*, hom_cell*, int, const double*, double, uint64_t*) {
  return HOM_EINVAL;
}
hom_status hom_server_poll(hom_server*, uint64_t, double*, double*, hom_info*) { return HOM_EINVAL; }
hom_status hom_server_times(hom_server*, uint64_t, double*) { return HOM_EINVAL; }
hom_status hom_server_destroy(hom_server*) { return HOM_EINVAL; }
}
