// Serving loop: continuous batching of Helmholtz solve requests.
#include "hh_internal.h"

extern "C" {
int hh_server_create(size_t, int, hh_server** out) {
  if (out) *out = nullptr;
  hh::set_error("serving not built yet");
  return HH_EINVAL;
}
int hh_submit(hh_server*, const hh_request*, uint64_t*) { return HH_EINVAL; }
int hh_poll(hh_server*, uint64_t, hh_result*) { return HH_EINVAL; }
double hh_server_clock(const hh_server*) { return 0.0; }
int hh_server_destroy(hh_server*) { return HH_OK; }
}
