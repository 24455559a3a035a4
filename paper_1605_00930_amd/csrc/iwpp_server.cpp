// iwpp_server.cpp -- continuous-batching request server (C ABI in iwpp.h).
#include "iwpp.h"

extern "C" {
int iwpp_server_create(size_t, int, int, int, int, iwpp_server** out) {
  if (out) *out = nullptr;
  return IWPP_E_UNSUPPORTED;
}
int iwpp_server_submit(iwpp_server*, const iwpp_image*, uint64_t*) { return IWPP_E_UNSUPPORTED; }
int iwpp_server_wait(iwpp_server*, uint64_t, int64_t, double*) { return IWPP_E_UNSUPPORTED; }
int iwpp_server_destroy(iwpp_server*) { return IWPP_E_UNSUPPORTED; }
}
