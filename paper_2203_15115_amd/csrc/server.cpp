// placeholder, replaced below
#include "afd_internal.h"
extern "C" {
int afd_server_create(afd_context*, uint64_t, int32_t, afd_server** out) { if (out) *out = nullptr; afd::set_error("server: not available"); return AFD_E_INVALID_ARG; }
int afd_server_submit(afd_server*, const afd_request*, afd_result*, uint64_t*) { return AFD_E_INVALID_ARG; }
int afd_server_poll(afd_server*, uint64_t) { return AFD_E_INVALID_ARG; }
int afd_server_wait(afd_server*, uint64_t, double) { return AFD_E_INVALID_ARG; }
double afd_server_clock(afd_server*) { return 0.0; }
void afd_server_destroy(afd_server*) {}
}
