// Serving entry points (include/fpm.h).  Placeholder until the request loop
// lands: every call reports FPM_E_UNSUPPORTED.
#include "fpm_internal.h"
#include "runtime.h"

using namespace fpm;

extern "C" {
fpm_status fpm_server_create(size_t, int32_t, fpm_server_t** out) {
  if (out) *out = nullptr;
  return fail(FPM_E_UNSUPPORTED, "serving is not built yet");
}
void fpm_server_destroy(fpm_server_t*) {}
fpm_status fpm_submit(fpm_server_t*, const fpm_tile_desc*, const float*, fpm_mem, uint64_t*) {
  return fail(FPM_E_UNSUPPORTED, "serving is not built yet");
}
fpm_status fpm_poll(fpm_server_t*, uint64_t, void*, void*, double*, fpm_request_stats*) {
  return fail(FPM_E_UNSUPPORTED, "serving is not built yet");
}
fpm_status fpm_wait(fpm_server_t*, uint64_t, double, void*, void*, double*, fpm_request_stats*) {
  return fail(FPM_E_UNSUPPORTED, "serving is not built yet");
}
fpm_status fpm_cancel(fpm_server_t*, uint64_t) {
  return fail(FPM_E_UNSUPPORTED, "serving is not built yet");
}
}
