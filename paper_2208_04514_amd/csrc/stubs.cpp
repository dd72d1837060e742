// Temporary: entry points whose implementation is not in this build yet.
#include "internal.hpp"
namespace dawn {
dawn_status autotune(Ctx*, GraphRec*, const int32_t*, int32_t, uint32_t, dawn_params*) {
  return fail(DAWN_E_DEVICE, "autotuner not built");
}
void server_stop(Server*) {}
dawn_status serve_submit(Ctx*, int32_t, const int32_t*, int32_t, int32_t*, uint32_t, uint64_t*) {
  return fail(DAWN_E_DEVICE, "serving not built");
}
dawn_status serve_poll(Ctx*, uint64_t, int32_t, dawn_query_stats*) {
  return fail(DAWN_E_NOT_FOUND, "serving not built");
}
}  // namespace dawn
