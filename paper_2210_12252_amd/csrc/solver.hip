// Block eigensolver (placeholder until the LOBPCG driver lands).
#include <hip/hip_runtime.h>

#include "device_state.hpp"
#include "helic_internal.h"

namespace helic {
void release_solver_state(DeviceState*) {}
}  // namespace helic

extern "C" helic_status helic_eigensolve(helic_basis h, int32_t, int32_t, double, int32_t, helic_prec,
                                         uint64_t, double*, double*, double*, int64_t, int32_t*, void*) {
  if (!h) return helic::fail(HELIC_ERR_INVALID, "null handle");
  return helic::fail(HELIC_ERR_UNSUPPORTED, "eigensolver not built yet");
}
