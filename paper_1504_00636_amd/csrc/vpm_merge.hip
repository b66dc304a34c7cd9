// Replacement from a given partition (vpm_merge).
#include "vpm_device.hpp"
#include "vpm_internal.h"

namespace vpm {

hipError_t launch_fixed_merge(const Workspace&, const LaunchCfg&, const Soa32&, const int64_t*, int64_t, int32_t,
                              const FixedParams&, const int32_t*, const int32_t*, const int32_t*) {
    return hipErrorNotSupported;
}

hipError_t launch_fp64_merge(const Workspace&, const LaunchCfg&, const Soa64&, const int64_t*, int64_t,
                             const Fp64Params&, const int32_t*, const int32_t*, const int32_t*) {
    return hipErrorNotSupported;
}

}  // namespace vpm
