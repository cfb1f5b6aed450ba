// 3-D sliding-window correlation (not yet implemented in this build).
#include "swc_device.hpp"
#include "swc_internal.h"

namespace swc {

bool cfg_ok_3d(const swc_problem&, const LaunchCfg&) { return false; }

hipError_t launch_corr3d(const swc_problem&, const int64_t*, const LaunchCfg&, const void*,
                         const void*, float*, uint8_t*, hipStream_t, int)
{
    return hipErrorNotSupported;
}

}  // namespace swc
