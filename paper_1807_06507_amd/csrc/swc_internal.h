// Host-side interfaces between the C ABI (swc_api.cpp) and the kernel
// translation units.  Internal to libswcorr.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <tuple>
#include <type_traits>
#include <utility>

#include "swcorr.h"

namespace swc {

// Launch `k` on stream `s` and return the status of this launch itself, from
// the launch call's own return value.  The runtime's per-thread "last error"
// is neither read nor cleared, so an error that other work left pending stays
// with its owner and is never reported as this launch's.
template <typename... KArgs, typename... Args>
inline hipError_t launch_kernel(void (*k)(KArgs...), dim3 grid, dim3 block, size_t smem,
                                hipStream_t s, Args&&... args)
{
    static_assert(sizeof...(KArgs) == sizeof...(Args), "kernel argument count");
    std::tuple<typename std::decay<KArgs>::type...> vals(std::forward<Args>(args)...);
    return std::apply(
        [&](auto&... v) {
            void* argv[] = {(void*)&v...};
            return hipLaunchKernel((const void*)k, grid, block, argv, smem, s);
        },
        vals);
}

// Evaluate a launch; return its status from the enclosing function on failure.
#define SWC_TRY(expr)                       \
    do {                                    \
        const hipError_t swc_e_ = (expr);   \
        if (swc_e_ != hipSuccess) return swc_e_; \
    } while (0)

// Errors after which the device cannot run further work (a fault in earlier
// work on it): every later call fails with them.
inline bool sticky_error(hipError_t e)
{
    switch (e) {
    case hipErrorIllegalAddress:
    case hipErrorLaunchFailure:
    case hipErrorAssert:
    case hipErrorLaunchTimeOut:
    case hipErrorECCNotCorrectable:
    case hipErrorContextIsDestroyed:
        return true;
    default:
        return false;
    }
}

// Injected failure for tests of error propagation: with SWC_FAULT_INJECT=launch
// in the environment when the library initialises, every entry point that
// would launch work returns SWC_ERR_LAUNCH instead, before touching the device.
bool fault_inject_launch();

// Status of a failed (or successful) launch: SWC_ERR_DEVICE for a sticky
// device error, SWC_ERR_LAUNCH for any other failure.
swc_status launch_status(hipError_t e);

// Resolved launch configuration.
struct LaunchCfg {
    int R;       // contiguous-axis elements per lane
    int TH;      // rows (2-D) / planes (3-D) / sample rows (1-D) per tile
    int wpb;     // waves per workgroup
    int minw;    // occupancy hint variant (0 = none)
    int TY = 0;  // 3-D: output rows per wave (0 = default)
};

// Kernel mode from (dtype, accum); -1 when the pair is invalid.
int mode_of(int32_t dtype, int32_t accum);

// Largest float f with f <= t (so that float v <= t  <=>  v <= f).
float missing_threshold(double t);

// Rounding-error factor for the float certification test (see the design
// notes): rho * u * n * (3 C Nt + 6 n), with C the longest add/subtract chain
// a window sum goes through and Nt the bound on terms in any partial sum.
double cert_factor(int mode, double n, double chain, double nterms);

// Per-dimension window offset: -floor(k/2) for FILL/CLIP, 0 for VALID.
inline int window_offset(int border, int k) { return border == SWC_BORDER_VALID ? 0 : -(k / 2); }

hipError_t launch_corr1d(const swc_problem& p, const int64_t* oshape, const LaunchCfg& L,
                         const void* x, const void* y, float* c, uint8_t* flags,
                         hipStream_t s, int force);
hipError_t launch_corr2d(const swc_problem& p, const int64_t* oshape, const LaunchCfg& L,
                         const void* x, const void* y, float* c, uint8_t* flags,
                         hipStream_t s, int force);
hipError_t launch_corr3d(const swc_problem& p, const int64_t* oshape, const LaunchCfg& L,
                         const void* x, const void* y, float* c, uint8_t* flags,
                         hipStream_t s, int force);

// Unfused baseline schemes (swc_scheme.hip): support check, workspace size
// and launch.  The workspace must hold scheme_workspace_bytes() bytes,
// 8-byte aligned.
bool scheme_supported(const swc_problem& p, int scheme);
uint64_t scheme_workspace_bytes(const swc_problem& p, int scheme);
hipError_t launch_scheme(const swc_problem& p, int scheme, const void* x, const void* y,
                         float* c, uint8_t* flags, void* ws, hipStream_t s, int force);

// Application kernels on a finished map (swc_mask.hip).
hipError_t launch_cloud_mask(const float* c, const uint8_t* flags, int64_t n, float tau,
                             float invalid, uint8_t* mask, hipStream_t s);
hipError_t launch_filter_detections(const float* c, const uint8_t* flags, int64_t n,
                                    const int64_t* idx, int64_t k, float tau, float invalid,
                                    uint8_t* keep, hipStream_t s);

// Whether a configuration is launchable for the problem (host check).
bool cfg_ok_2d(const swc_problem& p, const LaunchCfg& L);
bool cfg_ok_1d(const swc_problem& p, const LaunchCfg& L);
bool cfg_ok_3d(const swc_problem& p, const LaunchCfg& L);

}  // namespace swc
