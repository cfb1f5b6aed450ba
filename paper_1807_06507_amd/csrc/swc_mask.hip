// The application's consumer of the correlation map (Introduction and
// Conclusion): night-time light detections are false where moonlight is
// reflected by clouds, and there the visible/infrared correlation is close to
// -1.  Two bandwidth-bound kernels:
//   cloud mask          mask[i] = 1 when output i is valid and c[i] < -tau
//   detection filter    keep[j] = 0 when detection j sits on a cloud pixel,
//                       1 otherwise, 2 when its index is outside the map
// "Valid" means flags[i] == 0 when a flag map is given, else c[i] differs
// from the invalid value (a coefficient is never outside [-1, 1]).
#include "swc_device.hpp"
#include "swc_internal.h"

namespace swc {

namespace {

__device__ __forceinline__ bool is_cloud(const float* __restrict__ c,
                                         const uint8_t* __restrict__ flags, int64_t i,
                                         float neg_tau, float invalid)
{
    const float v = c[i];
    const bool valid = flags ? flags[i] == 0 : v != invalid;
    return valid && v < neg_tau;
}

// Four outputs per thread: c as one 16-byte load when aligned.
__global__ void __launch_bounds__(256)
cloud_mask_kernel(const float* __restrict__ c, const uint8_t* __restrict__ flags, int64_t n,
                  float neg_tau, float invalid, uint8_t* __restrict__ mask)
{
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (i0 >= n) return;
    if (i0 + 4 <= n && ((uintptr_t)(c + i0) & 15) == 0 && ((uintptr_t)(mask + i0) & 3) == 0 &&
        (!flags || ((uintptr_t)(flags + i0) & 3) == 0)) {
        const float4 v = *(const float4*)(c + i0);
        const uint32_t f = flags ? *(const uint32_t*)(flags + i0) : 0u;
        const float vv[4] = {v.x, v.y, v.z, v.w};
        uint32_t m = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const bool valid = flags ? ((f >> (8 * k)) & 0xFFu) == 0 : vv[k] != invalid;
            m |= (valid && vv[k] < neg_tau) ? (1u << (8 * k)) : 0u;
        }
        *(uint32_t*)(mask + i0) = m;
    } else {
        for (int64_t i = i0; i < n && i < i0 + 4; i++)
            mask[i] = is_cloud(c, flags, i, neg_tau, invalid) ? 1 : 0;
    }
}

__global__ void __launch_bounds__(256)
filter_kernel(const float* __restrict__ c, const uint8_t* __restrict__ flags, int64_t n,
              const int64_t* __restrict__ idx, int64_t k, float neg_tau, float invalid,
              uint8_t* __restrict__ keep)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= k) return;
    const int64_t i = idx[j];
    keep[j] = (i < 0 || i >= n) ? 2 : (is_cloud(c, flags, i, neg_tau, invalid) ? 0 : 1);
}

}  // namespace

hipError_t launch_cloud_mask(const float* c, const uint8_t* flags, int64_t n, float tau,
                             float invalid, uint8_t* mask, hipStream_t s)
{
    const int64_t groups = (n + 3) / 4;
    const int64_t blocks = (groups + 255) / 256;
    if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    return launch_kernel(&cloud_mask_kernel, dim3((unsigned)blocks), dim3(256), 0, s, c, flags, n,
                       -tau, invalid, mask);
}

hipError_t launch_filter_detections(const float* c, const uint8_t* flags, int64_t n,
                                    const int64_t* idx, int64_t k, float tau, float invalid,
                                    uint8_t* keep, hipStream_t s)
{
    const int64_t blocks = (k + 255) / 256;
    if (blocks >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    return launch_kernel(&filter_kernel, dim3((unsigned)blocks), dim3(256), 0, s, c, flags, n, idx,
                       k, -tau, invalid, keep);
}

}  // namespace swc
