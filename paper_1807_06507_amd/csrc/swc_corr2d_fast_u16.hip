// Instantiations of the register-resident 2-D kernel for MODE_U16.
#include "swc_corr2d_fast.hpp"
#include "swc_internal.h"

namespace swc {

template <int R, int KW>
static hipError_t go(const P2DF& g, bool vec, int grid, int wpb, size_t smem, hipStream_t s)
{
    if (vec)
        hipLaunchKernelGGL((corr2d_fast_kernel<MODE_U16, R, KW, true>), dim3(grid), dim3(wpb * kWave), smem, s, g);
    else
        hipLaunchKernelGGL((corr2d_fast_kernel<MODE_U16, R, KW, false>), dim3(grid), dim3(wpb * kWave), smem, s, g);
    return hipGetLastError();
}

hipError_t launch_fast2d_modeu16(const P2DF& g, int R, int KW, bool vec, int grid, int wpb, size_t smem, hipStream_t s)
{
    if (R == 4) {
        switch (KW) {
        case 3: return go<4, 3>(g, vec, grid, wpb, smem, s);
        case 5: return go<4, 5>(g, vec, grid, wpb, smem, s);
        case 7: return go<4, 7>(g, vec, grid, wpb, smem, s);
        case 9: return go<4, 9>(g, vec, grid, wpb, smem, s);
        case 15: return go<4, 15>(g, vec, grid, wpb, smem, s);
        case 31: return go<4, 31>(g, vec, grid, wpb, smem, s);
        default: break;
        }
    } else if (R == 8) {
        switch (KW) {
        case 7: return go<8, 7>(g, vec, grid, wpb, smem, s);
        case 15: return go<8, 15>(g, vec, grid, wpb, smem, s);
        case 31: return go<8, 31>(g, vec, grid, wpb, smem, s);
        default: break;
        }
    }
    return hipErrorNotSupported;
}

}  // namespace swc
