// Instantiations of the register-resident 2-D kernel for MODE_U8.
#include "swc_corr2d_fast.hpp"
#include "swc_internal.h"

namespace swc {

// Launch (occ == nullptr) or report resident workgroups per CU (occ != nullptr).
template <int R, int KW, bool VEC>
static hipError_t go1(const P2DF& g, int grid, int wpb, size_t smem, hipStream_t s, int* occ)
{
    if (occ)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            occ, corr2d_fast_kernel<MODE_U8, R, KW, VEC>, wpb * kWave, smem);
    return launch_kernel(&corr2d_fast_kernel<MODE_U8, R, KW, VEC>, dim3(grid), dim3(wpb * kWave), smem, s, g);
}

template <int R, int KW>
static hipError_t go(const P2DF& g, bool vec, int grid, int wpb, size_t smem, hipStream_t s, int* occ)
{
    return vec ? go1<R, KW, true>(g, grid, wpb, smem, s, occ)
               : go1<R, KW, false>(g, grid, wpb, smem, s, occ);
}

hipError_t launch_fast2d_modeu8(const P2DF& g, int R, int KW, bool vec, int grid, int wpb,
                                size_t smem, hipStream_t s, int* occ)
{
    if (R == 4) {
        switch (KW) {
        case 3: return go<4, 3>(g, vec, grid, wpb, smem, s, occ);
        case 5: return go<4, 5>(g, vec, grid, wpb, smem, s, occ);
        case 7: return go<4, 7>(g, vec, grid, wpb, smem, s, occ);
        case 9: return go<4, 9>(g, vec, grid, wpb, smem, s, occ);
        case 15: return go<4, 15>(g, vec, grid, wpb, smem, s, occ);
        case 31: return go<4, 31>(g, vec, grid, wpb, smem, s, occ);
        default: break;
        }
    } else if (R == 8) {
        switch (KW) {
        case 7: return go<8, 7>(g, vec, grid, wpb, smem, s, occ);
        case 15: return go<8, 15>(g, vec, grid, wpb, smem, s, occ);
        case 31: return go<8, 31>(g, vec, grid, wpb, smem, s, occ);
        default: break;
        }
    }
    return hipErrorNotSupported;
}

}  // namespace swc
