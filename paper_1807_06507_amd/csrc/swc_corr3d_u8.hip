// Instantiations of the fused 3-D kernel for MODE_U8.
#include "swc_corr3d.hpp"
#include "swc_internal.h"

namespace swc {

template <int KW, int TY>
static hipError_t go3(const P3D& g, bool vec, int cube, int grid, int wpb, hipStream_t s)
{
    const size_t smem = (size_t)wpb * tile3d_lds_per_wave<MODE_U8, TY>(4);
    if constexpr (TY == 2) {
        const size_t smemc = (size_t)wpb * cube_lds_per_wave<MODE_U8>(4);
        if (cube == 2 && vec) {
            return launch_kernel(&corr3d_kernel<MODE_U8, 4, KW, 2, true, 2>, dim3(grid),
                                 dim3(wpb * kWave), smemc, s, g);
        }
        if (cube == 1 && vec) {
            return launch_kernel(&corr3d_kernel<MODE_U8, 4, KW, 2, true, 1>, dim3(grid),
                                 dim3(wpb * kWave), smemc, s, g);
        }
    }
    if (vec)
        return launch_kernel(&corr3d_kernel<MODE_U8, 4, KW, TY, true, 0>, dim3(grid),
                             dim3(wpb * kWave), smem, s, g);
    return launch_kernel(&corr3d_kernel<MODE_U8, 4, KW, TY, false, 0>, dim3(grid),
                         dim3(wpb * kWave), smem, s, g);
}

template <int TY>
static hipError_t pick_kw(const P3D& g, int KW, bool vec, int cube, int grid, int wpb,
                          hipStream_t s)
{
    switch (KW) {
    case 3: return go3<3, TY>(g, vec, cube, grid, wpb, s);
    case 5: return go3<5, TY>(g, vec, cube, grid, wpb, s);
    case 7: return go3<7, TY>(g, vec, cube, grid, wpb, s);
    case 9: return go3<9, TY>(g, vec, cube, grid, wpb, s);
    default: return hipErrorNotSupported;
    }
}

hipError_t launch_fast3d_modeu8(const P3D& g, int KW, int TY, bool vec, int cube, int grid, int wpb,
                hipStream_t s)
{
    return TY == 4 ? pick_kw<4>(g, KW, vec, cube, grid, wpb, s)
                   : pick_kw<2>(g, KW, vec, cube, grid, wpb, s);
}

}  // namespace swc
