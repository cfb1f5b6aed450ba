// Host side of the fused 3-D kernel (swc_corr3d.hpp): geometry, launch
// configuration checks and dispatch to the per-mode instantiations.
#include "swc_corr3d.hpp"
#include "swc_internal.h"

namespace swc {

static int wq3_of(int kw, int sx)
{
    const int R = 4;
    const int span = kWave * R - (R - 1);
    if (span < kw) return 0;
    return (span - kw) / sx + 1;
}

bool cfg_ok_3d(const swc_problem& p, const LaunchCfg& L)
{
    const int mode = mode_of(p.dtype, p.accum);
    if (!fast3d_supported(mode, p.window[2])) return false;
    if (L.R != 4) return false;
    if (!(L.wpb == 1 || L.wpb == 2 || L.wpb == 4)) return false;
    if (L.TH < 1 || L.TH > 4096) return false;
    if (!(L.TY == 2 || L.TY == 4)) return false;
    for (int d = 0; d < 3; d++)
        if (p.shape[d] >= ((int64_t)1 << 30)) return false;
    // rows are addressed as raw buffers of at most 2^31 - 1 bytes
    if (p.shape[2] * 4 >= ((int64_t)1 << 31) - 64) return false;
    return wq3_of(p.window[2], p.step[2]) >= 1;
}

hipError_t launch_corr3d(const swc_problem& p, const int64_t* oshape, const LaunchCfg& L,
                         const void* x, const void* y, float* c, uint8_t* flags,
                         hipStream_t s, int force)
{
    const int mode = mode_of(p.dtype, p.accum);
    P3D g;
    g.x = x;
    g.y = y;
    g.c = c;
    g.flags = flags;
    g.D = (int)p.shape[0];
    g.H = (int)p.shape[1];
    g.W = (int)p.shape[2];
    g.OD = (int)oshape[0];
    g.OH = (int)oshape[1];
    g.OW = (int)oshape[2];
    g.kz = p.window[0];
    g.ky = p.window[1];
    g.sz = p.step[0];
    g.sy = p.step[1];
    g.sx = p.step[2];
    g.oz = window_offset(p.border, p.window[0]);
    g.oy = window_offset(p.border, p.window[1]);
    g.ox = window_offset(p.border, p.window[2]);
    g.border = p.border;
    g.invalid = p.invalid_value;
    g.miss_thr = missing_threshold(p.missing_le);
    g.force = force;
    g.TZ = L.TH;
    g.Wq = wq3_of(p.window[2], p.step[2]);
    g.tiles_x = (g.OW + g.Wq - 1) / g.Wq;
    g.tiles_y = (g.OH + L.TY - 1) / L.TY;
    g.tiles_z = (g.OD + g.TZ - 1) / g.TZ;
    const int64_t nt = (int64_t)g.tiles_x * g.tiles_y * g.tiles_z;
    if (nt >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    g.n_tiles = (int)nt;
    // certification: chain = z-march steps plus the per-step y and x sums
    const double nzs = (double)(g.TZ - 1) * g.sz + g.kz;
    const double chain = 2.0 * nzs + 2.0 * ((L.TY - 1) * g.sy + g.ky) + p.window[2] + 16.0;
    const double n = (double)g.kz * g.ky * p.window[2];
    const double nterms = (double)(g.kz + 1) * (g.ky + 1) * (p.window[2] + 1);
    g.cert_g = cert_factor(mode, n, chain, nterms);
    const size_t esz = p.dtype == SWC_U8 ? 1 : (p.dtype == SWC_U16 ? 2 : 4);
    const bool vec = ((uintptr_t)x % (esz * 4) == 0) && ((uintptr_t)y % (esz * 4) == 0) &&
                     (g.W % 4 == 0);
    const int kw = p.window[2];
    // specialised step: square (y, x) window, unit y step, two rows per wave,
    // vector loads, every plane addressable with 30-bit offsets
    const bool cube = vec && L.TY == 2 && p.window[1] == kw && p.step[1] == 1 &&
                      (int64_t)g.H * g.W * (int64_t)esz < ((int64_t)1 << 30) && !(force & 2);
    // halves: two 32-lane halves of 120 outputs on adjacent row pairs, when
    // that leaves fewer lanes past the last output column than whole waves
    int variant = cube ? 1 : 0;
    if (cube && p.step[2] == 1 && p.border != SWC_BORDER_VALID) {
        const int64_t lanes_whole = (int64_t)((g.OW + 247) / 248) * 64;
        const int64_t lanes_half = (int64_t)((g.OW + 119) / 120) * 32;
        if (lanes_half < lanes_whole) {
            variant = 2;
            g.Wq = 120;
            g.tiles_x = (g.OW + g.Wq - 1) / g.Wq;
            g.tiles_y = (g.OH + 2 * L.TY - 1) / (2 * L.TY);
            const int64_t nt2 = (int64_t)g.tiles_x * g.tiles_y * g.tiles_z;
            if (nt2 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
            g.n_tiles = (int)nt2;
        }
    }
    // waves per workgroup: halved while the LDS running sums would exceed 64 KB
    const int lds_wave = cube ? cube_lds_bytes(mode, 4) : tile3d_lds_bytes(mode, L.TY, 4);
    int wpb = L.wpb;
    while (wpb > 1 && (int64_t)wpb * lds_wave > 64 * 1024) wpb /= 2;
    const int grid = (int)(((int64_t)g.n_tiles + wpb - 1) / wpb);
    if (mode == MODE_U8) return launch_fast3d_modeu8(g, kw, L.TY, vec, variant, grid, wpb, s);
    if (mode == MODE_U16) return launch_fast3d_modeu16(g, kw, L.TY, vec, variant, grid, wpb, s);
    return launch_fast3d_modef64(g, kw, L.TY, vec, variant, grid, wpb, s);
}

}  // namespace swc
