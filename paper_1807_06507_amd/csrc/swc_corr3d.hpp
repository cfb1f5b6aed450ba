// Fused 3-D sliding-window correlation (Poyda & Zhizhin, arXiv 1807.06507:
// Section 1 steps 1-4 with the summation repeated once per dimension, as the
// n-dimensional remark of Section 1 describes).
//
// One wavefront owns a tile of TZ output planes x TY output rows x Wq output
// columns (lanes own R adjacent columns, as in the 2-D kernel) and marches
// along z.  Per step it forms, for the TY rows' window rows, the element
// difference of the five channel contributions between the plane entering
// the z-window and the plane leaving it; sums those differences over each
// output row's y-window in registers; takes the x-window through the DPP
// halo exchange of the 2-D kernel; and adds the result to the running 3-D
// sums S3[TY][R] kept in registers.  Because the 2-D box is linear, this is
// box(entering) - box(leaving) computed once.  Output planes are finished
// (epilogue + store) as soon as their z-window is complete.
// Tiles are numbered with y fastest, so the tiles that share a y-halo run at
// the same time and march z in step (their shared rows hit the same L2).
#pragma once

#include "swc_corr2d_fast.hpp"

namespace swc {

struct P3D {
    const void* x;
    const void* y;
    float* c;
    uint8_t* flags;
    int D, H, W, OD, OH, OW;
    int kz, ky, sz, sy, sx, oz, oy, ox;
    int border;
    float invalid;
    float miss_thr;
    int force;
    double cert_g;
    int TZ, Wq, tiles_x, tiles_y, tiles_z, n_tiles;
};

__host__ __device__ inline bool fast3d_supported(int mode, int KW)
{
    if (mode != MODE_U8 && mode != MODE_U16 && mode != MODE_F64) return false;
    return KW == 3 || KW == 5 || KW == 7 || KW == 9;
}

hipError_t launch_fast3d_modeu8(const P3D& g, int KW, int TY, bool vec, int grid, int wpb,
                                hipStream_t s);
hipError_t launch_fast3d_modeu16(const P3D& g, int KW, int TY, bool vec, int grid, int wpb,
                                 hipStream_t s);
hipError_t launch_fast3d_modef64(const P3D& g, int KW, int TY, bool vec, int grid, int wpb,
                                 hipStream_t s);

// Contribution difference (entering minus leaving) of one element pair, in
// the running-sum representation of Col<M> (integer modes keep 2*Sxy).
template <int M, class T>
__device__ __forceinline__ Col<M> col_delta(T a, T b, T ao, T bo, int m, int mo)
{
    Col<M> d;
    if constexpr (M == MODE_F64) {
        const double x = (double)a, y = (double)b, xo = (double)ao, yo = (double)bo;
        d.x = x - xo;
        d.y = y - yo;
        d.xx = __builtin_fma(x, x, -(xo * xo));
        d.yy = __builtin_fma(y, y, -(yo * yo));
        d.xy = __builtin_fma(x, y, -(xo * yo));
        d.miss = m - mo;
    } else {
        col_zero<M>(d);
        col_update_int<M>(d, (int)a, (int)b, (int)ao, (int)bo);
    }
    return d;
}

template <int M, int R, int KW, int TY, bool VEC>
__device__ __forceinline__ void tile3d(const P3D& g, const int tile)
{
    using T = typename Tr<M>::T;
    constexpr int LH = KW / 2;
    constexpr int RH = KW - 1 - LH;
    constexpr int NW = Run<T, R>::NW;
    constexpr bool kFloat = (M == MODE_F64);
    const int lane = threadIdx.x & (kWave - 1);

    // ---- tile geometry: y fastest, then x, then z ----
    const int ty = tile % g.tiles_y;
    const int rest = tile / g.tiles_y;
    const int tx = rest % g.tiles_x;
    const int tz = rest / g.tiles_x;
    const int pz0 = tz * g.TZ;
    const int pzn = min(g.TZ, g.OD - pz0);
    const int py0 = ty * TY;
    const int pyn = min(TY, g.OH - py0);
    const int q0 = tx * g.Wq;
    const int qw = min(g.Wq, g.OW - q0);
    const int D = g.D, H = g.H, W = g.W;
    const int E = q0 * g.sx + g.ox;
    const int Eal = (E >= 0) ? (E / R) * R : -((-E + R - 1) / R) * R;
    const bool fill = g.border == BORDER_FILL;
    const bool has_flags = g.flags != nullptr;

    // ---- per-lane column metadata ----
    const int c0 = Eal + lane * R;
    const bool edge = (Eal < 0) || (Eal + kWave * R > W);
    int cidx[R];
    uint32_t colok = 0;
#pragma unroll
    for (int j = 0; j < R; j++) {
        const int c = c0 + j;
        const bool ok = c >= 0 && c < W;
        colok |= ok ? (1u << j) : 0u;
        cidx[j] = ok ? c : (c < 0 ? 0 : W - 1);
    }
    const uint32_t lane_boff = VEC ? (uint32_t)((colok & 1u) ? c0 : 0) * (uint32_t)sizeof(T) : 0u;
    uint32_t omask = 0, fillb = 0;
    int qj[R];
    double ncol[R];
#pragma unroll
    for (int j = 0; j < R; j++) {
        const int qs = c0 + j - g.ox - LH;
        int q = -1;
        if (qs >= 0) {
            q = (g.sx == 1) ? qs : qs / g.sx;
            if (q * g.sx != qs) q = -1;
        }
        omask |= (q >= q0 && q < q0 + qw) ? (1u << j) : 0u;
        qj[j] = q;
        const int clo = q * g.sx + g.ox, chi = clo + KW - 1;
        fillb |= (fill && (clo < 0 || chi >= W)) ? (1u << j) : 0u;
        ncol[j] = (double)(min(chi, W - 1) - max(clo, 0) + 1);
    }

    // ---- rows of the y-windows of this tile's output rows ----
    const int ys = py0 * g.sy + g.oy;               // first window row
    const int nyr = (pyn - 1) * g.sy + g.ky;        // window rows in the tile
    double nrow[TY];
    bool rowb[TY];
#pragma unroll
    for (int t = 0; t < TY; t++) {
        const int lo = (py0 + t) * g.sy + g.oy, hi = lo + g.ky - 1;
        rowb[t] = fill && (lo < 0 || hi >= H);
        nrow[t] = (double)(min(hi, H - 1) - max(lo, 0) + 1);
    }
    // ---- planes ----
    const int zs = pz0 * g.sz + g.oz;               // first window plane
    const int nz = (pzn - 1) * g.sz + g.kz;

    const char* __restrict__ Xb = (const char*)g.x;
    const char* __restrict__ Yb = (const char*)g.y;
    const size_t plane = (size_t)H * (size_t)W;
    auto load = [&](int z, int r, T (&vx)[R], T (&vy)[R]) {
        const bool ok = z >= 0 && z < D && r >= 0 && r < H;
        const size_t rb = ok ? ((size_t)z * plane + (size_t)r * W) : 0;
        if constexpr (VEC) {
            uint32_t wx[NW], wy[NW];
            const T* px = (const T*)__builtin_assume_aligned(Xb + rb * sizeof(T) + lane_boff, sizeof(T) * R);
            const T* py = (const T*)__builtin_assume_aligned(Yb + rb * sizeof(T) + lane_boff, sizeof(T) * R);
            __builtin_memcpy(wx, px, sizeof(T) * R);
            __builtin_memcpy(wy, py, sizeof(T) * R);
            __builtin_memcpy(vx, wx, sizeof(T) * R);
            __builtin_memcpy(vy, wy, sizeof(T) * R);
        } else {
            const T* xr = (const T*)g.x + rb;
            const T* yr = (const T*)g.y + rb;
#pragma unroll
            for (int j = 0; j < R; j++) { vx[j] = xr[cidx[j]]; vy[j] = yr[cidx[j]]; }
        }
#pragma unroll
        for (int j = 0; j < R; j++) {
            const bool v = ok && (!edge || ((colok >> j) & 1u));
            vx[j] = v ? vx[j] : (T)0;
            vy[j] = v ? vy[j] : (T)0;
        }
    };

    Col<M> S3[TY][R];
#pragma unroll
    for (int t = 0; t < TY; t++)
#pragma unroll
        for (int j = 0; j < R; j++) col_zero<M>(S3[t][j]);
    float hmx = 0.f, hmy = 0.f;

    int next_ready = g.kz - 1;
    int pz = pz0;
    for (int li = 0; li < nz; li++) {
        const int zin = zs + li;
        const int zout = zin - g.kz;
        const bool has_out = li >= g.kz;
        // ---- y-window sums of the z-difference field ----
        Col<M> VY[TY][R];
#pragma unroll
        for (int t = 0; t < TY; t++)
#pragma unroll
            for (int j = 0; j < R; j++) col_zero<M>(VY[t][j]);
        for (int r = 0; r < nyr; r++) {
            T ax[R], ay[R], bx[R], by[R];
            load(zin, ys + r, ax, ay);
            if (has_out) {
                load(zout, ys + r, bx, by);
            } else {
#pragma unroll
                for (int j = 0; j < R; j++) { bx[j] = (T)0; by[j] = (T)0; }
            }
            int m[R], mo[R];
#pragma unroll
            for (int j = 0; j < R; j++) {
                m[j] = 0;
                mo[j] = 0;
                if constexpr (kFloat) {
                    m[j] = (is_missing(ax[j], g.miss_thr) || is_missing(ay[j], g.miss_thr)) ? 1 : 0;
                    mo[j] = (is_missing(bx[j], g.miss_thr) || is_missing(by[j], g.miss_thr)) ? 1 : 0;
                    ax[j] = m[j] ? 0.f : ax[j];
                    ay[j] = m[j] ? 0.f : ay[j];
                    bx[j] = mo[j] ? 0.f : bx[j];
                    by[j] = mo[j] ? 0.f : by[j];
                    hmx = fmaxf(hmx, __builtin_fabsf(ax[j]));
                    hmy = fmaxf(hmy, __builtin_fabsf(ay[j]));
                }
            }
#pragma unroll
            for (int j = 0; j < R; j++) {
                const Col<M> d = col_delta<M, T>(ax[j], ay[j], bx[j], by[j], m[j], mo[j]);
#pragma unroll
                for (int t = 0; t < TY; t++) {
                    const int lo = t * g.sy;
                    if (t < pyn && r >= lo && r < lo + g.ky) col_add<M>(VY[t][j], d);
                }
            }
        }
        // ---- x-window through the halo exchange, accumulated into S3 ----
#pragma unroll
        for (int t = 0; t < TY; t++) {
            Col<M> S, keepL[R > 1 ? R - 1 : 1], keepR[R > 1 ? R - 1 : 1];
            halo_window<M, R, KW>(VY[t], S, keepL, keepR);
#pragma unroll
            for (int j = 0; j < R; j++) {
                if (j > 0) {
                    const int ca = j + RH, cs = j - 1 - LH;
                    const Col<M>& va = ca < R ? VY[t][ca] : keepR[ca - RH - 1];
                    const Col<M>& vs = cs < 0 ? keepL[cs + LH] : VY[t][cs];
                    col_add<M>(S, va);
                    col_sub<M>(S, vs);
                }
                col_add<M>(S3[t][j], S);
            }
        }
        if (li != next_ready) continue;
        next_ready += g.sz;

        // ---- epilogue for output plane pz ----
        const int zlo = pz * g.sz + g.oz, zhi = zlo + g.kz - 1;
        const bool zb = fill && (zlo < 0 || zhi >= D);
        const double nzp = (double)(min(zhi, D - 1) - max(zlo, 0) + 1);
        double gx = 0.0, gy = 0.0;
        if constexpr (kFloat) {
            // bound on |x|, |y| over every value in the running sums: wave max
            float mx = hmx, my = hmy;
            for (int sft = 1; sft < kWave; sft <<= 1) {
                mx = fmaxf(mx, __shfl_xor(mx, sft));
                my = fmaxf(my, __shfl_xor(my, sft));
            }
            gx = g.cert_g * (double)mx * (double)mx;
            gy = g.cert_g * (double)my * (double)my;
        }
#pragma unroll
        for (int t = 0; t < TY; t++) {
            if (t >= pyn) continue;
            const size_t orow = ((size_t)pz * g.OH + (size_t)(py0 + t)) * (size_t)g.OW;
#pragma unroll
            for (int j = 0; j < R; j++) {
                if (!((omask >> j) & 1u)) continue;
                const Col<M>& A = S3[t][j];
                const bool fb = zb || rowb[t] || ((fillb >> j) & 1u);
                const double dn = nzp * nrow[t] * ncol[j];
                uint8_t fl = 0;
                float cv = 0.f;
                if (fb) {
                    fl = FL_BORDER;
                } else if constexpr (kFloat) {
                    if (A.miss > 0) {
                        fl = FL_MISSING;
                    } else {
                        Acc<MODE_F64> acc;
                        acc.x = A.x; acc.y = A.y; acc.xx = A.xx; acc.xy = A.xy; acc.yy = A.yy;
                        acc.miss = 0;
                        const int64_t clo = (int64_t)qj[j] * g.sx + g.ox;
                        const int64_t ylo = (int64_t)(py0 + t) * g.sy + g.oy;
                        WinBox wb{(int64_t)plane, (int64_t)W, max(zlo, 0), min(zhi, D - 1),
                                  max(ylo, (int64_t)0), min(ylo + g.ky - 1, (int64_t)H - 1),
                                  max(clo, (int64_t)0), min(clo + KW - 1, (int64_t)W - 1)};
                        // certification against the per-plane thresholds
                        const double N = __builtin_fma(dn, A.xy, -(A.x * A.y));
                        const double Vx = __builtin_fma(dn, A.xx, -(A.x * A.x));
                        const double Vy = __builtin_fma(dn, A.yy, -(A.y * A.y));
                        const bool cert = (Vx > gx) && (Vy > gy) && !(g.force & 1);
                        if (cert) {
                            cv = clamp_unit(N * rsqrt64(Vx * Vy));
                        } else {
                            fl = twopass_window((const float*)g.x, (const float*)g.y, wb.s0, wb.s1,
                                                wb.lo0, wb.hi0, wb.lo1, wb.hi1, wb.lo2, wb.hi2, &cv);
                        }
                    }
                } else {
                    const double sxv = (double)A.x, syv = (double)A.y;
                    const double N = __builtin_fma(0.5 * dn, (double)A.xy2, -(sxv * syv));
                    const double Vx = __builtin_fma(dn, (double)A.xx, -(sxv * sxv));
                    const double Vy = __builtin_fma(dn, (double)A.yy, -(syv * syv));
                    fl = (Vx == 0.0 ? FL_ZVAR_X : 0) | (Vy == 0.0 ? FL_ZVAR_Y : 0);
                    if (!fl) cv = rn32_certified(N, Vx, Vy, (g.force & 1) != 0);
                }
                if (fl) cv = g.invalid;
                g.c[orow + (uint32_t)qj[j]] = cv;
                if (has_flags) g.flags[orow + (uint32_t)qj[j]] = fl;
            }
        }
        ++pz;
    }
}

template <int M, int R, int KW, int TY, bool VEC>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(2, 8))) corr3d_kernel(P3D g)
{
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
    const int wpb = blockDim.x / kWave;
    const int tile = xcd_remap(blockIdx.x, gridDim.x) * wpb + wv;
    if (tile >= g.n_tiles) return;
    tile3d<M, R, KW, TY, VEC>(g, tile);
}

}  // namespace swc
