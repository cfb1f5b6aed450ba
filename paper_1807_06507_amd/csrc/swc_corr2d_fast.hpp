// Register-resident fused 2-D kernel (Poyda & Zhizhin, arXiv 1807.06507,
// Section 1 steps 1-4 in one pass) for window widths known at compile time.
//
// One wavefront computes a tile of TH output rows x Wq output columns.  Each
// lane owns R adjacent input columns of the tile (plus halo) and:
//  * step 1-2: marches down the rows keeping the five running column sums in
//    registers.  Entering rows are prefetched D rows ahead into a register
//    ring; every row's raw values are also parked in a small per-wave LDS
//    ring of k_h rows, from which the row leaving the window is read back
//    (no second trip to L2/HBM).  For integer input the running update uses
//    x^2 - x'^2 = (x - x')(x + x') and xy - x'y' = ((x-x')(y+y') + (x+x')(y-y'))/2,
//    so each of the three product sums costs one or two FP64 FMAs on exact
//    integers;
//  * step 3: receives the running sums of the k_w - 1 halo columns from its
//    two neighbour lanes through DPP wavefront shifts (wave_shr:1 /
//    wave_shl:1) and slides the k_w window over its own registers;
//  * step 4: epilogue and store for the columns that are output positions.
// Per-lane column metadata (output index, clipped column count, border bit)
// is computed once per tile; per-row quantities are wave-uniform.
#pragma once

#include "swc_device.hpp"

namespace swc {

struct P2DF {
    const void* x;
    const void* y;
    float* c;
    uint8_t* flags;
    int H, W, OH, OW;          // each below 2^31 (checked on the host)
    int kh, sh, sw, oh, ow;
    int border;
    float invalid;
    float miss_thr;
    int force;
    double cert_g;
    int TH, Wq, tiles_y, n_tiles;
};

// Which (mode, R, KW) combinations have a compiled register-resident kernel.
__host__ __device__ inline bool fast2d_supported(int mode, int R, int KW)
{
    if (mode != MODE_U8 && mode != MODE_U16 && mode != MODE_F64) return false;
    if (R == 4) return KW == 3 || KW == 5 || KW == 7 || KW == 9 || KW == 15 || KW == 31;
    if (R == 8) return KW == 7 || KW == 15 || KW == 31;
    return false;
}

// LDS bytes per wave: the raw-row ring (k_h rows) plus, for integer input,
// a stash of (N, Vx, Vy, estimate) for outputs that take the exact
// rounding decision.
__host__ __device__ inline int fast2d_ring_bytes(int mode, int R, int kh)
{
    const int esz = mode == MODE_U8 ? 1 : (mode == MODE_U16 ? 2 : 4);
    const int nw = (esz * R + 3) / 4;
    const int miss = (mode == MODE_F64) ? 1 : 0;
    return kh * kWave * 4 * (2 * nw + miss);
}
__host__ __device__ inline int fast2d_lds_per_wave(int mode, int R, int kh)
{
    const int stash = (mode == MODE_F64) ? 0 : 3 * 8 * R * kWave;
    return ((fast2d_ring_bytes(mode, R, kh) + 15) & ~15) + stash;
}

hipError_t launch_fast2d_modeu8(const P2DF& g, int R, int KW, bool vec, int grid, int wpb,
                                size_t smem,
                                hipStream_t s);
hipError_t launch_fast2d_modeu16(const P2DF& g, int R, int KW, bool vec, int grid, int wpb,
                                size_t smem,
                                 hipStream_t s);
hipError_t launch_fast2d_modef64(const P2DF& g, int R, int KW, bool vec, int grid, int wpb,
                                size_t smem,
                                 hipStream_t s);

// ---- DPP wavefront shifts (lane i <- lane i-1 / lane i+1) -----------------
__device__ __forceinline__ uint32_t dpp_from_left(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, true);   // wave_shr:1
}
__device__ __forceinline__ uint32_t dpp_from_right(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, true);   // wave_shl:1
}

template <bool LEFT, class V> __device__ __forceinline__ V dpp_move(V v)
{
    static_assert(sizeof(V) % 4 == 0, "32-bit multiples only");
    constexpr int NW = sizeof(V) / 4;
    uint32_t w[NW];
    __builtin_memcpy(w, &v, sizeof(V));
#pragma unroll
    for (int i = 0; i < NW; i++) w[i] = LEFT ? dpp_from_left(w[i]) : dpp_from_right(w[i]);
    V r;
    __builtin_memcpy(&r, w, sizeof(V));
    return r;
}

// ---- running column sums --------------------------------------------------
// Integer modes: Sx, Sy exact int32; Sxx, Syy, 2*Sxy exact integers (int32
// for u8, FP64 for u16).  Float mode: five FP64 sums of exact FP64 products
// plus a count of missing elements.
template <int M> struct Col;
template <> struct Col<MODE_U8> {
    int x, y;
    uint32_t xx, yy, xy2;   // modular arithmetic; true values < 2^32 (n <= 33025)
};
template <> struct Col<MODE_U16> {
    int x, y;
    double xx, yy, xy2;
};
template <> struct Col<MODE_F64> {
    double x, y, xx, yy, xy;
    int miss;
};

template <int M> __device__ __forceinline__ void col_zero(Col<M>& a) { a = Col<M>{}; }

template <bool LEFT, int M> __device__ __forceinline__ Col<M> col_dpp(const Col<M>& a)
{
    Col<M> r;
    r.x = dpp_move<LEFT>(a.x);
    r.y = dpp_move<LEFT>(a.y);
    r.xx = dpp_move<LEFT>(a.xx);
    r.yy = dpp_move<LEFT>(a.yy);
    if constexpr (M == MODE_F64) {
        r.xy = dpp_move<LEFT>(a.xy);
        r.miss = (int)dpp_move<LEFT>((uint32_t)a.miss);
    } else {
        r.xy2 = dpp_move<LEFT>(a.xy2);
    }
    return r;
}

template <int M> __device__ __forceinline__ void col_add(Col<M>& a, const Col<M>& b)
{
    a.x += b.x; a.y += b.y; a.xx += b.xx; a.yy += b.yy;
    if constexpr (M == MODE_F64) { a.xy += b.xy; a.miss += b.miss; }
    else a.xy2 += b.xy2;
}
template <int M> __device__ __forceinline__ void col_sub(Col<M>& a, const Col<M>& b)
{
    a.x -= b.x; a.y -= b.y; a.xx -= b.xx; a.yy -= b.yy;
    if constexpr (M == MODE_F64) { a.xy -= b.xy; a.miss -= b.miss; }
    else a.xy2 -= b.xy2;
}

// Running update with entering (x, y) and leaving (xo, yo) integer values.
template <int M>
__device__ __forceinline__ void col_update_int(Col<M>& a, int x, int y, int xo, int yo)
{
    const int dx = x - xo, sx = x + xo, dy = y - yo, sy = y + yo;
    a.x += dx;
    a.y += dy;
    if constexpr (M == MODE_U8) {
        // |dx| <= 255, sx <= 510: every product fits in int32; the sums are
        // kept modulo 2^32, exact because their true values stay below 2^32
        a.xx += (uint32_t)(dx * sx);
        a.yy += (uint32_t)(dy * sy);
        a.xy2 += (uint32_t)(dx * sy + sx * dy);
    } else {
        const double fdx = (double)dx, fsx = (double)sx, fdy = (double)dy, fsy = (double)sy;
        a.xx = __builtin_fma(fdx, fsx, a.xx);
        a.yy = __builtin_fma(fdy, fsy, a.yy);
        a.xy2 = __builtin_fma(fdx, fsy, a.xy2);
        a.xy2 = __builtin_fma(fsx, fdy, a.xy2);
    }
}

// ---- raw runs ---------------------------------------------------------------
template <class T, int R> struct Run {
    static constexpr int NW = (int)(sizeof(T) * R + 3) / 4;
    uint32_t x[NW];
    uint32_t y[NW];
};

// Issue the loads of one lane's run at row offset `roff` (elements).  VEC:
// aligned vector loads from the per-lane base pointers; otherwise one load
// per element from clamped columns.
template <class T, int R, bool VEC>
__device__ __forceinline__ void issue_run(const T* __restrict__ xl, const T* __restrict__ yl,
                                          int64_t roff, const int (&cidx)[R], Run<T, R>& out)
{
    if constexpr (VEC) {
        const T* px = (const T*)__builtin_assume_aligned(xl + roff, sizeof(T) * R);
        const T* py = (const T*)__builtin_assume_aligned(yl + roff, sizeof(T) * R);
        __builtin_memcpy(out.x, px, sizeof(T) * R);
        __builtin_memcpy(out.y, py, sizeof(T) * R);
    } else {
        T vx[R], vy[R];
#pragma unroll
        for (int j = 0; j < R; j++) {
            vx[j] = xl[roff + cidx[j]];
            vy[j] = yl[roff + cidx[j]];
        }
        uint32_t wx[Run<T, R>::NW] = {}, wy[Run<T, R>::NW] = {};
        __builtin_memcpy(wx, vx, sizeof(T) * R);
        __builtin_memcpy(wy, vy, sizeof(T) * R);
#pragma unroll
        for (int i = 0; i < Run<T, R>::NW; i++) { out.x[i] = wx[i]; out.y[i] = wy[i]; }
    }
}

template <int M, int R> constexpr int fast2d_depth()
{
    return 4;
}

// ---- halo exchange + first window sum ------------------------------------
// Lane-local column c (0 <= c < R own, c < 0 from lanes to the left, c >= R
// from lanes to the right).  Columns travel hop by hop through DPP wavefront
// shifts; each is added to the first window sum S (columns -LH..RH) on
// arrival, and only the 2(R-1) columns the later slides need are kept:
// keepL[c + LH] for c in [-LH, -LH + R - 2] (c < 0) and keepR[c - RH - 1]
// for c in [RH + 1, RH + R - 1] (c >= R).
template <int M, int R, int KW>
__device__ __forceinline__ void halo_window(const Col<M> (&V)[R], Col<M>& S,
                                            Col<M> (&keepL)[R > 1 ? R - 1 : 1],
                                            Col<M> (&keepR)[R > 1 ? R - 1 : 1])
{
    constexpr int LH = KW / 2;
    constexpr int RH = KW - 1 - LH;
    constexpr int NHL = (LH + R - 1) / R;
    constexpr int NHR = (RH + R - 1) / R;
    col_zero<M>(S);
#pragma unroll
    for (int c = 0; c < R; c++)
        if (c <= RH) col_add<M>(S, V[c]);
    Col<M> cur[R];
#pragma unroll
    for (int j = 0; j < R; j++) cur[j] = V[j];
#pragma unroll
    for (int h = 1; h <= NHL; h++) {
#pragma unroll
        for (int j = 0; j < R; j++) {
            if (j < h * R - LH) continue;
            cur[j] = col_dpp<true, M>(cur[j]);      // V[j] of lane t-h
            const int c = j - h * R;
            col_add<M>(S, cur[j]);
            if (c <= -LH + R - 2) keepL[c + LH] = cur[j];
        }
    }
#pragma unroll
    for (int j = 0; j < R; j++) cur[j] = V[j];
#pragma unroll
    for (int h = 1; h <= NHR; h++) {
#pragma unroll
        for (int j = 0; j < R; j++) {
            if (h * R + j > R + RH - 1) continue;
            cur[j] = col_dpp<false, M>(cur[j]);     // V[j] of lane t+h
            const int c = h * R + j;
            if (c <= RH) col_add<M>(S, cur[j]);
            if (c >= RH + 1) keepR[c - RH - 1] = cur[j];
        }
    }
}

// One tile of the fused 2-D correlation (see the file comment).  `smem` is
// this wave's LDS region of fast2d_lds_per_wave(M, R, kh) bytes.
template <int M, int R, int KW, bool VEC>
__device__ __forceinline__ void tile2d(const P2DF& g, const int tile, char* smem)
{
    using T = typename Tr<M>::T;
    constexpr int LH = KW / 2;
    constexpr int RH = KW - 1 - LH;
    constexpr int D = fast2d_depth<M, R>();
    constexpr int NW = Run<T, R>::NW;
    constexpr bool kFloat = (M == MODE_F64);
    const int lane = threadIdx.x & (kWave - 1);

    // ---- tile geometry (wave-uniform) ----
    const int tx = tile / g.tiles_y;
    const int ty = tile - tx * g.tiles_y;
    const int p0 = ty * g.TH;
    const int q0 = tx * g.Wq;
    const int ph = min(g.TH, g.OH - p0);
    const int qw = min(g.Wq, g.OW - q0);
    const int E = q0 * g.sw + g.ow;
    const int Eal = (E >= 0) ? (E / R) * R : -((-E + R - 1) / R) * R;
    const int H = g.H, W = g.W, kh = g.kh;
    const int i0 = p0 * g.sh + g.oh;                 // first marched row (may be < 0)
    const int nrows = (ph - 1) * g.sh + kh;
    const int rlo = max(i0, 0);
    const int rhi = min(i0 + nrows - 1, H - 1);
    const bool rows_inside = (i0 >= 0) && (i0 + nrows - 1 <= H - 1);
    // Alternate the march direction between vertically adjacent tiles: both
    // tiles that share a halo band then read it at the same moment (both at
    // the start or both at the end of their march), so one of them hits L2.
    const bool up = (ty & 1) != 0;
    const int i1 = i0 + nrows - 1;
    const bool fill = g.border == BORDER_FILL;
    const bool has_flags = g.flags != nullptr;

    // ---- per-lane column metadata (once per tile) ----
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
    // VEC: a lane's run is entirely inside or outside [0, W)
    const uint32_t lane_boff = VEC ? (uint32_t)((colok & 1u) ? c0 : 0) * (uint32_t)sizeof(T) : 0u;
    uint32_t omask = 0, fillb = 0;
    int qj[R];
    double ncol[R];
#pragma unroll
    for (int j = 0; j < R; j++) {
        const int qs = c0 + j - g.ow - LH;          // = q*sw when column c0+j is a centre
        int q = -1;
        if (qs >= 0) {
            q = (g.sw == 1) ? qs : qs / g.sw;
            if (q * g.sw != qs) q = -1;
        }
        omask |= (q >= q0 && q < q0 + qw) ? (1u << j) : 0u;
        qj[j] = q;
        const int clo = q * g.sw + g.ow, chi = clo + KW - 1;
        fillb |= (fill && (clo < 0 || chi >= W)) ? (1u << j) : 0u;
        ncol[j] = (double)(min(chi, W - 1) - max(clo, 0) + 1);
    }

    // ---- per-wave LDS: ring of the last k_h raw rows, zeroed, and a stash ----
    char* wbase = smem;
    uint32_t* ringx = (uint32_t*)wbase;                         // [kh][64][NW]
    uint32_t* ringy = ringx + kh * kWave * NW;
    int* ringm = (int*)(ringy + kh * kWave * NW);                // [kh][64] (float input)
    double* stash = (double*)(wbase + ((fast2d_ring_bytes(M, R, kh) + 15) & ~15));
    for (int s = 0; s < kh; s++) {
#pragma unroll
        for (int i = 0; i < NW; i++) {
            ringx[(s * kWave + lane) * NW + i] = 0u;
            ringy[(s * kWave + lane) * NW + i] = 0u;
        }
        if constexpr (kFloat) ringm[s * kWave + lane] = 0;
    }

    Col<M> V[R];
#pragma unroll
    for (int j = 0; j < R; j++) col_zero<M>(V[j]);
    float hmx = 0.f, hmy = 0.f;

    const char* __restrict__ Xb = (const char*)g.x;
    const char* __restrict__ Yb = (const char*)g.y;
    auto issue = [&](int r, Run<T, R>& out) {
        r = r < rlo ? rlo : (r > rhi ? rhi : r);
        if constexpr (VEC) {
            const size_t rb = (size_t)r * (size_t)W * sizeof(T);
            const T* px = (const T*)__builtin_assume_aligned(Xb + rb + lane_boff, sizeof(T) * R);
            const T* py = (const T*)__builtin_assume_aligned(Yb + rb + lane_boff, sizeof(T) * R);
            __builtin_memcpy(out.x, px, sizeof(T) * R);
            __builtin_memcpy(out.y, py, sizeof(T) * R);
        } else {
            const T* xr = (const T*)g.x + (size_t)r * W;
            const T* yr = (const T*)g.y + (size_t)r * W;
            T vx[R], vy[R];
#pragma unroll
            for (int j = 0; j < R; j++) { vx[j] = xr[cidx[j]]; vy[j] = yr[cidx[j]]; }
            uint32_t wx[NW] = {}, wy[NW] = {};
            __builtin_memcpy(wx, vx, sizeof(T) * R);
            __builtin_memcpy(wy, vy, sizeof(T) * R);
#pragma unroll
            for (int i = 0; i < NW; i++) { out.x[i] = wx[i]; out.y[i] = wy[i]; }
        }
    };

    Run<T, R> pf[D];
#pragma unroll
    for (int u = 0; u < D; u++) issue(up ? i1 - u : i0 + u, pf[u]);

    int slot = 0;
    int next_ready = kh - 1;
    int p = up ? p0 + ph - 1 : p0;
    const int pstep = up ? -1 : 1;
    const int rstep = up ? -1 : 1;
    for (int base = 0; base < nrows; base += D) {
#pragma unroll
        for (int u = 0; u < D; u++) {
            const int li = base + u;
            if (li >= nrows) break;
            const int row = up ? i1 - li : i0 + li;
            // ---- current row (zero outside the array) ----
            uint32_t wx[NW], wy[NW];
#pragma unroll
            for (int i = 0; i < NW; i++) { wx[i] = pf[u].x[i]; wy[i] = pf[u].y[i]; }
            if (!rows_inside && (row < rlo || row > rhi)) {
#pragma unroll
                for (int i = 0; i < NW; i++) { wx[i] = 0u; wy[i] = 0u; }
            }
            if (edge) {
                T vx[R], vy[R];
                __builtin_memcpy(vx, wx, sizeof(T) * R);
                __builtin_memcpy(vy, wy, sizeof(T) * R);
#pragma unroll
                for (int j = 0; j < R; j++) {
                    vx[j] = ((colok >> j) & 1u) ? vx[j] : (T)0;
                    vy[j] = ((colok >> j) & 1u) ? vy[j] : (T)0;
                }
                __builtin_memcpy(wx, vx, sizeof(T) * R);
                __builtin_memcpy(wy, vy, sizeof(T) * R);
            }
            issue(row + D * rstep, pf[u]);
            // ---- leaving row from the ring (zeros for the first k_h rows) ----
            const int bw = (slot * kWave + lane) * NW;
            uint32_t ox[NW], oy[NW];
#pragma unroll
            for (int i = 0; i < NW; i++) { ox[i] = ringx[bw + i]; oy[i] = ringy[bw + i]; }
            int omiss = 0, nmiss = 0;
            if constexpr (kFloat) omiss = ringm[slot * kWave + lane];
            T ax[R], ay[R], bx[R], by[R];
            __builtin_memcpy(ax, wx, sizeof(T) * R);
            __builtin_memcpy(ay, wy, sizeof(T) * R);
            __builtin_memcpy(bx, ox, sizeof(T) * R);
            __builtin_memcpy(by, oy, sizeof(T) * R);
            if constexpr (kFloat) {
#pragma unroll
                for (int j = 0; j < R; j++) {
                    const bool m = is_missing(ax[j], g.miss_thr) || is_missing(ay[j], g.miss_thr);
                    ax[j] = m ? 0.f : ax[j];
                    ay[j] = m ? 0.f : ay[j];
                    nmiss |= m ? (1 << j) : 0;
                    hmx = fmaxf(hmx, __builtin_fabsf(ax[j]));
                    hmy = fmaxf(hmy, __builtin_fabsf(ay[j]));
                }
                __builtin_memcpy(wx, ax, sizeof(T) * R);
                __builtin_memcpy(wy, ay, sizeof(T) * R);
                ringm[slot * kWave + lane] = nmiss;
            }
            // same lane, same address: the read above returns the old row
#pragma unroll
            for (int i = 0; i < NW; i++) { ringx[bw + i] = wx[i]; ringy[bw + i] = wy[i]; }
            slot = (slot + 1 == kh) ? 0 : slot + 1;
            // ---- step 2: running column sums ----
#pragma unroll
            for (int j = 0; j < R; j++) {
                if constexpr (kFloat) {
                    const double x = (double)ax[j], y = (double)ay[j];
                    const double xo = (double)bx[j], yo = (double)by[j];
                    V[j].x += x - xo;
                    V[j].y += y - yo;
                    V[j].xx = __builtin_fma(x, x, __builtin_fma(-xo, xo, V[j].xx));
                    V[j].yy = __builtin_fma(y, y, __builtin_fma(-yo, yo, V[j].yy));
                    V[j].xy = __builtin_fma(x, y, __builtin_fma(-xo, yo, V[j].xy));
                    V[j].miss += ((nmiss >> j) & 1) - ((omiss >> j) & 1);
                } else {
                    col_update_int<M>(V[j], (int)ax[j], (int)ay[j], (int)bx[j], (int)by[j]);
                }
            }
            if (li != next_ready) continue;
            next_ready += g.sh;

            // ---- step 3: window sums along the row ----
            Col<M> S, keepL[R > 1 ? R - 1 : 1], keepR[R > 1 ? R - 1 : 1];
            halo_window<M, R, KW>(V, S, keepL, keepR);
            double gx = 0.0, gy = 0.0;   // certification thresholds (float input)
            if constexpr (kFloat) {
                const double Mx = (double)fmaxf(hmx, fmaxf(__uint_as_float(dpp_from_left(__float_as_uint(hmx))),
                                                    __uint_as_float(dpp_from_right(__float_as_uint(hmx)))));
                const double My = (double)fmaxf(hmy, fmaxf(__uint_as_float(dpp_from_left(__float_as_uint(hmy))),
                                                    __uint_as_float(dpp_from_right(__float_as_uint(hmy)))));
                gx = g.cert_g * Mx * Mx;
                gy = g.cert_g * My * My;
            }
            // wave-uniform row quantities
            const int rlo_w = p * g.sh + g.oh, rhi_w = rlo_w + kh - 1;
            const bool row_b = fill && (rlo_w < 0 || rhi_w >= H);
            const int rl = max(rlo_w, 0), rh_ = min(rhi_w, H - 1);
            const double nrow = (double)(rh_ - rl + 1);
            const size_t orow = (size_t)p * (size_t)g.OW;
            float* __restrict__ crow = g.c + orow;

            uint32_t pending = 0;
            float cvals[R];
            uint8_t fls[R];
#pragma unroll
            for (int j = 0; j < R; j++) {
                if (j > 0) {
                    const int ca = j + RH, cs = j - 1 - LH;
                    const Col<M>& va = ca < R ? V[ca] : keepR[ca - RH - 1];
                    const Col<M>& vs = cs < 0 ? keepL[cs + LH] : V[cs];
                    col_add<M>(S, va);
                    col_sub<M>(S, vs);
                }
                // ---- step 4: epilogue (branch-free; rare cases deferred) ----
                const bool fb = row_b || ((fillb >> j) & 1u);
                const double dn = nrow * ncol[j];
                uint8_t fl = 0;
                float cv;
                if constexpr (kFloat) {
                    const double N = __builtin_fma(dn, S.xy, -(S.x * S.y));
                    const double Vx = __builtin_fma(dn, S.xx, -(S.x * S.x));
                    const double Vy = __builtin_fma(dn, S.yy, -(S.y * S.y));
                    const bool cert = (Vx > gx) && (Vy > gy);
                    // FP64 rsqrt estimate (relative error ~2^-23) and one Newton step
                    const double q = Vx * Vy;
                    double r = __builtin_amdgcn_rsq(q);
                    const double e = __builtin_fma(q * r, r, -1.0);
                    r = r * __builtin_fma(e, -0.5, 1.0);
                    cv = clamp_unit(N * r);
                    const bool bad = fb || (S.miss > 0);
                    if (bad) {
                        fl = fb ? FL_BORDER : FL_MISSING;
                        cv = g.invalid;
                    }
                    const bool pend = !bad && (!cert || (g.force & 1));
                    pending |= pend ? (1u << j) : 0u;
                } else {
                    const double sx = (double)S.x, sy = (double)S.y;
                    const double N = __builtin_fma(0.5 * dn, (double)S.xy2, -(sx * sy));
                    const double Vx = __builtin_fma(dn, (double)S.xx, -(sx * sx));
                    const double Vy = __builtin_fma(dn, (double)S.yy, -(sy * sy));
                    // certified RN32 estimate: v_rsq_f64 (relative error well
                    // below 2^-20) and one Newton step leave < 2^-38; outputs
                    // whose 29 discarded mantissa bits lie within 2^15 of the
                    // midpoint pattern take the exact decision
                    const double q = Vx * Vy;
                    double r = __builtin_amdgcn_rsq(q);
                    const double e = __builtin_fma(q * r, r, -1.0);
                    r = r * __builtin_fma(e, -0.5, 1.0);
                    const double a = __builtin_fabs(N) * r;
                    const uint32_t t = (uint32_t)__double_as_longlong(a) & 0x1FFFFFFFu;
                    const bool amb = (t - (0x10000000u - (1u << 15))) <= (2u << 15);
                    const float f = (float)a;
                    cv = (N < 0.0) ? -f : f;
                    const bool bad = fb || (q == 0.0);   // Vx, Vy >= 0 are exact integers
                    if (bad) {
                        fl = fb ? FL_BORDER : (uint8_t)((Vx == 0.0 ? FL_ZVAR_X : 0) | (Vy == 0.0 ? FL_ZVAR_Y : 0));
                        cv = g.invalid;
                    }
                    const bool pend = !bad && (amb || (g.force & 1));
                    pending |= pend ? (1u << j) : 0u;
                    if (pend) {
                        double* st = stash + (size_t)(j * kWave + lane) * 3;
                        st[0] = N; st[1] = Vx; st[2] = Vy;
                    }
                }
                cvals[j] = cv;
                fls[j] = fl;
            }
            // rare path: exact decisions / two-pass recomputation
            if (pending) {
                for (int j = 0; j < R; j++) {
                    if (!((pending >> j) & 1u)) continue;
                    if constexpr (kFloat) {
                        const int64_t clo = (int64_t)qj[j] * g.sw + g.ow;
                        const int64_t cl = clo < 0 ? 0 : clo;
                        const int64_t ch = clo + KW - 1 > W - 1 ? W - 1 : clo + KW - 1;
                        float cvr = 0.f;
                        const uint8_t f2 = twopass_window((const float*)g.x, (const float*)g.y,
                                                          (int64_t)W, 1, rl, rh_, cl, ch, 0, 0, &cvr);
#pragma unroll
                        for (int jj = 0; jj < R; jj++)
                            if (jj == j) { fls[jj] = f2; cvals[jj] = f2 ? g.invalid : cvr; }
                    } else {
                        const double* st = stash + (size_t)(j * kWave + lane) * 3;
                        const double N = st[0];
                        // any estimate far inside half an ulp selects the right bucket
                        const double a = __builtin_fabs(N) / __builtin_sqrt(st[1] * st[2]);
                        float f = rn32_exact_decide(__builtin_fabs(N), st[1], st[2], a);
                        f = N < 0.0 ? -f : f;
#pragma unroll
                        for (int jj = 0; jj < R; jj++)
                            if (jj == j) cvals[jj] = f;
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < R; j++) {
                if ((omask >> j) & 1u) {
                    crow[(uint32_t)qj[j]] = cvals[j];
                    if (has_flags) g.flags[orow + (uint32_t)qj[j]] = fls[j];
                }
            }
            p += pstep;
        }
    }
}

// Occupancy target: three waves per SIMD for the integer kernels with R = 4
// (their register and LDS footprints allow it), two otherwise.
template <int M, int R> constexpr int fast2d_min_waves() { return (M != MODE_F64 && R == 4) ? 3 : 2; }

template <int M, int R, int KW, bool VEC>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(fast2d_min_waves<M, R>(), 8))) corr2d_fast_kernel(P2DF g)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int wv = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    const int tile = xcd_remap(blockIdx.x, gridDim.x) * wpb + wv;
    if (tile >= g.n_tiles) return;
    tile2d<M, R, KW, VEC>(g, tile, smem + (size_t)wv * fast2d_lds_per_wave(M, R, g.kh));
}

}  // namespace swc
