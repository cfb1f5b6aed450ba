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

#include <type_traits>

#include "swc_device.hpp"
#include "swc_internal.h"

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
    int vst;                   // bit 0: whole-vector stores of c, bit 1: of flags
};

// Which (mode, R, KW) combinations have a compiled register-resident kernel.
__host__ __device__ inline bool fast2d_supported(int mode, int R, int KW)
{
    if (mode != MODE_U8 && mode != MODE_U16 && mode != MODE_F64) return false;
    if (R == 4) return KW == 3 || KW == 5 || KW == 7 || KW == 9 || KW == 15 || KW == 31;
    if (R == 8) return KW == 7 || KW == 15 || KW == 31;
    return false;
}

// LDS bytes per wave: the raw-row ring (k_h rows of x and y as read; the
// missing positions of a float row are found again when it leaves).
__host__ __device__ constexpr int fast2d_ring_bytes(int mode, int R, int kh)
{
    return kh * kWave * 4 * (2 * (((mode == MODE_U8 ? 1 : (mode == MODE_U16 ? 2 : 4)) * R + 3) / 4));
}
// Windows that reach more than two lanes to either side (k_w/2 > 2R) take
// their sums along the row from prefix sums over the wave's columns, kept in
// a per-wave LDS row of R (64 + 1) entries per channel.  (Each output then
// costs two LDS entries read and one written, which the LDS bandwidth of a
// CU makes dearer than the hop-by-hop exchange up to two hops.)
__host__ __device__ constexpr bool fast2d_prefix(int R, int kw)
{
    return kw / 2 > 2 * R || kw - 1 - kw / 2 > 2 * R;
}
__host__ __device__ constexpr int fast2d_col_bytes(int mode)
{
    return mode == MODE_U8 ? 20 : (mode == MODE_U16 ? 32 : 48);
}
__host__ __device__ constexpr int fast2d_prefix_entries(int R) { return R * (kWave + 1); }
__host__ __device__ constexpr int fast2d_prefix_bytes(int mode, int R, int kw)
{
    return fast2d_prefix(R, kw) ? ((fast2d_col_bytes(mode) * fast2d_prefix_entries(R) + 15) & ~15)
                                : 0;
}
// Wide windows: the tile code reads the row leaving the window a second time
// (it is k_h rows behind the entering one, mostly an Infinity Cache hit)
// instead of parking k_h rows in LDS, where a ring above 24 KB per wave
// (taking k_h = k_w) would hold the resident waves per CU below six; so do
// windows whose prefix row and ring together would pass 16 KB per wave (the
// integer kernels keep three waves per SIMD, which that would not allow).
// Vector row loads only (the leaving row is read like the entering one).
__host__ __device__ constexpr bool fast2d_reread(int mode, int R, int KW, bool vec)
{
    return vec && (fast2d_ring_bytes(mode, R, KW) > 24 * 1024 ||
                   (fast2d_prefix(R, KW) &&
                    fast2d_ring_bytes(mode, R, KW) + fast2d_prefix_bytes(mode, R, KW) > 16 * 1024));
}
__host__ __device__ inline int fast2d_ring_region(int mode, int R, int kh, int kw, bool vec)
{
    return fast2d_reread(mode, R, kw, vec) ? 0 : ((fast2d_ring_bytes(mode, R, kh) + 15) & ~15);
}
__host__ __device__ inline int fast2d_lds_per_wave(int mode, int R, int kh, int kw, bool vec)
{
    return fast2d_ring_region(mode, R, kh, kw, vec) + fast2d_prefix_bytes(mode, R, kw);
}

// Certification factor (float input) of the sums of a tile that marches
// th_ext input rows: chain = operations on any partial sum (2 per marched
// row, then the sums along the row), nterms bounds the elements a partial
// sum holds.  The prefix form sums every column of the wave (in-lane
// totals and prefixes, a six-step scan, one difference).
__host__ inline double fast2d_cert(int mode, int R, int kh, int kw, double th_ext)
{
    if (fast2d_prefix(R, kw))
        return cert_factor(mode, (double)kh * kw, 2.0 * th_ext + 2.0 * R + 10.0,
                           (double)(kh + 1) * (kWave * R + 1));
    return cert_factor(mode, (double)kh * kw, 2.0 * th_ext + 2.0 * kw + 2.0 * R + 2.0,
                       (double)(kh + 1) * (kw + 1));
}

// Output columns per tile when outputs are lane-aligned (unit column step,
// centred windows): whole lanes of halo on each side, so every output lane
// holds R outputs and stores them as vectors.
__host__ __device__ inline int fast2d_wq_aligned(int R, int kw)
{
    const int lh = kw / 2, rh = kw - 1 - lh;
    const int h = ((lh > rh ? lh : rh) + R - 1) / R;
    return (kWave - 2 * h) * R;
}

// Buffer descriptor word 3 for raw (untyped) buffer access on gfx9-family
// GPUs; an access whose offset is at or beyond the record count is dropped
// (stores) or returns zero (loads).
constexpr int kBufWord3 = 0x00020000;
constexpr uint32_t kOffNone = 0x80000000u;   // offset that is always out of range

// Launch the kernel for (R, KW, vec), or with occ != nullptr only report how
// many of its workgroups (wpb waves, smem bytes of LDS) fit on one CU.
hipError_t launch_fast2d_modeu8(const P2DF& g, int R, int KW, bool vec, int grid, int wpb,
                                size_t smem, hipStream_t s, int* occ = nullptr);
hipError_t launch_fast2d_modeu16(const P2DF& g, int R, int KW, bool vec, int grid, int wpb,
                                 size_t smem, hipStream_t s, int* occ = nullptr);
hipError_t launch_fast2d_modef64(const P2DF& g, int R, int KW, bool vec, int grid, int wpb,
                                 size_t smem, hipStream_t s, int* occ = nullptr);

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

// a + (b of lane t-1) (LEFT) or a + (b of lane t+1), with 0 taken beyond the
// wave's ends: one DPP-modified add.  The two wait states a DPP source needs
// after its VALU write are inserted here (the compiler does not see inside).
template <bool LEFT> __device__ __forceinline__ uint32_t add_shifted(uint32_t a, uint32_t b)
{
    uint32_t r;
    if constexpr (LEFT)
        asm("s_nop 1\n\tv_add_u32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
            : "=&v"(r) : "v"(b), "v"(a));
    else
        asm("s_nop 1\n\tv_add_u32_dpp %0, %1, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
            : "=&v"(r) : "v"(b), "v"(a));
    return r;
}
template <bool LEFT> __device__ __forceinline__ int add_shifted(int a, int b)
{
    return (int)add_shifted<LEFT>((uint32_t)a, (uint32_t)b);
}
template <bool LEFT> __device__ __forceinline__ double add_shifted(double a, double b)
{
    return a + dpp_move<LEFT>(b);
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

// a += b of the lane to the left (LEFT) or right, channel by channel (32-bit
// integer channels as DPP-modified adds, FP64 channels moved, then added).
template <bool LEFT, int M> __device__ __forceinline__ void col_add_shifted(Col<M>& a, const Col<M>& b)
{
    a.x = add_shifted<LEFT>(a.x, b.x);
    a.y = add_shifted<LEFT>(a.y, b.y);
    a.xx = add_shifted<LEFT>(a.xx, b.xx);
    a.yy = add_shifted<LEFT>(a.yy, b.yy);
    if constexpr (M == MODE_F64) {
        a.xy = add_shifted<LEFT>(a.xy, b.xy);
        a.miss = add_shifted<LEFT>(a.miss, b.miss);
    } else {
        a.xy2 = add_shifted<LEFT>(a.xy2, b.xy2);
    }
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

#ifndef SWC_FAST2D_EPI_GROUP
#define SWC_FAST2D_EPI_GROUP 1
#endif

// Rows prefetched ahead into registers.  One is enough for the integer
// kernels, which keep three waves per SIMD to cover the latency; the float
// kernel (two waves) looks further ahead.  A variant build may override it.
template <int M, int R> constexpr int fast2d_depth()
{
#ifdef SWC_FAST2D_DEPTH
    return SWC_FAST2D_DEPTH;
#else
    return M == MODE_F64 ? 2 : 1;
#endif
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

// Window sums of one output row along the contiguous axis: S_0 from the
// halo exchange, then S_{j+1} = S_j + V[j+RH+1] - V[j-LH]; emit(j, S_j) for
// every lane column j in order.
template <int M, int R, int KW, class Emit>
__device__ __forceinline__ void hslide(const Col<M> (&V)[R], Emit&& emit)
{
    constexpr int LH = KW / 2;
    constexpr int RH = KW - 1 - LH;
    Col<M> S, keepL[R > 1 ? R - 1 : 1], keepR[R > 1 ? R - 1 : 1];
    halo_window<M, R, KW>(V, S, keepL, keepR);
#pragma unroll
    for (int j = 0; j < R; j++) {
        if (j > 0) {
            const int ca = j + RH, cs = j - 1 - LH;
            const Col<M>& va = ca < R ? V[ca] : keepR[ca - RH - 1];
            const Col<M>& vs = cs < 0 ? keepL[cs + LH] : V[cs];
            col_add<M>(S, va);
            col_sub<M>(S, vs);
        }
        emit(j, S);
    }
}

// Window sums of one output row when the halo reaches only the adjacent
// lanes (k_w/2 <= R): each lane sends its right neighbour the sums of its
// last 1..LH columns and its left neighbour the sums of its first 1..RH
// columns (DPP), then forms
//   outputs 0..LH      from a prefix chain over its own columns plus the
//                      received left sums (and right sums once the window
//                      passes the lane's last column),
//   outputs near R-1   from a suffix chain plus the received right sums,
//   any in between     by sliding.
// Only additions are used outside the middle block, and no partial sum
// holds a column outside the output's window.
template <int M, int R, int KW>
__host__ __device__ constexpr bool hsum_one_hop()
{
    return KW / 2 <= R && KW - 1 - KW / 2 <= R && KW >= 3;
}

template <int M, int R, int KW, bool EARLY, class Emit>
__device__ __forceinline__ void hsum_onehop(const Col<M> (&V)[R], Emit&& emit)
{
    constexpr int LH = KW / 2;
    constexpr int RH = KW - 1 - LH;
    constexpr int JL = LH < R - 1 ? LH : R - 1;                   // last left-block output
    constexpr int JR = (R - 1 - RH) > (JL + 1) ? (R - 1 - RH) : (JL + 1);  // first right-block output
    // sums of this lane's last m columns (the right neighbour's Lx[m]) and
    // of its first m columns (the left neighbour's Rx[m]); each is shifted
    // across the lanes where it is added
    Col<M> Lx[LH + 1];
    Lx[1] = V[R - 1];
#pragma unroll
    for (int m = 2; m <= LH; m++) {
        Lx[m] = Lx[m - 1];
        col_add<M>(Lx[m], V[R - m]);
    }
    const Col<M>& suf = Lx[LH];
    Col<M> Rx[RH + 1];
    Rx[1] = V[0];
#pragma unroll
    for (int m = 2; m <= RH; m++) {
        Rx[m] = Rx[m - 1];
        if (m <= R) col_add<M>(Rx[m], V[m - 1]);
    }
    const Col<M>& pre = Rx[RH];
    // float input with windows up to 7 wide (EARLY): the partial sums are
    // shifted across the lanes as soon as they are formed, so the moves of
    // their FP64 channels overlap the adds that follow (measured faster
    // there; wider windows would hold too many shifted sums at once);
    // otherwise they are shifted where they are added, 32-bit channels as
    // DPP-modified adds
    constexpr bool kEarly = EARLY && (M == MODE_F64) && KW <= 7;
    Col<M> LxS[kEarly ? LH + 1 : 1], RxS[kEarly ? RH + 1 : 1];
    if constexpr (kEarly) {
#pragma unroll
        for (int m = 1; m <= LH; m++) LxS[m] = col_dpp<true, M>(Lx[m]);
#pragma unroll
        for (int m = 1; m <= RH; m++) RxS[m] = col_dpp<false, M>(Rx[m]);
    }
    // left block: own columns 0..min(j+RH, R-1)
    Col<M> last;
    {
        Col<M> P = pre;                       // V[0 .. min(RH, R) - 1]
#pragma unroll
        for (int j = 0; j <= JL; j++) {
            const int b = j + RH;
            if (b <= R - 1) col_add<M>(P, V[b]);
            Col<M> S = P;
            if constexpr (kEarly) {
                if (j < LH) col_add<M>(S, LxS[LH - j]);
                if (b > R - 1) col_add<M>(S, RxS[b - R + 1]);
            } else {
                if (j < LH) col_add_shifted<true, M>(S, Lx[LH - j]);
                if (b > R - 1) col_add_shifted<false, M>(S, Rx[b - R + 1]);
            }
            emit(j, S);
            if (j == JL) last = S;
        }
    }
    // middle block: windows strictly inside the lane
#pragma unroll
    for (int j = JL + 1; j < JR; j++) {
        col_add<M>(last, V[j + RH]);
        col_sub<M>(last, V[j - 1 - LH]);
        emit(j, last);
    }
    // right block: own columns j-LH .. R-1, descending
    if constexpr (JR <= R - 1) {
        Col<M> Q = suf;                       // V[R-LH .. R-1]
#pragma unroll
        for (int j = R - 1; j >= JR; j--) {
            const int a = j - LH;
            if (a < R - LH) col_add<M>(Q, V[a]);
            Col<M> S = Q;
            const int mr = j + RH - (R - 1);
            if (mr > 0) {
                if constexpr (kEarly) col_add<M>(S, RxS[mr]);
                else col_add_shifted<false, M>(S, Rx[mr]);
            }
            emit(j, S);
        }
    }
}

// One-hop window sums when no window reaches both neighbours (k_w/2 + 1 + k_w/2
// <= R: the outputs near the lane's left edge read only the left neighbour,
// those near its right edge only the right one): the left half of the
// outputs is formed first with the left neighbour's suffix sums, then the
// right half with the right neighbour's prefix sums, so only one side's
// partial sums are held at a time (fewer registers at R = 8).
template <int M, int R, int KW>
__host__ __device__ constexpr bool hsum_two_phase()
{
    return KW / 2 + (KW - 1 - KW / 2) <= R - 1 && KW >= 3;
}

template <int M, int R, int KW, class Emit>
__device__ __forceinline__ void hsum_twophase(const Col<M> (&V)[R], Emit&& emit)
{
    constexpr int LH = KW / 2;
    constexpr int RH = KW - 1 - LH;
    // output j reads columns j - LH .. j + RH: outputs j < LH reach into the
    // left neighbour, outputs j > R - 1 - RH into the right one, and those
    // in between lie inside the lane
    {
        Col<M> Lx[LH + 1];               // sums of the left neighbour's last m columns
        Lx[1] = V[R - 1];
#pragma unroll
        for (int m = 2; m <= LH; m++) {
            Lx[m] = Lx[m - 1];
            col_add<M>(Lx[m], V[R - m]);
        }
        Col<M> P = V[0];                 // V[0 .. j + RH]
#pragma unroll
        for (int c = 1; c < RH; c++) col_add<M>(P, V[c]);
#pragma unroll
        for (int j = 0; j < LH; j++) {
            col_add<M>(P, V[j + RH]);
            Col<M> S = P;
            col_add_shifted<true, M>(S, Lx[LH - j]);
            emit(j, S);
        }
        // windows inside the lane: output LH reads columns 0 .. LH + RH
        // (P holds 0 .. LH - 1 + RH), the next ones slide by one column
        if constexpr (LH <= R - 1 - RH) {
            Col<M> S = P;
            col_add<M>(S, V[LH + RH]);
            emit(LH, S);
#pragma unroll
            for (int j = LH + 1; j <= R - 1 - RH; j++) {
                col_add<M>(S, V[j + RH]);
                col_sub<M>(S, V[j - 1 - LH]);
                emit(j, S);
            }
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    {
        Col<M> Rx[RH + 1];               // sums of the right neighbour's first m columns
        Rx[1] = V[0];
#pragma unroll
        for (int m = 2; m <= RH; m++) {
            Rx[m] = Rx[m - 1];
            col_add<M>(Rx[m], V[m - 1]);
        }
        Col<M> Q = V[R - 1];             // V[j - LH .. R - 1]
#pragma unroll
        for (int c = 2; c <= LH; c++) col_add<M>(Q, V[R - c]);
#pragma unroll
        for (int j = R - 1; j > R - 1 - RH; j--) {
            col_add<M>(Q, V[j - LH]);
            Col<M> S = Q;
            col_add_shifted<false, M>(S, Rx[j + RH - (R - 1)]);
            emit(j, S);
        }
    }
}

// Lanes a window sum of lane t reads: the columns -LH .. R-1+RH relative to
// the lane's first column lie in lanes t - reach_l .. t + reach_r (the
// one-hop form and the multi-hop slide reach the same lanes).
template <int R, int KW> __host__ __device__ constexpr int reach_l() { return (KW / 2 + R - 1) / R; }
template <int R, int KW> __host__ __device__ constexpr int reach_r()
{
    return (KW - 1 - KW / 2 + R - 1) / R;
}

// Max of a non-negative per-lane value over lanes t - reach_l .. t + reach_r
// (each step widens the covered range by one lane; lanes past the wave's ends
// contribute zero).
template <int R, int KW> __device__ __forceinline__ float reach_max(float v)
{
    float ml = v, mr = v;
#pragma unroll
    for (int h = 0; h < reach_l<R, KW>(); h++)
        ml = fmaxf(ml, __uint_as_float(dpp_from_left(__float_as_uint(ml))));
#pragma unroll
    for (int h = 0; h < reach_r<R, KW>(); h++)
        mr = fmaxf(mr, __uint_as_float(dpp_from_right(__float_as_uint(mr))));
    return fmaxf(ml, mr);
}

// Every channel of a Col at once (F(field, field of b) for each field).
template <int M, class F> __device__ __forceinline__ void col_each(Col<M>& a, const Col<M>& b, F&& f)
{
    f(a.x, b.x); f(a.y, b.y); f(a.xx, b.xx); f(a.yy, b.yy);
    if constexpr (M == MODE_F64) { f(a.xy, b.xy); f(a.miss, b.miss); }
    else f(a.xy2, b.xy2);
}

// ---- two-hop windows --------------------------------------------------------
// A word of the lane `h` lanes to the left (h > 0) or right (h < 0), through
// the LDS crossbar (ds_bpermute, one instruction whatever the distance).
// Lanes whose source lies beyond the wave's ends get a wrapped-around word;
// the callers use it only in halo lanes, which store no output.
template <int H, class V> __device__ __forceinline__ V lane_from(V v)
{
    static_assert(sizeof(V) % 4 == 0, "32-bit multiples only");
    constexpr int NW = sizeof(V) / 4;
    const int lane = threadIdx.x & (kWave - 1);
    const int addr = ((lane - H) & (kWave - 1)) << 2;
    uint32_t w[NW];
    __builtin_memcpy(w, &v, sizeof(V));
#pragma unroll
    for (int i = 0; i < NW; i++) w[i] = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)w[i]);
    V r;
    __builtin_memcpy(&r, w, sizeof(V));
    return r;
}
template <int H, int M> __device__ __forceinline__ Col<M> col_from(const Col<M>& a)
{
    Col<M> r = a;
    col_each<M>(r, a, [](auto& d, const auto& v) __attribute__((always_inline)) { d = lane_from<H>(v); });
    return r;
}

// Window sums of one output row when the window reaches exactly two lanes
// to a side (R <= k_w/2 - (R-1) and k_w/2 <= 2R, likewise to the right): every
// output's window holds the whole adjacent lanes and a part of the next ones.
// Output j = (suffix of lane t-2) + T(t-1) + T(t) + T(t+1) + (prefix of lane
// t+2): the lane totals of the neighbours move one hop by DPP, the partial
// sums two hops through the LDS crossbar (one instruction per word instead
// of two DPP moves).  Additions only; no partial sum holds a column outside
// the output's window.
template <int M, int R, int KW>
__host__ __device__ constexpr bool hsum_two_hop()
{
    return KW / 2 - (R - 1) >= R && KW / 2 - R <= R - 1 &&
           (KW - 1 - KW / 2) - (R - 1) >= R && (KW - 1 - KW / 2) - R <= R - 1 &&
           (KW / 2 > R || KW - 1 - KW / 2 > R);
}

template <int M, int R, int KW, class Emit>
__device__ __forceinline__ void hsum_twohop(const Col<M> (&V)[R], Emit&& emit)
{
    constexpr int LH = KW / 2;
    constexpr int RH = KW - 1 - LH;
    constexpr int MS = LH - R;        // columns of lane t-2 in output 0's window
    constexpr int MP = RH - R;        // columns of lane t+2 in output R-1's window
    auto add = [](Col<M>& d, const Col<M>& v) __attribute__((always_inline)) {
        col_each<M>(d, v, [](auto& a, const auto& b) __attribute__((always_inline)) { a = a + b; });
    };
    // own suffix sums (last m columns) and prefix sums (first m columns)
    Col<M> Suf[MS > 0 ? MS : 1], Pre[MP > 0 ? MP : 1];
    if constexpr (MS > 0) {
        Suf[0] = V[R - 1];
#pragma unroll
        for (int m = 1; m < MS; m++) { Suf[m] = Suf[m - 1]; add(Suf[m], V[R - 1 - m]); }
    }
    if constexpr (MP > 0) {
        Pre[0] = V[0];
#pragma unroll
        for (int m = 1; m < MP; m++) { Pre[m] = Pre[m - 1]; add(Pre[m], V[m]); }
    }
    // the partial sums leave first (their round trip is the longest)
    Col<M> L2[MS > 0 ? MS : 1], R2[MP > 0 ? MP : 1];
#pragma unroll
    for (int m = 0; m < MS; m++) L2[m] = col_from<2, M>(Suf[m]);
#pragma unroll
    for (int m = 0; m < MP; m++) R2[m] = col_from<-2, M>(Pre[m]);
    Col<M> T = V[0];
#pragma unroll
    for (int c = 1; c < R; c++) add(T, V[c]);
    Col<M> C = col_dpp<true, M>(T);            // T of lane t-1
    add(C, T);
    add(C, col_dpp<false, M>(T));              // + T of lane t+1
#pragma unroll
    for (int j = 0; j < R; j++) {
        Col<M> S = C;
        const int ml = MS - j;                 // columns of lane t-2: LH - j - R
        const int mr = j + 1 + MP - R;         // columns of lane t+2: RH - (R-1-j) - R
        if (ml > 0) add(S, L2[ml - 1]);
        if (mr > 0) add(S, R2[mr - 1]);
        emit(j, S);
    }
}

// ---- prefix form for wide windows ----------------------------------------
// 32-bit integer channels wrap modulo 2^32 here: a prefix over the wave's
// columns may pass 2^31, the window sums themselves do not, so their
// differences are exact.
__device__ __forceinline__ int wrap_add(int a, int b) { return (int)((uint32_t)a + (uint32_t)b); }
__device__ __forceinline__ int wrap_sub(int a, int b) { return (int)((uint32_t)a - (uint32_t)b); }
__device__ __forceinline__ uint32_t wrap_add(uint32_t a, uint32_t b) { return a + b; }
__device__ __forceinline__ uint32_t wrap_sub(uint32_t a, uint32_t b) { return a - b; }
__device__ __forceinline__ double wrap_add(double a, double b) { return a + b; }
__device__ __forceinline__ double wrap_sub(double a, double b) { return a - b; }

// One step of the wavefront scan on every channel: a += a of the lane the
// DPP control names (zero where it names none).
template <int CTRL, int RMASK, bool BC, int M> __device__ __forceinline__ void col_scan_step(Col<M>& a)
{
    col_each<M>(a, a, [](auto& d, const auto& v) __attribute__((always_inline)) {
        d = wrap_add(d, dppv<CTRL, RMASK, BC>(v));
    });
}

// Entry of prefix column c = R*l + i (0 <= i < R, 0 <= l <= 64) in the LDS
// row: blocks of 65 entries by i, so the 64 lanes of a wave touch 64
// consecutive entries of every channel array.
__device__ __forceinline__ int prefix_entry(int i, int l) { return i * (kWave + 1) + l; }

// The row holds one array per channel, fast2d_prefix_entries(R) entries
// each, in field order.
template <int M, int R, class F>
__device__ __forceinline__ void col_lds_each(char* base, int e, Col<M>& a, F&& f)
{
    constexpr int NE = fast2d_prefix_entries(R);
    int off = 0;
    col_each<M>(a, a, [&](auto& d, const auto&) __attribute__((always_inline)) {
        using FT = std::remove_reference_t<decltype(d)>;
        f(d, (FT*)(base + off) + e);
        off += (int)sizeof(FT) * NE;
    });
}

// Window sums of one output row when the window reaches more than two lanes
// to a side: P[c] = sum of the wave's columns left of column c, from the lane's
// column total, a DPP wavefront scan of the totals and the in-lane prefix;
// the lanes write P of their columns (lane 63 also P[64 R]) to the LDS row,
// and output j of lane t is P[R t + j + RH + 1] - P[R t + j - LH].  Outputs
// whose window passes the wave's ends (halo lanes, never stored) read
// clamped entries.  `prow`: this wave's LDS row.
template <int M, int R, int KW, class Emit>
__device__ __forceinline__ void hsum_prefix(const Col<M> (&V)[R], Emit&& emit, char* prow)
{
    static_assert(sizeof(Col<M>) == fast2d_col_bytes(M), "channel layout");
    constexpr int LH = KW / 2;
    constexpr int RH = KW - 1 - LH;
    const int lane = threadIdx.x & (kWave - 1);
    Col<M> T = V[0];
#pragma unroll
    for (int j = 1; j < R; j++)
        col_each<M>(T, V[j], [](auto& d, const auto& v) __attribute__((always_inline)) { d = wrap_add(d, v); });
    Col<M> I = T;
    col_scan_step<0x111, 0xf, true>(I);     // row_shr:1
    col_scan_step<0x112, 0xf, true>(I);     // row_shr:2
    col_scan_step<0x114, 0xf, true>(I);     // row_shr:4
    col_scan_step<0x118, 0xf, true>(I);     // row_shr:8
    col_scan_step<0x142, 0xa, false>(I);    // row_bcast:15 -> rows 1, 3
    col_scan_step<0x143, 0xc, false>(I);    // row_bcast:31 -> rows 2, 3
    Col<M> P = col_dpp<true, M>(I);         // columns of the lanes to the left
#pragma unroll
    for (int j = 0; j < R; j++) {
        if (j > 0)
            col_each<M>(P, V[j - 1], [](auto& d, const auto& v) __attribute__((always_inline)) { d = wrap_add(d, v); });
        col_lds_each<M, R>(prow, prefix_entry(j, lane), P,
                           [](auto& d, auto* q) __attribute__((always_inline)) { *q = d; });
    }
    if (lane == kWave - 1)
        col_lds_each<M, R>(prow, prefix_entry(0, kWave), I,
                           [](auto& d, auto* q) __attribute__((always_inline)) { *q = d; });
    wave_lds_sync();
    // float input (two waves per SIMD, registers to spare): every read is
    // issued before the first difference is needed, so the LDS latency is
    // paid once per row; integer input (three waves per SIMD) reads output
    // by output
    constexpr int NB = (M == MODE_F64) ? R : 1;
#pragma unroll
    for (int j0 = 0; j0 < R; j0 += NB) {
        Col<M> A[NB], S[NB];
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int j = j0 + b;
            // left end: column R t + j - LH; right end + 1: R t + j + RH + 1
            const int dl = j - LH, dr = j + RH + 1;
            const int il = ((dl % R) + R) % R, ir = dr % R;
            const int tl = lane + (dl - il) / R, tr = lane + (dr - ir) / R;
            const int el = tl < 0 ? prefix_entry(0, 0) : prefix_entry(il, tl);
            const int er = (tr > kWave || (tr == kWave && ir != 0)) ? prefix_entry(0, kWave)
                                                                     : prefix_entry(ir, tr);
            col_lds_each<M, R>(prow, el, A[b], [](auto& d, auto* q) __attribute__((always_inline)) { d = *q; });
            col_lds_each<M, R>(prow, er, S[b], [](auto& d, auto* q) __attribute__((always_inline)) { d = *q; });
        }
#pragma unroll
        for (int b = 0; b < NB; b++) {
            col_each<M>(S[b], A[b], [](auto& d, const auto& v) __attribute__((always_inline)) { d = wrap_sub(d, v); });
            emit(j0 + b, S[b]);
        }
    }
    // the next row's writes must not pass this row's reads of other lanes
    wave_lds_sync();
}

// Window sums of one output row, whichever form fits the window width
// (EARLY: see hsum_onehop; it also selects the two-hop form, which single
// launches use; prow: the LDS row of the prefix form).
template <int M, int R, int KW, bool EARLY, class Emit>
__device__ __forceinline__ void hsum_row(const Col<M> (&V)[R], Emit&& emit, char* prow)
{
    if constexpr (hsum_two_phase<M, R, KW>())
        hsum_twophase<M, R, KW>(V, emit);
    else if constexpr (hsum_one_hop<M, R, KW>())
        hsum_onehop<M, R, KW, EARLY>(V, emit);
    else if constexpr (fast2d_prefix(R, KW))
        hsum_prefix<M, R, KW>(V, emit, prow);
    else if constexpr (M == MODE_F64 && EARLY && hsum_two_hop<M, R, KW>())
        hsum_twohop<M, R, KW>(V, emit);      // (single launches of float input: the integer
                                             // kernels' 168 VGPRs and the batch kernel's two
                                             // rows of prefetch spill with it)
    else
        hslide<M, R, KW>(V, emit);
}

typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));
typedef uint32_t v2u32 __attribute__((ext_vector_type(2)));

// NW consecutive 32-bit words at byte offset `off` of a raw buffer.
template <int NW>
__device__ __forceinline__ void buf_load_words(__amdgpu_buffer_rsrc_t rs, uint32_t off, uint32_t* w)
{
    if constexpr (NW == 1) {
        w[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
    } else if constexpr (NW == 2) {
        const v2u32 v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
        w[0] = v.x; w[1] = v.y;
    } else {
        static_assert(NW % 4 == 0, "1, 2 or a multiple of 4 words");
#pragma unroll
        for (int i = 0; i < NW; i += 4) {
            const v4u32 v = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 4u * i, 0, 0);
            w[i] = v.x; w[i + 1] = v.y; w[i + 2] = v.z; w[i + 3] = v.w;
        }
    }
}


// Returns v unchanged but hides it from the optimiser, so that values derived
// from per-lane constants are recomputed where they are used instead of being
// hoisted out of the row loop (where they would only occupy registers).
template <class T> __device__ __forceinline__ T opaque(T v)
{
    asm volatile("" : "+v"(v));
    return v;
}

template <bool B> struct BoolTag {
    static constexpr bool value = B;
};
template <int V> struct IntTag {
    static constexpr int value = V;
};

// Correctly rounded float32 of N / sqrt(q), q = Vx Vy, from exact integers
// (q > 0): FP64 rsqrt estimate and one Newton step (relative error < 2^-38);
// `amb` is set when the 29 discarded mantissa bits lie within 2^15 of the
// rounding midpoint, where only the exact decision is trustworthy.
__device__ __forceinline__ float rn32_fast(double N, double q, bool& amb)
{
    const double a = newton_ratio(N, q);
    const uint32_t lo = (uint32_t)__double_as_longlong(a) & 0x1FFFFFFFu;
    amb = (lo - (0x10000000u - (1u << 15))) <= (2u << 15);
    return (float)a;
}

// One tile of the fused 2-D correlation (see the file comment).  `smem` is
// this wave's LDS region of fast2d_lds_per_wave(M, R, kh) bytes.  `tile` is
// wave-uniform.
// SINGLE: a launch of its own, one tile per wave.  A persistent caller
// (SINGLE false) sets the waves' priorities itself, and the float exchange
// shifts its sums where they are added, which needs fewer registers (its
// kernel holds the code of every window width in one register allocation).
template <int M, int R, int KW, bool VEC, bool SINGLE = true>
__device__ __forceinline__ void tile2d(const P2DF& g, const int tile, char* smem)
{
    using T = typename Tr<M>::T;
    constexpr int LH = KW / 2;
    // Rows prefetched ahead.  When the leaving row is read too (two loads
    // per row in flight): float input looks two rows ahead, except where the
    // two-hop exchange holds its partial sums (single launches, k_w = 15 at
    // R = 4), which leaves registers for one; integer input one.
    constexpr bool kTwoHop = M == MODE_F64 && SINGLE && hsum_two_hop<M, R, KW>();
    constexpr int D = fast2d_reread(M, R, KW, VEC) ? ((M == MODE_F64 && !kTwoHop) ? 2 : 1)
                                                   : fast2d_depth<M, R>();
    constexpr int NW = Run<T, R>::NW;
    constexpr bool kFloat = (M == MODE_F64);
    constexpr uint32_t kFull = (1u << R) - 1u;
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
    // every output column of the tile has its whole window inside [0, W)
    const bool cols_inside = (E >= 0) && ((q0 + qw - 1) * g.sw + g.ow + KW - 1 <= W - 1);
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
    // VEC: integer rows have W a multiple of R (a run is wholly inside or
    // outside [0, W)); a float run crossing W reads zeros past it (raw buffer
    // loads are range-checked per dword)
    // per column: byte offset of its output in the output row (kOffNone when
    // the column is not an output of this tile), clipped column count
    // (packed 8 bits each), FILL-border bit
    uint32_t omask = 0, fillb = 0;
    uint32_t qoff[R];
    uint32_t ncolp[(R + 3) / 4] = {};
#pragma unroll
    for (int j = 0; j < R; j++) {
        const int qs = c0 + j - g.ow - LH;          // = q*sw when column c0+j is a centre
        int q = -1;
        if (qs >= 0) {
            q = (g.sw == 1) ? qs : qs / g.sw;
            if (q * g.sw != qs) q = -1;
        }
        const bool out = q >= q0 && q < q0 + qw;
        omask |= out ? (1u << j) : 0u;
        qoff[j] = out ? (uint32_t)q * 4u : kOffNone;
        const int clo = q * g.sw + g.ow, chi = clo + KW - 1;
        fillb |= (fill && (clo < 0 || chi >= W)) ? (1u << j) : 0u;
        ncolp[j / 4] |= (uint32_t)(min(chi, W - 1) - max(clo, 0) + 1) << (8 * (j % 4));
    }
    // lane-aligned outputs (unit column step, centred windows, every lane
    // either full or empty): each lane stores its R results as vectors
    const bool lane_aligned = __builtin_amdgcn_ballot_w64(omask != 0u && omask != kFull) == 0;
    const bool tile_vec = (g.vst & 1) && lane_aligned;
    const uint32_t voff = omask ? (uint32_t)c0 * 4u : kOffNone;    // c0 = first output column
    const uint32_t vfoff = omask ? (uint32_t)c0 : kOffNone;

    // ---- per-wave LDS: ring of the last k_h raw rows, zeroed ----
    // rings of 4+ words per lane are word-major ([kh][NW][64]: 32-bit accesses
    // of a wave hit 64 consecutive words, no bank conflicts); 1-2 words per
    // lane stay lane-major ([kh][64][NW], read and written as one access)
    constexpr bool kWordMajor = NW >= 4;
    auto ring_at = [&](int slot, int i) __attribute__((always_inline)) {
        return kWordMajor ? (slot * NW + i) * kWave + lane : (slot * kWave + lane) * NW + i;
    };
    constexpr bool kReread = fast2d_reread(M, R, KW, VEC);
    uint32_t* ringx = (uint32_t*)smem;
    // LDS row of the prefix form (wide windows), after the ring
    char* const prow = smem + (kReread ? 0 : ((fast2d_ring_bytes(M, R, kh) + 15) & ~15));
    uint32_t* ringy = ringx + kh * kWave * NW;
    if constexpr (!kReread) {
        for (int s = 0; s < kh; s++) {
#pragma unroll
            for (int i = 0; i < NW; i++) {
                ringx[ring_at(s, i)] = 0u;
                ringy[ring_at(s, i)] = 0u;
            }
        }
    }

    Col<M> V[R];
#pragma unroll
    for (int j = 0; j < R; j++) col_zero<M>(V[j]);
    float hmx = 0.f, hmy = 0.f;

    const char* __restrict__ Xb = (const char*)g.x;
    const char* __restrict__ Yb = (const char*)g.y;
    // VEC: raw buffer loads over one input row; rows outside the array have a
    // zero record count and lanes outside it an out-of-range offset, so both
    // read zeros
    const uint32_t lane_vo = (colok & 1u) ? (uint32_t)c0 * (uint32_t)sizeof(T) : kOffNone;
    auto issue = [&](int r, Run<T, R>& out) {
        if constexpr (VEC) {
            const bool rin = r >= 0 && r < H;
            const size_t rb = (size_t)(rin ? r : 0) * (size_t)W * sizeof(T);
            const int nrec = rin ? W * (int)sizeof(T) : 0;
            const __amdgpu_buffer_rsrc_t bx =
                __builtin_amdgcn_make_buffer_rsrc((void*)(Xb + rb), (short)0, nrec, kBufWord3);
            const __amdgpu_buffer_rsrc_t by =
                __builtin_amdgcn_make_buffer_rsrc((void*)(Yb + rb), (short)0, nrec, kBufWord3);
            buf_load_words<NW>(bx, lane_vo, out.x);
            buf_load_words<NW>(by, lane_vo, out.y);
        } else {
            r = r < rlo ? rlo : (r > rhi ? rhi : r);
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

    // ---- step 3-4 for output row p: window sums along the row, epilogue,
    //      store.  IN:
    //        2: the output row's window rows and every output column of the
    //           tile are interior (full windows, no border handling);
    //        1: lane-aligned outputs (every lane's columns all outputs or
    //           none) whose windows take their own clipped counts and
    //           FILL-border bits: the tiles along the array's edges then
    //           cost about as much as interior ones, so none of them holds
    //           up the end of the launch;
    //        0: the general case. ----
    auto out_row = [&](int p, auto in_tag, auto fl_tag, float (&cvals)[R],
                       uint32_t (&flw)[(R + 3) / 4]) {
        constexpr int IN = decltype(in_tag)::value;
        constexpr bool FL = decltype(fl_tag)::value;   // a flag map is written
        const int rlo_w = p * g.sh + g.oh, rhi_w = rlo_w + kh - 1;
        const bool row_b = fill && (rlo_w < 0 || rhi_w >= H);
        uint32_t fillb_r = 0, ncolp_r[(R + 3) / 4] = {};
        if constexpr (IN != 2) {
            fillb_r = opaque(fillb);
#pragma unroll
            for (int i = 0; i < (R + 3) / 4; i++) ncolp_r[i] = opaque(ncolp[i]);
        }
        auto ncol_r = [&](int j) -> int { return (int)((ncolp_r[j / 4] >> (8 * (j % 4))) & 0xFFu); };
        const int rl = max(rlo_w, 0), rh_ = min(rhi_w, H - 1);
        const int nrow_i = rh_ - rl + 1;
        const double nrow = (double)nrow_i;
        const double dn_in = (double)(kh * KW);
        double gx = 0.0, gy = 0.0;   // certification thresholds (float input)
        if constexpr (kFloat) {
            // M covers every column any window sum of this lane touched:
            // the lanes t - reach_l .. t + reach_r (the prefix form sums
            // every column of the wave: the wave's maximum)
            double Mx, My;
            if constexpr (fast2d_prefix(R, KW)) {
                Mx = (double)wave_max(hmx);
                My = (double)wave_max(hmy);
            } else {
                Mx = (double)reach_max<R, KW>(hmx);
                My = (double)reach_max<R, KW>(hmy);
            }
            gx = g.cert_g * Mx * Mx;
            gy = g.cert_g * My * My;
        }
        // lanes with an output that needs the rare path: the compare results
        // are combined as wave masks (scalar registers).  Interior rows of
        // interior tiles skip the per-column output test (there a column that
        // is not an output lies inside the array, so it is a well-formed
        // window that rarely needs the rare path, which tests each output
        // itself); lanes without any output are dropped once at the end.
        uint64_t pend_w = 0;
        const bool force_exact = (g.force & 1) != 0;
        const uint64_t fx_w = force_exact ? ~0ull : 0ull;
        auto out_w = [&](int j) -> uint64_t {
            if constexpr (IN >= 1) return ~0ull;   // lane-aligned: a lane's columns are all outputs or none
            else return __builtin_amdgcn_ballot_w64(((omask >> j) & 1u) != 0u);
        };
        // Window quantities of output j from its sums: N, Vx, Vy (exact
        // integers for integer input) and the FILL-border bit.
        auto nvv = [&](int j, const Col<M>& S, double& N, double& Vx, double& Vy, bool& fb)
            __attribute__((always_inline)) {
            double dn;
            if constexpr (IN == 2) {
                dn = dn_in;
                fb = false;
            } else if constexpr (IN == 1) {
                dn = (double)(nrow_i * ncol_r(j));
                fb = row_b | (((fillb_r >> j) & 1u) != 0u);
            } else {
                dn = nrow * (double)ncol_r(j);
                fb = row_b || ((fillb_r >> j) & 1u);
            }
            if constexpr (kFloat) {
                N = __builtin_fma(dn, S.xy, -(S.x * S.y));
                Vx = __builtin_fma(dn, S.xx, -(S.x * S.x));
                Vy = __builtin_fma(dn, S.yy, -(S.y * S.y));
            } else {
                const double sx = (double)S.x, sy = (double)S.y;
                N = __builtin_fma(0.5 * dn, (double)S.xy2, -(sx * sy));
                Vx = __builtin_fma(dn, (double)S.xx, -(sx * sx));
                Vy = __builtin_fma(dn, (double)S.yy, -(sy * sy));
            }
        };
        hsum_row<M, R, KW, SINGLE>(V, [&](int j, const Col<M>& S) __attribute__((always_inline)) {
            double N, Vx, Vy;
            bool fb;
            nvv(j, S, N, Vx, Vy, fb);
            const double q = Vx * Vy;
            float cv;
            bool bad;
            if constexpr (kFloat) {
                const bool cert = (Vx > gx) & (Vy > gy);
                // FP64 rsqrt estimate and one Newton step
                cv = clamp_unit(newton_ratio(N, q));
                bad = fb | (S.miss > 0);
                // (one ballot of the per-lane test: measured faster than
                // combining the masks for float input)
                const bool pnd = (!bad) & ((!cert) | force_exact) & (((omask >> j) & 1u) != 0);
                pend_w |= __builtin_amdgcn_ballot_w64(pnd);
                if (FL) {
                    const uint32_t fl = fb ? FL_BORDER : (S.miss > 0 ? FL_MISSING : 0);
                    flw[j / 4] |= fl << (8 * (j % 4));
                }
            } else {
                bool amb;
                cv = rn32_fast(N, q, amb);
                // Vx, Vy >= 0 are exact integers: a zero product is a zero variance
                bad = fb | (q == 0.0);
                pend_w |= (__builtin_amdgcn_ballot_w64(amb) | fx_w) &
                          ~__builtin_amdgcn_ballot_w64(bad) & out_w(j);
                if (FL) {
                    const uint32_t fl = fb ? FL_BORDER
                                           : ((Vx == 0.0 ? FL_ZVAR_X : 0u) | (Vy == 0.0 ? FL_ZVAR_Y : 0u));
                    flw[j / 4] |= fl << (8 * (j % 4));
                }
            }
            // opaque: keep the estimate unconditional (straight-line code
            // instead of a branch around it for the rare invalid lanes)
            const float cvo = opaque(cv);
            cvals[j] = bad ? g.invalid : cvo;
            // epilogues are scheduled in groups of SWC_FAST2D_EPI_GROUP
            // outputs: interleaving more of them hides more latency but
            // costs registers
            if ((j % SWC_FAST2D_EPI_GROUP) == SWC_FAST2D_EPI_GROUP - 1)
                __builtin_amdgcn_sched_barrier(0);
        }, prow);
        // rare path: exact decisions (integer input) / two-pass recomputation
        // (float input) for the outputs whose fast result is not certified.
        // The window sums are recomputed (the slide is deterministic), so the
        // common path keeps nothing for them.
        if (pend_w & __builtin_amdgcn_ballot_w64(omask != 0u)) {
            hsum_row<M, R, KW, SINGLE>(V, [&](int j, const Col<M>& S) __attribute__((always_inline)) {
                double N, Vx, Vy;
                bool fb;
                nvv(j, S, N, Vx, Vy, fb);
                const double q = Vx * Vy;
                if constexpr (kFloat) {
                    const bool pend = !fb && S.miss <= 0 &&
                                      (!((Vx > gx) && (Vy > gy)) || force_exact) &&
                                      ((omask >> j) & 1u);
                    if (pend) {
                        const int clo = (int)(opaque(qoff[j]) >> 2) * g.sw + g.ow;
                        const int64_t cl = max(clo, 0);
                        const int64_t ch = min(clo + KW - 1, W - 1);
                        float cvr = 0.f;
                        const uint8_t f2 = twopass_window((const float*)g.x, (const float*)g.y,
                                                          (int64_t)W, 1, rl, rh_, cl, ch, 0, 0, &cvr);
                        flw[j / 4] = (flw[j / 4] & ~(0xFFu << (8 * (j % 4)))) |
                                     ((uint32_t)f2 << (8 * (j % 4)));
                        cvals[j] = f2 ? g.invalid : cvr;
                    }
                } else {
                    bool amb;
                    (void)rn32_fast(N, q, amb);
                    const bool pend = !fb && q != 0.0 && (amb || force_exact) && ((omask >> j) & 1u);
                    if (pend) {
                        const double aN = __builtin_fabs(N);
                        // any estimate far inside half an ulp selects the right bucket
                        const float f = rn32_exact_decide(aN, Vx, Vy, aN / __builtin_sqrt(q));
                        cvals[j] = N < 0.0 ? -f : f;
                    }
                }
            }, prow);
        }
    };

    // ---- stores of one step: buffer stores over an output row; columns
    //      that are not outputs of this tile carry an out-of-range offset,
    //      and a step without an output row stores through a zero-length
    //      record.  Every step issues the same stores (flag stores only when
    //      a flag map is written), so the loads still in flight can be
    //      counted exactly when the next row is waited for (stores share
    //      that counter). ----
    auto store_row = [&](bool emit, int64_t orow_p, auto svec_tag, auto fl_tag,
                         const float (&cvals)[R], const uint32_t (&flw)[(R + 3) / 4]) {
        constexpr bool SVEC = decltype(svec_tag)::value;
        constexpr bool FL = decltype(fl_tag)::value;   // flag stores (none without a map)
        const int64_t orow = emit ? orow_p : 0;
        const __amdgpu_buffer_rsrc_t rc =
            __builtin_amdgcn_make_buffer_rsrc(g.c + orow, (short)0, emit ? g.OW * 4 : 0, kBufWord3);
        if constexpr (SVEC) {
#pragma unroll
            for (int j = 0; j < R; j += 4) {
                v4u32 v = {__float_as_uint(cvals[j]), __float_as_uint(cvals[j + 1]),
                           __float_as_uint(cvals[j + 2]), __float_as_uint(cvals[j + 3])};
                __builtin_amdgcn_raw_buffer_store_b128(v, rc, voff + 4u * j, 0, 0);
            }
        } else {
#pragma unroll
            for (int j = 0; j < R; j++)
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(cvals[j]), rc, qoff[j], 0, 0);
        }
        if constexpr (FL) {
            const __amdgpu_buffer_rsrc_t rf = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(g.flags + orow), (short)0, emit ? g.OW : 0, kBufWord3);
            if constexpr (SVEC) {
#pragma unroll
                for (int i = 0; i < R / 4; i++)
                    __builtin_amdgcn_raw_buffer_store_b32(flw[i], rf, vfoff + 4u * i, 0, 0);
            } else {
#pragma unroll
                for (int j = 0; j < R; j++) {
                    const uint32_t qo = opaque(qoff[j]);
                    __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(flw[j / 4] >> (8 * (j % 4))), rf,
                                                         qo == kOffNone ? kOffNone : qo >> 2, 0, 0);
                }
            }
        }
    };

    // Prefetch ring of D rows in registers.  The first pass of the loop
    // (base = -D) only fills it, so that every load is issued from the same
    // place in the loop body and the compiler can count the loads still in
    // flight when it waits for the oldest one.
    // ---- the march down the tile ----
    auto march = [&](auto svec_tag, auto fl_tag) {
        Run<T, R> pf[D];
        Run<T, R> pfo[kReread ? D : 1];     // leaving rows (second read)
        // rows are issued in order, one per step: keep the next row's index
        // and byte offset in scalar registers instead of recomputing them
        const int64_t rowbytes = (int64_t)W * (int64_t)sizeof(T);
        int r_next = up ? i1 : i0;
        int64_t off_next = (int64_t)r_next * rowbytes;
        const int64_t off_step = up ? -rowbytes : rowbytes;
        // march index of the next row issued: the row leaving the window
        // with it is k_h rows behind, or none during the first k_h rows
        int li_next = 0;
        auto issue_next = [&](Run<T, R>& out, Run<T, R>& outo) {
            if constexpr (VEC) {
                const bool rin = (unsigned)r_next < (unsigned)H;
                const int nrec = rin ? (int)rowbytes : 0;
                const int64_t o = rin ? off_next : 0;
                const __amdgpu_buffer_rsrc_t bx =
                    __builtin_amdgcn_make_buffer_rsrc((void*)(Xb + o), (short)0, nrec, kBufWord3);
                const __amdgpu_buffer_rsrc_t by =
                    __builtin_amdgcn_make_buffer_rsrc((void*)(Yb + o), (short)0, nrec, kBufWord3);
                buf_load_words<NW>(bx, lane_vo, out.x);
                buf_load_words<NW>(by, lane_vo, out.y);
                if constexpr (kReread) {
                    const int ro = up ? r_next + kh : r_next - kh;
                    const bool oin = li_next >= kh && (unsigned)ro < (unsigned)H;
                    const int nreco = oin ? (int)rowbytes : 0;
                    const int64_t oo = oin ? off_next - (int64_t)kh * off_step : 0;
                    const __amdgpu_buffer_rsrc_t bxo =
                        __builtin_amdgcn_make_buffer_rsrc((void*)(Xb + oo), (short)0, nreco, kBufWord3);
                    const __amdgpu_buffer_rsrc_t byo =
                        __builtin_amdgcn_make_buffer_rsrc((void*)(Yb + oo), (short)0, nreco, kBufWord3);
                    buf_load_words<NW>(bxo, lane_vo, outo.x);
                    buf_load_words<NW>(byo, lane_vo, outo.y);
                }
            } else {
                issue(r_next, out);
            }
            r_next += up ? -1 : 1;
            off_next += off_step;
            li_next++;
        };
        // output rows are emitted in order: element offset of row p
        int64_t orow = (int64_t)(up ? p0 + ph - 1 : p0) * (int64_t)g.OW;
        const int64_t orow_step = up ? -(int64_t)g.OW : (int64_t)g.OW;
        int slot = 0;
        bool dirty = false;      // wave-uniform: a missing value has entered the tile
        int next_ready = kh - 1;
        int p = up ? p0 + ph - 1 : p0;
        const int pstep = up ? -1 : 1;
        // Waves sharing a SIMD are issued oldest first, so with equal tiles
        // the oldest would finish long before the others and leave its SIMD
        // short of waves at the end.  Each wave instead lowers its priority
        // as its march progresses (3 for the first quarter of the rows down
        // to 0 for the last), so that waves behind catch up and the waves of
        // a SIMD finish together.  (A persistent caller sets priorities itself.)
        const int q1 = nrows >> 2, q2 = nrows >> 1, q3 = nrows - q1;
        if constexpr (SINGLE) __builtin_amdgcn_s_setprio(3);
        for (int base = -D; base < nrows; base += D) {
            // (the first step of each D-row group at or past a quarter mark)
            if constexpr (SINGLE) {
                if ((unsigned)(q1 - base) < (unsigned)D) __builtin_amdgcn_s_setprio(2);
                if ((unsigned)(q2 - base) < (unsigned)D) __builtin_amdgcn_s_setprio(1);
                if ((unsigned)(q3 - base) < (unsigned)D) __builtin_amdgcn_s_setprio(0);
            }
#pragma unroll
            for (int u = 0; u < D; u++) {
                const int li = base + u;
                if (li >= nrows) break;
                const int row = up ? i1 - li : i0 + li;
                if (li >= 0) {
                // ---- current row (zero outside the array) ----
                uint32_t wx[NW], wy[NW];
#pragma unroll
                for (int i = 0; i < NW; i++) { wx[i] = pf[u].x[i]; wy[i] = pf[u].y[i]; }
                if (!VEC && !rows_inside && (row < rlo || row > rhi)) {
#pragma unroll
                    for (int i = 0; i < NW; i++) { wx[i] = 0u; wy[i] = 0u; }
                }
                if (!VEC && edge) {
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
                // ---- leaving row from the ring (zeros for the first k_h rows),
                //      or from its second read ----
                uint32_t ox[NW], oy[NW];
#pragma unroll
                for (int i = 0; i < NW; i++) {
                    if constexpr (kReread) {
                        ox[i] = pfo[u].x[i];
                        oy[i] = pfo[u].y[i];
                    } else {
                        ox[i] = ringx[ring_at(slot, i)];
                        oy[i] = ringy[ring_at(slot, i)];
                    }
                }
                if constexpr (!kReread) {
                    // the entering row as read (same lane, same address: the
                    // reads above return the old row)
#pragma unroll
                    for (int i = 0; i < NW; i++) {
                        ringx[ring_at(slot, i)] = wx[i];
                        ringy[ring_at(slot, i)] = wy[i];
                    }
                    slot = (slot + 1 == kh) ? 0 : slot + 1;
                }
                int omiss = 0, nmiss = 0;
                T ax[R], ay[R], bx[R], by[R];
                __builtin_memcpy(ax, wx, sizeof(T) * R);
                __builtin_memcpy(ay, wy, sizeof(T) * R);
                __builtin_memcpy(bx, ox, sizeof(T) * R);
                __builtin_memcpy(by, oy, sizeof(T) * R);
                if constexpr (kFloat) {
                    // positions outside the array read zero and are never
                    // missing, whatever the threshold
                    const bool row_in = (unsigned)row < (unsigned)H;
                    // the leaving row's missing positions, found again (rows
                    // outside the array, and the first k_h rows of the march,
                    // read zero and are never missing); none while no missing
                    // value has entered the tile
                    if (kReread || dirty) {
                        const int rowo = up ? row + kh : row - kh;
                        const bool rowo_in = li >= kh && (unsigned)rowo < (unsigned)H;
#pragma unroll
                        for (int j = 0; j < R; j++) {
                            const bool inb = rowo_in && ((colok >> j) & 1u);
                            const bool m = inb && (is_missing(bx[j], g.miss_thr) ||
                                                   is_missing(by[j], g.miss_thr));
                            bx[j] = m ? 0.f : bx[j];
                            by[j] = m ? 0.f : by[j];
                            omiss |= m ? (1 << j) : 0;
                        }
                    }
#pragma unroll
                    for (int j = 0; j < R; j++) {
                        const bool inb = row_in && ((colok >> j) & 1u);
                        const bool m = inb && (is_missing(ax[j], g.miss_thr) ||
                                               is_missing(ay[j], g.miss_thr));
                        ax[j] = m ? 0.f : ax[j];
                        ay[j] = m ? 0.f : ay[j];
                        nmiss |= m ? (1 << j) : 0;
                        hmx = fmaxf(hmx, __builtin_fabsf(ax[j]));
                        hmy = fmaxf(hmy, __builtin_fabsf(ay[j]));
                    }
                    if constexpr (!kReread) dirty = dirty || __builtin_amdgcn_ballot_w64(nmiss != 0) != 0;
                }
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
                }
                // refill this prefetch slot only now: its registers are free, and
                // the rows in the other slots stay in flight
                issue_next(pf[u], pfo[kReread ? u : 0]);
                const bool emit = li >= 0 && li == next_ready;
                float cvals[R];
                uint32_t flw[(R + 3) / 4];
#pragma unroll
                for (int j = 0; j < R; j++) cvals[j] = 0.f;
#pragma unroll
                for (int i = 0; i < (R + 3) / 4; i++) flw[i] = 0u;
                if (emit) {
                    next_ready += g.sh;
                    const int rw = p * g.sh + g.oh;
                    const bool row_in = rw >= 0 && rw + kh - 1 <= H - 1;
                    if (row_in && cols_inside)
                        out_row(p, IntTag<2>{}, fl_tag, cvals, flw);
                    else if (lane_aligned)
                        out_row(p, IntTag<1>{}, fl_tag, cvals, flw);
                    else
                        out_row(p, IntTag<0>{}, fl_tag, cvals, flw);
                }
                store_row(emit, orow, svec_tag, fl_tag, cvals, flw);
                if (emit) {
                    p += pstep;
                    orow += orow_step;
                }
            }
        }
    };
    // whole-vector stores for the tile (every output lane full, flags
    // either absent or aligned as well).  Separate code for launches with
    // and without a flag map (without, no flag is formed or stored).
    if (has_flags) {
        if (tile_vec && (g.vst & 2))
            march(BoolTag<true>{}, BoolTag<true>{});
        else
            march(BoolTag<false>{}, BoolTag<true>{});
    } else {
        if (tile_vec)
            march(BoolTag<true>{}, BoolTag<false>{});
        else
            march(BoolTag<false>{}, BoolTag<false>{});
    }
}


// Occupancy target (waves per SIMD the register allocation must allow):
// three for the integer kernels with R = 4, two otherwise.  The macros let a
// variant build try other targets.
#ifndef SWC_FAST2D_WAVES_INT4
#define SWC_FAST2D_WAVES_INT4 3
#endif
#ifndef SWC_FAST2D_WAVES_OTHER
#define SWC_FAST2D_WAVES_OTHER 2
#endif
template <int M, int R> constexpr int fast2d_min_waves()
{
    return (M != MODE_F64 && R == 4) ? SWC_FAST2D_WAVES_INT4 : SWC_FAST2D_WAVES_OTHER;
}

template <int M, int R, int KW, bool VEC>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(fast2d_min_waves<M, R>(), 8))) corr2d_fast_kernel(P2DF g)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int wpb = blockDim.x / kWave;
    // the wave index is uniform across the wave; say so, so that all tile
    // geometry lives in scalar registers
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int tile = xcd_remap(blockIdx.x, gridDim.x) * wpb + wv;
    if (tile >= g.n_tiles) return;
    tile2d<M, R, KW, VEC>(g, tile, smem + (size_t)wv * fast2d_lds_per_wave(M, R, g.kh, KW, VEC));
}

}  // namespace swc
