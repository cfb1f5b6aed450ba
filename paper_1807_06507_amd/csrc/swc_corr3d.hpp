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

#include <stddef.h>
#include <type_traits>

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

// `cube`: 0 general step; 1 the specialised step (k_y == k_x, unit y step,
// TY == 2, vector loads, planes below 2^30 bytes); 2 the specialised step in
// halves (also centred windows, unit x step, Wq = 120, tiles of 4 rows).
// The host checks those conditions.
hipError_t launch_fast3d_modeu8(const P3D& g, int KW, int TY, bool vec, int cube, int grid,
                                int wpb, hipStream_t s);
hipError_t launch_fast3d_modeu16(const P3D& g, int KW, int TY, bool vec, int cube, int grid,
                                 int wpb, hipStream_t s);
hipError_t launch_fast3d_modef64(const P3D& g, int KW, int TY, bool vec, int cube, int grid,
                                 int wpb, hipStream_t s);

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

// a += col_delta(a, b, ao, bo) without forming the difference first: the
// product channels take the entering and leaving products as two FMAs into
// the sum (two roundings, as the difference and its addition have).
template <int M, class T>
__device__ __forceinline__ void col_accum_delta(Col<M>& s, T a, T b, T ao, T bo)
{
    if constexpr (M == MODE_F64) {
        const double x = (double)a, y = (double)b, xo = (double)ao, yo = (double)bo;
        s.x += x - xo;
        s.y += y - yo;
        s.xx = __builtin_fma(x, x, __builtin_fma(-xo, xo, s.xx));
        s.yy = __builtin_fma(y, y, __builtin_fma(-yo, yo, s.yy));
        s.xy = __builtin_fma(x, y, __builtin_fma(-xo, yo, s.xy));
    } else {
        col_update_int<M>(s, (int)a, (int)b, (int)ao, (int)bo);
    }
}

// LDS bytes per wave for the running 3-D sums (TY rows x R columns).
template <int M, int TY> __host__ __device__ constexpr int tile3d_lds_per_wave(int R)
{
    return TY * R * (int)sizeof(Col<M>) * kWave;
}
// The specialised step keeps the missing counts in registers: float slots
// hold the five FP64 sums only (10 words), so 8 waves' sums fit one CU.
template <int M> __host__ __device__ constexpr int cube_slot_words()
{
    return M == MODE_F64 ? 10 : (int)(sizeof(Col<M>) / 4);
}
template <int M> __host__ __device__ constexpr int cube_lds_per_wave(int R)
{
    return 2 * R * cube_slot_words<M>() * 4 * kWave;
}
__host__ __device__ inline int cube_lds_bytes(int mode, int R)
{
    return mode == MODE_U8 ? cube_lds_per_wave<MODE_U8>(R)
                           : (mode == MODE_U16 ? cube_lds_per_wave<MODE_U16>(R)
                                               : cube_lds_per_wave<MODE_F64>(R));
}
__host__ __device__ inline int tile3d_lds_bytes(int mode, int TY, int R)
{
    const int cb = mode == MODE_U8 ? (int)sizeof(Col<MODE_U8>)
                                   : (mode == MODE_U16 ? (int)sizeof(Col<MODE_U16>)
                                                       : (int)sizeof(Col<MODE_F64>));
    return TY * R * cb * kWave;
}

// Running 3-D sums of one (row, column) slot in LDS, one 32-bit word per
// lane per component, components strided by 64 lanes (conflict-free).
template <int M> struct S3Slot {
    uint32_t* base;   // word 0 of this slot for lane 0
    static constexpr int NDW = (int)(sizeof(Col<M>) / 4);
    __device__ __forceinline__ void add(int lane, const Col<M>& v) const
    {
        uint32_t w[NDW], a[NDW];
        __builtin_memcpy(a, &v, sizeof(Col<M>));
#pragma unroll
        for (int i = 0; i < NDW; i++) w[i] = base[i * kWave + lane];
        Col<M> cur;
        __builtin_memcpy(&cur, w, sizeof(Col<M>));
        col_add<M>(cur, v);
        __builtin_memcpy(w, &cur, sizeof(Col<M>));
#pragma unroll
        for (int i = 0; i < NDW; i++) base[i * kWave + lane] = w[i];
        (void)a;
    }
    __device__ __forceinline__ Col<M> get(int lane) const
    {
        uint32_t w[NDW];
#pragma unroll
        for (int i = 0; i < NDW; i++) w[i] = base[i * kWave + lane];
        Col<M> cur;
        __builtin_memcpy(&cur, w, sizeof(Col<M>));
        return cur;
    }
    __device__ __forceinline__ void zero(int lane) const
    {
#pragma unroll
        for (int i = 0; i < NDW; i++) base[i * kWave + lane] = 0u;
    }
};

// Fields of Col<M> one at a time: F-th field by reference, its 32-bit word
// offset in the struct, and the field count (the missing count is last).
template <int M> constexpr int col_nfields() { return M == MODE_F64 ? 6 : 5; }
template <int M, int F> __device__ __forceinline__ auto& col_field(Col<M>& c)
{
    if constexpr (M == MODE_F64) {
        if constexpr (F == 0) return c.x;
        else if constexpr (F == 1) return c.y;
        else if constexpr (F == 2) return c.xx;
        else if constexpr (F == 3) return c.yy;
        else if constexpr (F == 4) return c.xy;
        else return c.miss;
    } else {
        if constexpr (F == 0) return c.x;
        else if constexpr (F == 1) return c.y;
        else if constexpr (F == 2) return c.xx;
        else if constexpr (F == 3) return c.yy;
        else return c.xy2;
    }
}
template <int M, int F> constexpr int col_field_word()
{
    if constexpr (M == MODE_F64) return F < 5 ? 2 * F : 10;
    else if constexpr (M == MODE_U16) return F < 2 ? F : 2 + 2 * (F - 2);
    else return F;
}
static_assert(offsetof(Col<MODE_F64>, miss) == 40 && offsetof(Col<MODE_F64>, xy) == 32, "layout");
static_assert(offsetof(Col<MODE_U16>, xx) == 8 && offsetof(Col<MODE_U16>, xy2) == 24, "layout");
static_assert(offsetof(Col<MODE_U8>, xy2) == 16, "layout");

// Window sums of one channel along x when the halo reaches only the adjacent
// lanes (k_x/2 <= R): the left neighbour's suffix sums and the right
// neighbour's prefix sums arrive by DPP; each output adds its in-lane part
// (a prefix or a suffix of the lane's columns) and the received sums.
// Additions only; no partial sum holds a column outside the output's window.
template <class V, int R, int KW>
__device__ __forceinline__ void hsum_scalar(const V (&v)[R], V (&out)[R])
{
    constexpr int LH = KW / 2;
    constexpr int RH = KW - 1 - LH;
    static_assert(LH <= R && RH <= R, "one-hop windows only");
    V P[R + 1], Q[R + 1];     // P[m]: first m columns; Q[m]: last m columns
    P[1] = v[0];
    Q[1] = v[R - 1];
#pragma unroll
    for (int m = 2; m <= R; m++) {
        P[m] = P[m - 1] + v[m - 1];
        Q[m] = Q[m - 1] + v[R - m];
    }
    V Lx[LH + 1], Rx[RH + 1];
#pragma unroll
    for (int m = 1; m <= LH; m++) Lx[m] = dpp_move<true>(Q[m]);
#pragma unroll
    for (int m = 1; m <= RH; m++) Rx[m] = dpp_move<false>(P[m]);
#pragma unroll
    for (int j = 0; j < R; j++) {
        const int a = j - LH > 0 ? j - LH : 0;
        const int b = j + RH < R - 1 ? j + RH : R - 1;
        static_assert(KW + 1 >= R, "in-lane part is a prefix or a suffix");
        V acc = (a == 0) ? P[b + 1] : Q[R - a];
        if (j < LH) acc = acc + Lx[LH - j];
        if (j + RH > R - 1) acc = acc + Rx[j + RH - (R - 1)];
        out[j] = acc;
    }
}

// One row of entering and leaving raw values per lane.
template <class T, int R> struct Row3 {
    static constexpr int NW = Run<T, R>::NW;
    uint32_t xi[NW], yi[NW], xo[NW], yo[NW];
};

template <int M, int R, int KW, int TY, bool VEC>
__device__ __forceinline__ void tile3d(const P3D& g, const int tile, char* smem)
{
    using T = typename Tr<M>::T;
    constexpr int LH = KW / 2;
    constexpr int NW = Run<T, R>::NW;
    constexpr bool kFloat = (M == MODE_F64);
    const int lane = threadIdx.x & (kWave - 1);

    // ---- tile geometry (wave-uniform): y fastest, then x, then z ----
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
    // VEC (W a multiple of R): a lane's run is entirely inside or outside [0, W)
    const uint32_t lane_vo = (colok & 1u) ? (uint32_t)c0 * (uint32_t)sizeof(T) : kOffNone;
    uint32_t omask = 0, fillb = 0;
    int qj[R];
    int ncol[R];
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
        ncol[j] = min(chi, W - 1) - max(clo, 0) + 1;
    }

    // ---- rows of the y-windows of this tile's output rows ----
    const int ys = py0 * g.sy + g.oy;               // first window row
    const int nyr = (pyn - 1) * g.sy + g.ky;        // window rows in the tile
    // ---- planes ----
    const int zs = pz0 * g.sz + g.oz;               // first window plane
    const int nz = (pzn - 1) * g.sz + g.kz;

    const char* __restrict__ Xb = (const char*)g.x;
    const char* __restrict__ Yb = (const char*)g.y;
    const int64_t rowbytes = (int64_t)W * (int64_t)sizeof(T);
    const int64_t planebytes = (int64_t)H * rowbytes;

    // raw buffer over row r of plane z (zero records outside the volume)
    auto rsrc = [&](const char* A, int z, int r) {
        const bool ok = (unsigned)z < (unsigned)D && (unsigned)r < (unsigned)H;
        const int64_t o = ok ? (int64_t)z * planebytes + (int64_t)r * rowbytes : 0;
        return __builtin_amdgcn_make_buffer_rsrc((void*)(A + o), (short)0, ok ? (int)rowbytes : 0,
                                                 kBufWord3);
    };
    auto load_row = [&](int zin, int zout, int r, Row3<T, R>& out) __attribute__((always_inline)) {
        if constexpr (VEC) {
            buf_load_words<NW>(rsrc(Xb, zin, r), lane_vo, out.xi);
            buf_load_words<NW>(rsrc(Yb, zin, r), lane_vo, out.yi);
            buf_load_words<NW>(rsrc(Xb, zout, r), lane_vo, out.xo);
            buf_load_words<NW>(rsrc(Yb, zout, r), lane_vo, out.yo);
        } else {
            auto one = [&](int z, int rr, uint32_t (&wx)[NW], uint32_t (&wy)[NW]) {
                const bool ok = (unsigned)z < (unsigned)D && (unsigned)rr < (unsigned)H;
                const size_t rb = ok ? ((size_t)z * (size_t)H + (size_t)rr) * (size_t)W : 0;
                const T* xr = (const T*)g.x + rb;
                const T* yr = (const T*)g.y + rb;
                T vx[R], vy[R];
#pragma unroll
                for (int j = 0; j < R; j++) {
                    const bool v = ok && ((colok >> j) & 1u);
                    vx[j] = v ? xr[cidx[j]] : (T)0;
                    vy[j] = v ? yr[cidx[j]] : (T)0;
                }
                uint32_t tx_[NW] = {}, ty_[NW] = {};
                __builtin_memcpy(tx_, vx, sizeof(T) * R);
                __builtin_memcpy(ty_, vy, sizeof(T) * R);
#pragma unroll
                for (int i = 0; i < NW; i++) { wx[i] = tx_[i]; wy[i] = ty_[i]; }
            };
            one(zin, r, out.xi, out.yi);
            one(zout, r, out.xo, out.yo);
        }
    };

    // running 3-D sums in LDS: slot (t, j) at word offset (t*R + j) * NDW * 64
    constexpr int NDW = S3Slot<M>::NDW;
    uint32_t* s3w = (uint32_t*)smem;
    auto slot = [&](int t, int j) { return S3Slot<M>{s3w + (t * R + j) * NDW * kWave}; };
#pragma unroll
    for (int t = 0; t < TY; t++)
#pragma unroll
        for (int j = 0; j < R; j++) slot(t, j).zero(lane);
    float hmx = 0.f, hmy = 0.f;

    int next_ready = g.kz - 1;
    int pz = pz0;
    for (int li = 0; li < nz; li++) {
        const int zin = zs + li;
        const int zout = li >= g.kz ? zin - g.kz : -1;     // -1: nothing leaves yet
        // ---- y-window sums of the z-difference field (registers) ----
        Col<M> VY[TY][R];
#pragma unroll
        for (int t = 0; t < TY; t++)
#pragma unroll
            for (int j = 0; j < R; j++) col_zero<M>(VY[t][j]);
        auto consume = [&](int r, Row3<T, R>& rw) __attribute__((always_inline)) {
            T ax[R], ay[R], bx[R], by[R];
            __builtin_memcpy(ax, rw.xi, sizeof(T) * R);
            __builtin_memcpy(ay, rw.yi, sizeof(T) * R);
            __builtin_memcpy(bx, rw.xo, sizeof(T) * R);
            __builtin_memcpy(by, rw.yo, sizeof(T) * R);
            int m[R], mo[R];
#pragma unroll
            for (int j = 0; j < R; j++) { m[j] = 0; mo[j] = 0; }
            if constexpr (kFloat) {
                // missing values are rare: test the row's extremes first
                float lo = ax[0], hi = ax[0];
                bool nan = false;
#pragma unroll
                for (int j = 0; j < R; j++) {
                    lo = fminf(lo, fminf(fminf(ax[j], ay[j]), fminf(bx[j], by[j])));
                    hi = fmaxf(hi, fmaxf(fmaxf(ax[j], ay[j]), fmaxf(bx[j], by[j])));
                    nan = nan | (ax[j] != ax[j]) | (ay[j] != ay[j]) | (bx[j] != bx[j]) |
                          (by[j] != by[j]);
                }
                const bool clean = (lo > g.miss_thr) & (hi < __builtin_inff()) & !nan;
                if (__builtin_amdgcn_ballot_w64(!clean)) {
                    // positions outside the volume read zero and are never missing
                    const bool row_in = (unsigned)(ys + r) < (unsigned)H;
                    const bool in_i = row_in && (unsigned)zin < (unsigned)D;
                    const bool in_o = row_in && (unsigned)zout < (unsigned)D;
#pragma unroll
                    for (int j = 0; j < R; j++) {
                        const bool col_in = (colok >> j) & 1u;
                        m[j] = (in_i && col_in &&
                                (is_missing(ax[j], g.miss_thr) | is_missing(ay[j], g.miss_thr))) ? 1 : 0;
                        mo[j] = (in_o && col_in &&
                                 (is_missing(bx[j], g.miss_thr) | is_missing(by[j], g.miss_thr))) ? 1 : 0;
                        ax[j] = m[j] ? 0.f : ax[j];
                        ay[j] = m[j] ? 0.f : ay[j];
                        bx[j] = mo[j] ? 0.f : bx[j];
                        by[j] = mo[j] ? 0.f : by[j];
                    }
                }
#pragma unroll
                for (int j = 0; j < R; j++) {
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
        };
        // rows in pairs: the next row's loads are in flight while one is used
        Row3<T, R> A, B;
        load_row(zin, zout, ys, A);
        for (int r = 0; r < nyr; r += 2) {
            if (r + 1 < nyr) load_row(zin, zout, ys + r + 1, B);
            consume(r, A);
            if (r + 1 >= nyr) break;
            if (r + 2 < nyr) load_row(zin, zout, ys + r + 2, A);
            consume(r + 1, B);
        }
        // ---- x-window sums, added to the running 3-D sums ----
#pragma unroll
        for (int t = 0; t < TY; t++) {
            if (t >= pyn) continue;
            static_assert(!fast2d_prefix(R, KW), "3-D x windows stay within one hop");
            hsum_row<M, R, KW, false>(VY[t], [&](int j, const Col<M>& S) __attribute__((always_inline)) {
                slot(t, j).add(lane, S);
            }, nullptr);
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
            const int ylo = (py0 + t) * g.sy + g.oy, yhi = ylo + g.ky - 1;
            const bool rowb = fill && (ylo < 0 || yhi >= H);
            const double nrow = (double)(min(yhi, H - 1) - max(ylo, 0) + 1);
            const size_t orow = ((size_t)pz * g.OH + (size_t)(py0 + t)) * (size_t)g.OW;
#pragma unroll
            for (int j = 0; j < R; j++) {
                if (!((omask >> j) & 1u)) continue;
                const Col<M> A3 = slot(t, j).get(lane);
                const bool fb = zb || rowb || ((fillb >> j) & 1u);
                const double dn = nzp * nrow * (double)ncol[j];
                uint8_t fl = 0;
                float cv = 0.f;
                if (fb) {
                    fl = FL_BORDER;
                } else if constexpr (kFloat) {
                    if (A3.miss > 0) {
                        fl = FL_MISSING;
                    } else {
                        const int64_t clo = (int64_t)qj[j] * g.sx + g.ox;
                        WinBox wb{(int64_t)H * W, (int64_t)W, max(zlo, 0), min(zhi, D - 1),
                                  max(ylo, 0), min(yhi, H - 1),
                                  max(clo, (int64_t)0), min(clo + KW - 1, (int64_t)W - 1)};
                        // certification against the per-plane thresholds
                        const double N = __builtin_fma(dn, A3.xy, -(A3.x * A3.y));
                        const double Vx = __builtin_fma(dn, A3.xx, -(A3.x * A3.x));
                        const double Vy = __builtin_fma(dn, A3.yy, -(A3.y * A3.y));
                        const bool cert = (Vx > gx) && (Vy > gy) && !(g.force & 1);
                        if (cert) {
                            cv = clamp_unit(newton_ratio(N, Vx * Vy));
                        } else {
                            fl = twopass_window((const float*)g.x, (const float*)g.y, wb.s0, wb.s1,
                                                wb.lo0, wb.hi0, wb.lo1, wb.hi1, wb.lo2, wb.hi2, &cv);
                        }
                    }
                } else {
                    const double sxv = (double)A3.x, syv = (double)A3.y;
                    const double N = __builtin_fma(0.5 * dn, (double)A3.xy2, -(sxv * syv));
                    const double Vx = __builtin_fma(dn, (double)A3.xx, -(sxv * sxv));
                    const double Vy = __builtin_fma(dn, (double)A3.yy, -(syv * syv));
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

// The step for the common shape: k_y == k_x (= KW), unit y step, TY = 2
// output rows, contiguous rows a multiple of R long (vector loads), planes
// below 2^30 bytes.  The KW + 1 window rows of a step are unrolled, so which
// output rows a row feeds is known at compile time: row 0 feeds only output
// row 0, row KW only output row 1, rows 1..KW-1 both, and their sum is formed
// once.  Each step's four planes (x and y, entering and leaving) are raw
// buffers over the whole plane (zero records outside the volume); a row is
// one offset shared by the four loads, out of range for rows and lanes
// outside the volume.  Missing values (float input) are screened on the
// entering values only: until a tile has met one, the planes leaving its
// window had none either, so the per-element masking runs only from the
// first missing value on.  The epilogue of a finished plane runs right after
// the running sum of an output is updated.
// HALF: the wave is two 32-lane halves on the same columns (120 outputs per
// row) and on vertically adjacent row pairs (the wave covers 4 output rows):
// narrow volumes waste fewer lanes on columns past the last output.  Lanes 0
// and 31 of each half are its halo; the DPP exchange between the halves only
// reaches halo lanes, whose outputs are not stored.
template <int M, int R, int KW, bool HALF>
__device__ __forceinline__ void tile3d_cube(const P3D& g, const int tile, char* smem)
{
    using T = typename Tr<M>::T;
    constexpr int TY = 2;
    constexpr int NYR = KW + 1;
    constexpr int LH = KW / 2;
    constexpr int NW = Run<T, R>::NW;
    constexpr bool kFloat = (M == MODE_F64);
    constexpr uint32_t kFar = 0x40000000u;   // >= every plane's byte size
    const int lane = threadIdx.x & (kWave - 1);

    // ---- tile geometry (wave-uniform): y fastest, then x, then z ----
    const int ty = tile % g.tiles_y;
    const int rest = tile / g.tiles_y;
    const int tx = rest % g.tiles_x;
    const int tz = rest / g.tiles_x;
    const int pz0 = tz * g.TZ;
    const int pzn = min(g.TZ, g.OD - pz0);
    // output rows of this lane: py0, py0 + 1 (per lane in HALF mode)
    const int py0 = HALF ? ty * (2 * TY) + TY * (lane >> 5) : ty * TY;
    const int pyn = min(TY, g.OH - py0);
    const int q0 = tx * g.Wq;
    const int qw = min(g.Wq, g.OW - q0);
    const int D = g.D, H = g.H, W = g.W;
    const int E = q0 * g.sx + g.ox;
    const int Eal = (E >= 0) ? (E / R) * R : -((-E + R - 1) / R) * R;
    const bool fill = g.border == BORDER_FILL;
    const bool has_flags = g.flags != nullptr;

    // ---- per-lane columns: W is a multiple of R, so a run is wholly inside
    //      or wholly outside [0, W) ----
    const int c0 = Eal + (HALF ? (lane & 31) : lane) * R;
    const uint32_t lane_vo = (c0 >= 0 && c0 < W) ? (uint32_t)c0 * (uint32_t)sizeof(T) : kFar;
    uint32_t omask = 0, fillb = 0;
    int qj[R];
    int ncol[R];
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
        ncol[j] = min(chi, W - 1) - max(clo, 0) + 1;
    }

    const int ys = py0 + g.oy;                       // first window row (unit y step)
    const int zs = pz0 * g.sz + g.oz;                // first window plane
    const int nz = (pzn - 1) * g.sz + g.kz;
    const uint32_t rowbytes = (uint32_t)W * (uint32_t)sizeof(T);
    const uint32_t planebytes = (uint32_t)H * rowbytes;
    const char* __restrict__ Xb = (const char*)g.x;
    const char* __restrict__ Yb = (const char*)g.y;
    auto prs = [&](const char* A, int z) {
        const bool ok = (unsigned)z < (unsigned)D;
        const size_t o = ok ? (size_t)z * (size_t)planebytes : 0;
        return __builtin_amdgcn_make_buffer_rsrc((void*)(A + o), (short)0,
                                                 ok ? (int)planebytes : 0, kBufWord3);
    };
    // byte offset of window row r (0..NYR-1) for this lane
    uint32_t voff[NYR];
#pragma unroll
    for (int r = 0; r < NYR; r++) {
        const int row = ys + r;
        const uint32_t ro = ((unsigned)row < (unsigned)H) ? (uint32_t)row * rowbytes : kFar;
        voff[r] = lane_vo + ro;
    }

    // running 3-D sums: LDS slot (t, j) holds the FP64 (or integer) sums,
    // lane-strided; float input keeps the missing counts in registers
    constexpr int NDW = cube_slot_words<M>();
    uint32_t* s3w = (uint32_t*)smem;
#pragma unroll
    for (int t = 0; t < TY; t++)
#pragma unroll
        for (int j = 0; j < R; j++)
#pragma unroll
            for (int i = 0; i < NDW; i++) s3w[((t * R + j) * NDW + i) * kWave + lane] = 0u;
    int s3miss[TY][R];
#pragma unroll
    for (int t = 0; t < TY; t++)
#pragma unroll
        for (int j = 0; j < R; j++) s3miss[t][j] = 0;
    float hmx = 0.f, hmy = 0.f;
    bool dirty = false;          // wave-uniform: a missing value has entered this tile

    // rows of the first (or only) row pair: the most any lane has
    const int pyn_w = HALF ? min(TY, g.OH - ty * (2 * TY)) : pyn;
    int next_ready = g.kz - 1;
    int pz = pz0;
    // One z step.  DIRTY = false: no missing value has entered the tile, so
    // the entering rows are only screened and no missing counts are carried;
    // a step whose screen finds one returns false before it has changed any
    // state but the value maxima, and is taken again with DIRTY = true.  The
    // DIRTY step first reads its rows once for the missing counts alone
    // (window sums of the entering-minus-leaving indicators, added to the
    // running counts), then once more for the masked values, so that neither
    // pass holds more registers than the clean step.
    auto zstep = [&](const int li, auto dirty_c) __attribute__((always_inline)) -> bool {
        constexpr bool DIRTY = decltype(dirty_c)::value;
        bool found = false;
        const int zin = zs + li;
        const int zout = li >= g.kz ? zin - g.kz : -1;
        const __amdgpu_buffer_rsrc_t rxi = prs(Xb, zin), ryi = prs(Yb, zin);
        const __amdgpu_buffer_rsrc_t rxo = prs(Xb, zout), ryo = prs(Yb, zout);
        Row3<T, R> rw[3];
        auto issue = [&](int r) __attribute__((always_inline)) {
            Row3<T, R>& o = rw[r % 3];
            buf_load_words<NW>(rxi, voff[r], o.xi);
            buf_load_words<NW>(ryi, voff[r], o.yi);
            buf_load_words<NW>(rxo, voff[r], o.xo);
            buf_load_words<NW>(ryo, voff[r], o.yo);
        };
        if constexpr (kFloat && DIRTY) {
            int V0m[R], MIDm[R];
#pragma unroll
            for (int r = 0; r < NYR; r++) {
                uint32_t wxi[NW], wyi[NW], wxo[NW], wyo[NW];
                buf_load_words<NW>(rxi, voff[r], wxi);
                buf_load_words<NW>(ryi, voff[r], wyi);
                buf_load_words<NW>(rxo, voff[r], wxo);
                buf_load_words<NW>(ryo, voff[r], wyo);
                T ax[R], ay[R], bx[R], by[R];
                __builtin_memcpy(ax, wxi, sizeof(T) * R);
                __builtin_memcpy(ay, wyi, sizeof(T) * R);
                __builtin_memcpy(bx, wxo, sizeof(T) * R);
                __builtin_memcpy(by, wyo, sizeof(T) * R);
                // positions outside the volume read zero and are never missing
                const bool row_in = (unsigned)(ys + r) < (unsigned)H && c0 >= 0 && c0 < W;
                const bool in_i = row_in && (unsigned)zin < (unsigned)D;
                const bool in_o = row_in && (unsigned)zout < (unsigned)D;
#pragma unroll
                for (int j = 0; j < R; j++) {
                    const int dm = ((in_i && (is_missing(ax[j], g.miss_thr) |
                                              is_missing(ay[j], g.miss_thr))) ? 1 : 0) -
                                   ((in_o && (is_missing(bx[j], g.miss_thr) |
                                              is_missing(by[j], g.miss_thr))) ? 1 : 0);
                    if (r == 0) {
                        V0m[j] = dm;
                    } else if (r == 1) {
                        MIDm[j] = dm;
                    } else if (r < KW) {
                        MIDm[j] += dm;
                    } else {
                        V0m[j] += MIDm[j];
                        MIDm[j] += dm;
                    }
                }
            }
#pragma unroll
            for (int t = 0; t < TY; t++) {
                if (t >= pyn_w) continue;
                int o[R];
                hsum_scalar<int, R, KW>(t == 0 ? V0m : MIDm, o);
#pragma unroll
                for (int j = 0; j < R; j++) s3miss[t][j] += o[j];
            }
        }
        Col<M> V0[R], MID[R];    // MID becomes output row 1's sums after the last row
        issue(0);
        issue(1);
#pragma unroll
        for (int r = 0; r < NYR; r++) {
            if (r + 2 < NYR) issue(r + 2);
            Row3<T, R>& rr = rw[r % 3];
            T ax[R], ay[R], bx[R], by[R];
            __builtin_memcpy(ax, rr.xi, sizeof(T) * R);
            __builtin_memcpy(ay, rr.yi, sizeof(T) * R);
            __builtin_memcpy(bx, rr.xo, sizeof(T) * R);
            __builtin_memcpy(by, rr.yo, sizeof(T) * R);
            int m[R], mo[R];
#pragma unroll
            for (int j = 0; j < R; j++) { m[j] = 0; mo[j] = 0; }
            if constexpr (kFloat && !DIRTY) {
                // entering values: finite and above the threshold?  (the
                // leaving plane entered earlier and passed this test then)
                bool ok = true;
                float mxr = 0.f, myr = 0.f;
#pragma unroll
                for (int j = 0; j < R; j++) {
                    ok = ok & (ax[j] > g.miss_thr) & (ay[j] > g.miss_thr);
                    mxr = fmaxf(mxr, __builtin_fabsf(ax[j]));
                    myr = fmaxf(myr, __builtin_fabsf(ay[j]));
                }
                ok = ok & (mxr < __builtin_inff()) & (myr < __builtin_inff());
                if (__builtin_amdgcn_ballot_w64(!ok)) {
                    found = true;                 // the step is taken again, masked
                } else {
                    hmx = fmaxf(hmx, mxr);
                    hmy = fmaxf(hmy, myr);
                }
            }
            if constexpr (kFloat && DIRTY) {
                // positions outside the volume read zero and are never missing
                const bool row_in = (unsigned)(ys + r) < (unsigned)H && c0 >= 0 && c0 < W;
                const bool in_i = row_in && (unsigned)zin < (unsigned)D;
                const bool in_o = row_in && (unsigned)zout < (unsigned)D;
#pragma unroll
                for (int j = 0; j < R; j++) {
                    m[j] = (in_i && (is_missing(ax[j], g.miss_thr) |
                                     is_missing(ay[j], g.miss_thr))) ? 1 : 0;
                    mo[j] = (in_o && (is_missing(bx[j], g.miss_thr) |
                                      is_missing(by[j], g.miss_thr))) ? 1 : 0;
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
                if (r == 0) {
                    V0[j] = col_delta<M, T>(ax[j], ay[j], bx[j], by[j], 0, 0);
                } else if (r == 1) {
                    MID[j] = col_delta<M, T>(ax[j], ay[j], bx[j], by[j], 0, 0);
                } else {
                    if (r == KW) col_add<M>(V0[j], MID[j]);
                    col_accum_delta<M, T>(MID[j], ax[j], ay[j], bx[j], by[j]);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
        }

        if constexpr (!DIRTY) {
            if (found) return false;             // nothing of this step was kept
        }
        // ---- x-window sums, running 3-D sums, and (plane finished) the epilogue ----
        const bool ready = li == next_ready;
        if (ready) next_ready += g.sz;
        const int zlo = pz * g.sz + g.oz, zhi = zlo + g.kz - 1;
        const bool zb = fill && (zlo < 0 || zhi >= D);
        const double nzp = (double)(min(zhi, D - 1) - max(zlo, 0) + 1);
        double gx = 0.0, gy = 0.0;
        if constexpr (kFloat) {
            if (ready) {
                float mx = hmx, my = hmy;
                for (int sft = 1; sft < kWave; sft <<= 1) {
                    mx = fmaxf(mx, __shfl_xor(mx, sft));
                    my = fmaxf(my, __shfl_xor(my, sft));
                }
                gx = g.cert_g * (double)mx * (double)mx;
                gy = g.cert_g * (double)my * (double)my;
            }
        }
#pragma unroll
        for (int t = 0; t < TY; t++) {
            if (t >= pyn_w) continue;
            Col<M>(&VV)[R] = t == 0 ? V0 : MID;
            // x-window sums channel by channel, added into the running sums
            auto chan = [&](auto fidx) __attribute__((always_inline)) {
                constexpr int F = decltype(fidx)::value;
                using FV = std::remove_reference_t<decltype(col_field<M, F>(VV[0]))>;
                FV v[R], o[R];
#pragma unroll
                for (int j = 0; j < R; j++) v[j] = col_field<M, F>(VV[j]);
                hsum_scalar<FV, R, KW>(v, o);
                if constexpr (M == MODE_F64 && F == 5) {
#pragma unroll
                    for (int j = 0; j < R; j++) s3miss[t][j] += o[j];
                    return;
                }
                constexpr int w0 = col_field_word<M, F>();
#pragma unroll
                for (int j = 0; j < R; j++) {
                    uint32_t* b = s3w + (t * R + j) * NDW * kWave + w0 * kWave + lane;
                    if constexpr (sizeof(FV) == 8) {
                        uint32_t lo = b[0], hi = b[kWave];
                        FV cur;
                        const uint32_t ww[2] = {lo, hi};
                        __builtin_memcpy(&cur, ww, 8);
                        cur = cur + o[j];
                        uint32_t nw[2];
                        __builtin_memcpy(nw, &cur, 8);
                        b[0] = nw[0];
                        b[kWave] = nw[1];
                    } else {
                        FV cur;
                        const uint32_t w = b[0];
                        __builtin_memcpy(&cur, &w, 4);
                        cur = cur + o[j];
                        uint32_t nw;
                        __builtin_memcpy(&nw, &cur, 4);
                        b[0] = nw;
                    }
                }
            };
            chan(std::integral_constant<int, 0>{});
            chan(std::integral_constant<int, 1>{});
            chan(std::integral_constant<int, 2>{});
            chan(std::integral_constant<int, 3>{});
            chan(std::integral_constant<int, 4>{});
            if (!ready) continue;
            const int ylo = (py0 + t) + g.oy, yhi = ylo + KW - 1;
            const bool rowb = fill && (ylo < 0 || yhi >= H);
            const double nrow = (double)(min(yhi, H - 1) - max(ylo, 0) + 1);
            const size_t orow = ((size_t)pz * g.OH + (size_t)(py0 + t)) * (size_t)g.OW;
#pragma unroll
            for (int j = 0; j < R; j++) {
                if (!((omask >> j) & 1u) || t >= pyn) continue;
                Col<M> A3;
                {
                    uint32_t w[NDW];
#pragma unroll
                    for (int i = 0; i < NDW; i++) w[i] = s3w[((t * R + j) * NDW + i) * kWave + lane];
                    __builtin_memcpy(&A3, w, NDW * 4);
                    if constexpr (M == MODE_F64) A3.miss = s3miss[t][j];
                }
                const bool fb = zb || rowb || ((fillb >> j) & 1u);
                const double dn = nzp * nrow * (double)ncol[j];
                uint8_t fl = 0;
                float cv = 0.f;
                if (fb) {
                    fl = FL_BORDER;
                } else if constexpr (kFloat) {
                    if (DIRTY && A3.miss > 0) {
                        fl = FL_MISSING;
                    } else {
                        const double N = __builtin_fma(dn, A3.xy, -(A3.x * A3.y));
                        const double Vx = __builtin_fma(dn, A3.xx, -(A3.x * A3.x));
                        const double Vy = __builtin_fma(dn, A3.yy, -(A3.y * A3.y));
                        const bool cert = (Vx > gx) && (Vy > gy) && !(g.force & 1);
                        if (cert) {
                            cv = clamp_unit(newton_ratio(N, Vx * Vy));
                        } else {
                            const int64_t clo = (int64_t)qj[j] * g.sx + g.ox;
                            fl = twopass_window((const float*)g.x, (const float*)g.y,
                                                (int64_t)H * W, (int64_t)W, max(zlo, 0),
                                                min(zhi, D - 1), max(ylo, 0), min(yhi, H - 1),
                                                max(clo, (int64_t)0),
                                                min(clo + KW - 1, (int64_t)W - 1), &cv);
                        }
                    }
                } else {
                    const double sxv = (double)A3.x, syv = (double)A3.y;
                    const double N = __builtin_fma(0.5 * dn, (double)A3.xy2, -(sxv * syv));
                    const double Vx = __builtin_fma(dn, (double)A3.xx, -(sxv * sxv));
                    const double Vy = __builtin_fma(dn, (double)A3.yy, -(syv * syv));
                    fl = (Vx == 0.0 ? FL_ZVAR_X : 0) | (Vy == 0.0 ? FL_ZVAR_Y : 0);
                    if (!fl) cv = rn32_certified(N, Vx, Vy, (g.force & 1) != 0);
                }
                if (fl) cv = g.invalid;
                g.c[orow + (uint32_t)qj[j]] = cv;
                if (has_flags) g.flags[orow + (uint32_t)qj[j]] = fl;
            }
        }
        if (ready) ++pz;
        return true;
    };
    for (int li = 0; li < nz; li++) {
        if constexpr (kFloat) {
            if (!dirty) {
                if (zstep(li, std::false_type{})) continue;
                dirty = true;
            }
            zstep(li, std::true_type{});
        } else {
            zstep(li, std::false_type{});
        }
    }
}

// CUBE: 0 general step, 1 specialised step, 2 specialised step in halves
template <int M, int R, int KW, int TY, bool VEC, int CUBE>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(2, 8))) corr3d_kernel(P3D g)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
    const int wpb = blockDim.x / kWave;
    const int tile = xcd_remap(blockIdx.x, gridDim.x) * wpb + wv;
    if (tile >= g.n_tiles) return;
    if constexpr (CUBE != 0)
        tile3d_cube<M, R, KW, CUBE == 2>(g, tile, smem + (size_t)wv * cube_lds_per_wave<M>(R));
    else
        tile3d<M, R, KW, TY, VEC>(g, tile, smem + (size_t)wv * tile3d_lds_per_wave<M, TY>(R));
}

}  // namespace swc
