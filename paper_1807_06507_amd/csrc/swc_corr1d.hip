// 1-D sliding-window correlation (Poyda & Zhizhin, arXiv 1807.06507: the
// one-dimensional moving sum of Section 1, applied to x, y, xy, x^2, y^2,
// then the one-pass formula per position).
//
// Work decomposition: one wavefront owns a contiguous segment of outputs and
// walks the window-end positions e of that segment in rows of 64*R
// consecutive positions (lane t owns positions row + t*R .. row + t*R + R-1).
// With S_e the sum over [e-k+1, e]:
//     S_e = S_{e-1} + v_e - v_{e-k}
// so a row of S values is  carry + (prefix over the row of d_e = v_e - v_{e-k}):
// an in-lane prefix over R positions, a wavefront scan of the lane totals
// (DPP row shifts + row broadcasts) and the carry from the previous row.
// Entering values come from HBM (coalesced); the value k positions back is
// read from a per-wave LDS ring that holds the last k + 64R positions, split
// into R sub-rings by position mod R so that every LDS access of a wavefront
// touches consecutive words.  Windows whose ring does not fit in LDS re-read
// the leaving values from global memory instead (they were read k positions
// earlier by the same wave and are normally still in L2).  The carry starts
// from a direct sum of the k positions before the segment.
#include "swc_device.hpp"
#include "swc_internal.h"

namespace swc {

struct P1D {
    const void* x;
    const void* y;
    float* c;
    uint8_t* flags;
    int64_t N, ON;
    int k, s, off;        // window, step, window start offset (-k/2 or 0)
    int border;
    float invalid;
    float miss_thr;
    int force;
    double cert_g;
    int64_t seg;          // outputs per wave
    int64_t n_waves;
    int ring;             // ring positions (power of two, multiple of R)
};

constexpr int kR1 = 8;    // positions per lane per row

// ---- wavefront inclusive scan (64 lanes) via DPP -------------------------
template <int CTRL, int RMASK, bool BC>
__device__ __forceinline__ uint32_t dppm(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, RMASK, 0xf, BC);
}

template <int CTRL, int RMASK, bool BC, class V> __device__ __forceinline__ V dppv(V v)
{
    constexpr int NW = sizeof(V) / 4;
    uint32_t w[NW];
    __builtin_memcpy(w, &v, sizeof(V));
#pragma unroll
    for (int i = 0; i < NW; i++) w[i] = dppm<CTRL, RMASK, BC>(w[i]);
    V r;
    __builtin_memcpy(&r, w, sizeof(V));
    return r;
}

// Inclusive prefix sum over the 64 lanes (lane order).
template <class V> __device__ __forceinline__ V wave_incl_scan(V v)
{
    v += dppv<0x111, 0xf, true>(v);   // row_shr:1
    v += dppv<0x112, 0xf, true>(v);   // row_shr:2
    v += dppv<0x114, 0xf, true>(v);   // row_shr:4
    v += dppv<0x118, 0xf, true>(v);   // row_shr:8
    v += dppv<0x142, 0xa, false>(v);  // row_bcast:15 -> rows 1, 3
    v += dppv<0x143, 0xc, false>(v);  // row_bcast:31 -> rows 2, 3
    return v;
}

template <class V> __device__ __forceinline__ V lane63(V v)
{
    constexpr int NW = sizeof(V) / 4;
    uint32_t w[NW];
    __builtin_memcpy(w, &v, sizeof(V));
#pragma unroll
    for (int i = 0; i < NW; i++) w[i] = (uint32_t)__builtin_amdgcn_readlane((int)w[i], 63);
    V r;
    __builtin_memcpy(&r, w, sizeof(V));
    return r;
}

__device__ __forceinline__ float wave_max(float v)
{
    v = fmaxf(v, __uint_as_float(dppm<0x111, 0xf, true>(__float_as_uint(v))));
    v = fmaxf(v, __uint_as_float(dppm<0x112, 0xf, true>(__float_as_uint(v))));
    v = fmaxf(v, __uint_as_float(dppm<0x114, 0xf, true>(__float_as_uint(v))));
    v = fmaxf(v, __uint_as_float(dppm<0x118, 0xf, true>(__float_as_uint(v))));
    v = fmaxf(v, __uint_as_float(dppm<0x142, 0xa, false>(__float_as_uint(v))));
    v = fmaxf(v, __uint_as_float(dppm<0x143, 0xc, false>(__float_as_uint(v))));
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(v), 63));
}

// Channel accumulator for 1-D: integer modes keep Sx, Sy as int and the
// product sums as exact integers in FP64; the float mode keeps five FP64
// sums and a missing count.
template <int M> struct Ch {
    double x, y, xx, yy, xy;
    int miss;
};

template <int M> __device__ __forceinline__ Ch<M> ch_zero() { return Ch<M>{0, 0, 0, 0, 0, 0}; }
template <int M> __device__ __forceinline__ void ch_add(Ch<M>& a, const Ch<M>& b)
{
    a.x += b.x; a.y += b.y; a.xx += b.xx; a.yy += b.yy; a.xy += b.xy; a.miss += b.miss;
}

// d_e = v_e - v_{e-k} for one position (values already zero outside [0, N)
// and sanitized; m/mo: missing bits).
template <int M>
__device__ __forceinline__ Ch<M> ch_diff(float x, float y, float xo, float yo, int m, int mo)
{
    Ch<M> d;
    const double a = (double)x, b = (double)y, ao = (double)xo, bo = (double)yo;
    d.x = a - ao;
    d.y = b - bo;
    d.xx = __builtin_fma(a, a, -(ao * ao));
    d.yy = __builtin_fma(b, b, -(bo * bo));
    d.xy = __builtin_fma(a, b, -(ao * bo));
    d.miss = m - mo;
    return d;
}

template <int M, class T> __device__ __forceinline__ float as_val(T v) { return (float)v; }

template <int M, bool RING>
__global__ void __launch_bounds__(256) corr1d_kernel(P1D g)
{
    using T = typename Tr<M>::T;
    constexpr int R = kR1;
    constexpr bool kFloat = !Tr<M>::kInt;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
    const int wpb = blockDim.x / kWave;
    const int64_t w = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * wpb + wv;
    if (w >= g.n_waves) return;

    const T* __restrict__ X = (const T*)g.x;
    const T* __restrict__ Y = (const T*)g.y;
    const int64_t N = g.N;
    const int k = g.k;
    // ring: R sub-rings of ring/R entries for x, y (values as float) and a
    // missing bit per position
    const int ring = g.ring;
    const int sub = ring / R;
    const size_t wave_bytes = (size_t)ring * (kFloat ? 9 : 8);
    float* rx = (float*)(smem + (size_t)wv * wave_bytes);
    float* ry = rx + ring;
    uint8_t* rm = (uint8_t*)(ry + ring);

    const int64_t p_first = w * g.seg;
    const int64_t p_last = min(p_first + g.seg, g.ON) - 1;
    const int64_t e_first = p_first * g.s + g.off + k - 1;   // window end of p_first
    const int64_t e_last = p_last * g.s + g.off + k - 1;
    const int kal = ((k + R - 1) / R) * R;
    const int64_t e_base = e_first - kal;                     // ring position 0

    auto load_val = [&](const T* __restrict__ A, int64_t e) -> float {
        return (e >= 0 && e < N) ? (float)A[e] : 0.f;
    };
    auto slot_of = [&](int64_t e, int& sr, int& si) {
        const int64_t d = e - e_base;                  // >= 0 for every position used
        sr = (int)(d % R);
        si = (int)((d / R) & (sub - 1));
    };

    // ---- init: positions [e_first - kal, e_first - 1] into the ring; carry
    //      = sum over [e_first - k, e_first - 1] ----
    Ch<M> part = ch_zero<M>();
    float mx = 0.f, my = 0.f;
    for (int i = lane; i < kal; i += kWave) {
        const int64_t e = e_base + i;
        float a = load_val(X, e), b = load_val(Y, e);
        int m = 0;
        if constexpr (kFloat) {
            m = (is_missing(a, g.miss_thr) || is_missing(b, g.miss_thr)) ? 1 : 0;
            if (m) { a = 0.f; b = 0.f; }
        }
        if constexpr (RING) {
            int sr, si;
            slot_of(e, sr, si);
            rx[sr * sub + si] = a;
            ry[sr * sub + si] = b;
            rm[sr * sub + si] = (uint8_t)m;
        }
        if (i >= kal - k) {
            Ch<M> d = ch_diff<M>(a, b, 0.f, 0.f, m, 0);
            ch_add<M>(part, d);
            mx = fmaxf(mx, __builtin_fabsf(a));
            my = fmaxf(my, __builtin_fabsf(b));
        }
    }
    Ch<M> carry;
    {
        Ch<M> sc;
        sc.x = lane63(wave_incl_scan(part.x));
        sc.y = lane63(wave_incl_scan(part.y));
        sc.xx = lane63(wave_incl_scan(part.xx));
        sc.yy = lane63(wave_incl_scan(part.yy));
        sc.xy = lane63(wave_incl_scan(part.xy));
        sc.miss = lane63(wave_incl_scan(part.miss));
        carry = sc;
    }
    float MX = wave_max(mx), MY = wave_max(my);
    wave_lds_sync();

    // certification factor for this wave's chain (float input)
    const double gcert = g.cert_g;

    for (int64_t row = e_first; row <= e_last; row += kWave * R) {
        const int64_t e0 = row + (int64_t)lane * R;
        float a[R], b[R], ao[R], bo[R];
        int m[R], mo[R];
        // entering values
#pragma unroll
        for (int j = 0; j < R; j++) {
            a[j] = load_val(X, e0 + j);
            b[j] = load_val(Y, e0 + j);
        }
        float lmx = 0.f, lmy = 0.f;
#pragma unroll
        for (int j = 0; j < R; j++) {
            m[j] = 0;
            if constexpr (kFloat) {
                m[j] = (is_missing(a[j], g.miss_thr) || is_missing(b[j], g.miss_thr)) ? 1 : 0;
                a[j] = m[j] ? 0.f : a[j];
                b[j] = m[j] ? 0.f : b[j];
                lmx = fmaxf(lmx, __builtin_fabsf(a[j]));
                lmy = fmaxf(lmy, __builtin_fabsf(b[j]));
            }
        }
        if constexpr (RING) {
            // park the entering values first: for k < 64R a position's
            // leaving value can be an entering value of this same row
            wave_lds_sync();   // previous row's reads are ordered before these writes
#pragma unroll
            for (int j = 0; j < R; j++) {
                int sr, si;
                slot_of(e0 + j, sr, si);
                rx[sr * sub + si] = a[j];
                ry[sr * sub + si] = b[j];
                rm[sr * sub + si] = (uint8_t)m[j];
            }
            wave_lds_sync();
            // leaving values (k positions back) from the ring
#pragma unroll
            for (int j = 0; j < R; j++) {
                int sr, si;
                slot_of(e0 + j - k, sr, si);
                ao[j] = rx[sr * sub + si];
                bo[j] = ry[sr * sub + si];
                mo[j] = rm[sr * sub + si];
            }
        } else {
            // leaving values re-read from global memory
#pragma unroll
            for (int j = 0; j < R; j++) {
                ao[j] = load_val(X, e0 + j - k);
                bo[j] = load_val(Y, e0 + j - k);
                mo[j] = 0;
                if constexpr (kFloat) {
                    mo[j] = (is_missing(ao[j], g.miss_thr) || is_missing(bo[j], g.miss_thr)) ? 1 : 0;
                    ao[j] = mo[j] ? 0.f : ao[j];
                    bo[j] = mo[j] ? 0.f : bo[j];
                }
            }
        }
        if constexpr (kFloat) {
            MX = fmaxf(MX, wave_max(lmx));
            MY = fmaxf(MY, wave_max(lmy));
        }
        // in-lane prefix of d
        Ch<M> P[R];
#pragma unroll
        for (int j = 0; j < R; j++) {
            P[j] = ch_diff<M>(a[j], b[j], ao[j], bo[j], m[j], mo[j]);
            if (j > 0) ch_add<M>(P[j], P[j - 1]);
        }
        // wavefront scan of lane totals -> exclusive offsets
        Ch<M> tot = P[R - 1];
        Ch<M> inc;
        inc.x = wave_incl_scan(tot.x);
        inc.y = wave_incl_scan(tot.y);
        inc.xx = wave_incl_scan(tot.xx);
        inc.yy = wave_incl_scan(tot.yy);
        inc.xy = wave_incl_scan(tot.xy);
        inc.miss = wave_incl_scan(tot.miss);
        Ch<M> base;
        base.x = carry.x + (inc.x - tot.x);
        base.y = carry.y + (inc.y - tot.y);
        base.xx = carry.xx + (inc.xx - tot.xx);
        base.yy = carry.yy + (inc.yy - tot.yy);
        base.xy = carry.xy + (inc.xy - tot.xy);
        base.miss = carry.miss + (inc.miss - tot.miss);
        carry.x += lane63(inc.x);
        carry.y += lane63(inc.y);
        carry.xx += lane63(inc.xx);
        carry.yy += lane63(inc.yy);
        carry.xy += lane63(inc.xy);
        carry.miss += lane63(inc.miss);
        const double gx = gcert * (double)MX * (double)MX;
        const double gy = gcert * (double)MY * (double)MY;

        // ---- outputs ending at e0 + j ----
#pragma unroll
        for (int j = 0; j < R; j++) {
            const int64_t e = e0 + j;
            if (e > e_last) continue;
            const int64_t qs = e - (int64_t)(g.off + k - 1);     // = p*s
            if (qs < 0) continue;
            int64_t p = qs;
            if (g.s != 1) {
                p = qs / g.s;
                if (p * g.s != qs) continue;
            }
            if (p < p_first || p > p_last) continue;
            Ch<M> S = base;
            ch_add<M>(S, P[j]);
            const int64_t lo = e - k + 1;
            const bool bord = lo < 0 || e > N - 1;
            const int64_t nl = (e < N - 1 ? e : N - 1) - (lo > 0 ? lo : 0) + 1;
            uint8_t fl = (g.border == BORDER_FILL && bord) ? FL_BORDER : 0;
            float cv = 0.f;
            if (!fl && S.miss > 0) fl = FL_MISSING;
            if (!fl) {
                const double dn = (double)nl;
                if constexpr (kFloat) {
                    const double Nn = __builtin_fma(dn, S.xy, -(S.x * S.y));
                    const double Vx = __builtin_fma(dn, S.xx, -(S.x * S.x));
                    const double Vy = __builtin_fma(dn, S.yy, -(S.y * S.y));
                    const bool cert = (Vx > gx) && (Vy > gy) && !(g.force & 1);
                    if (cert) {
                        cv = clamp_unit(Nn * rsqrt64(Vx * Vy));
                    } else {
                        const int64_t cl = lo > 0 ? lo : 0, ch = e < N - 1 ? e : N - 1;
                        fl = twopass_window((const float*)g.x, (const float*)g.y, 0, 0, 0, 0, 0,
                                            0, cl, ch, &cv);
                    }
                } else {
                    // exact integers: every sum below 2^53
                    const double Nn = __builtin_fma(dn, S.xy, -(S.x * S.y));
                    const double Vx = __builtin_fma(dn, S.xx, -(S.x * S.x));
                    const double Vy = __builtin_fma(dn, S.yy, -(S.y * S.y));
                    fl = (Vx == 0.0 ? FL_ZVAR_X : 0) | (Vy == 0.0 ? FL_ZVAR_Y : 0);
                    if (!fl) cv = rn32_certified(Nn, Vx, Vy, (g.force & 1) != 0);
                }
            }
            if (fl) cv = g.invalid;
            g.c[p] = cv;
            if (g.flags) g.flags[p] = fl;
        }
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static int ring_positions(int k)
{
    const int need = ((k + kR1 - 1) / kR1) * kR1 + kWave * kR1;
    int r = kWave * kR1;
    while (r < need) r <<= 1;
    return r;
}

static size_t lds_per_wave_1d(int mode, int k)
{
    return (size_t)ring_positions(k) * (mode >= MODE_F64 ? 9 : 8);
}

// The LDS ring is used when it fits in 64 KB per workgroup.
static bool ring_fits_1d(int mode, int k, int wpb)
{
    return lds_per_wave_1d(mode, k) * (size_t)wpb <= 64 * 1024;
}

bool cfg_ok_1d(const swc_problem& p, const LaunchCfg& L)
{
    const int mode = mode_of(p.dtype, p.accum);
    if (mode != MODE_U8 && mode != MODE_U16 && mode != MODE_F64) return false;
    if (!(L.wpb == 1 || L.wpb == 2 || L.wpb == 4)) return false;
    if (L.TH < 1 || L.TH > (1 << 20)) return false;
    return L.R == kR1;
}

template <int M>
static hipError_t go1d(const P1D& g, int grid, int wpb, size_t smem, hipStream_t s)
{
    if (smem)
        hipLaunchKernelGGL((corr1d_kernel<M, true>), dim3(grid), dim3(wpb * kWave), smem, s, g);
    else
        hipLaunchKernelGGL((corr1d_kernel<M, false>), dim3(grid), dim3(wpb * kWave), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_corr1d(const swc_problem& p, const int64_t* oshape, const LaunchCfg& L,
                         const void* x, const void* y, float* c, uint8_t* flags,
                         hipStream_t s, int force)
{
    const int mode = mode_of(p.dtype, p.accum);
    P1D g;
    g.x = x;
    g.y = y;
    g.c = c;
    g.flags = flags;
    g.N = p.shape[0];
    g.ON = oshape[0];
    g.k = p.window[0];
    g.s = p.step[0];
    g.off = window_offset(p.border, g.k);
    g.border = p.border;
    g.invalid = p.invalid_value;
    g.miss_thr = missing_threshold(p.missing_le);
    g.force = force;
    // outputs per wave: TH rows of 64*R window-end positions
    const int64_t span = (int64_t)L.TH * kWave * kR1;
    g.seg = span / g.s > 0 ? span / g.s : 1;
    g.n_waves = (g.ON + g.seg - 1) / g.seg;
    g.ring = ring_positions(g.k);
    const double rows = (double)(g.seg * g.s) / (kWave * kR1) + 1.0;
    const double chain = 2.0 * (double)(g.seg * g.s + g.k) + 16.0 * rows + 64.0;
    g.cert_g = cert_factor(mode, (double)g.k, chain, (double)g.k + 3.0);
    const int64_t grid64 = (g.n_waves + L.wpb - 1) / L.wpb;
    if (grid64 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const size_t smem =
        ring_fits_1d(mode, g.k, L.wpb) ? lds_per_wave_1d(mode, g.k) * (size_t)L.wpb : 0;
    switch (mode) {
    case MODE_U8: return go1d<MODE_U8>(g, (int)grid64, L.wpb, smem, s);
    case MODE_U16: return go1d<MODE_U16>(g, (int)grid64, L.wpb, smem, s);
    default: return go1d<MODE_F64>(g, (int)grid64, L.wpb, smem, s);
    }
}

}  // namespace swc
