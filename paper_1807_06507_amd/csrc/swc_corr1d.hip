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
// Entering values and the values k positions back are both read through
// raw buffers over the wave's span (the latter were read by the same wave a
// few rows earlier and come from L2); positions outside the array read as
// zero.  All per-lane index arithmetic is 32-bit, relative to the span
// start, and the next row's loads are in flight while a row is processed.
// The carry starts from a direct sum of the k positions before the segment.
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
    int vst;              // output base 16-byte aligned: whole-vector stores allowed
    int ring_g;           // RING kernel: groups of 8 positions in the per-wave LDS ring
};

constexpr int kR1 = 8;    // positions per lane per row

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

// Raw buffer over one wave's span of an input array: position d of the span
// (span position 0 = array index e_base) is read at byte offset d * esz;
// positions outside the array read as zero (out-of-range offsets).
struct SpanBuf {
    __amdgpu_buffer_rsrc_t rs;
    int shift;      // e_base - max(e_base, 0) (<= 0), in elements
};

constexpr int kBufWord3_1d = 0x00020000;   // raw buffer access (gfx9 family)

template <class T>
__device__ __forceinline__ SpanBuf span_buf(const T* A, int64_t N, int64_t e_base)
{
    const int64_t eb0 = e_base > 0 ? e_base : 0;
    const int64_t avail = N - eb0 > 0 ? N - eb0 : 0;
    const int64_t bytes = avail * (int64_t)sizeof(T);
    const int nrec = (int)(bytes < 0x7FFFFFF0ll ? bytes : 0x7FFFFFF0ll);
    SpanBuf b;
    b.rs = __builtin_amdgcn_make_buffer_rsrc((void*)(A + eb0), (short)0, nrec, kBufWord3_1d);
    b.shift = (int)(e_base - eb0);
    return b;
}

template <class T>
__device__ __forceinline__ float span_load(const SpanBuf& b, int d)
{
    // positions before the array get an offset far beyond any record count
    // (never a wrapped negative offset)
    const int o = d + b.shift;
    const uint32_t off = o >= 0 ? (uint32_t)o * (uint32_t)sizeof(T) : 0x80000000u;
    if constexpr (sizeof(T) == 4) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(b.rs, off, 0, 0));
    } else if constexpr (sizeof(T) == 2) {
        return (float)__builtin_amdgcn_raw_buffer_load_b16(b.rs, off, 0, 0);
    } else {
        return (float)__builtin_amdgcn_raw_buffer_load_b8(b.rs, off, 0, 0);
    }
}

// R consecutive span positions d0 .. d0+R-1.  f32 input with the whole run
// inside the array: 16-byte loads (dword aligned; the memory system takes
// unaligned vector accesses); otherwise one load per element.
template <class T, int R>
__device__ __forceinline__ void span_load_run(const SpanBuf& b, int d0, bool whole, float (&v)[R])
{
    if constexpr (sizeof(T) == 4 && R % 4 == 0) {
        if (whole) {
            const uint32_t off = (uint32_t)(d0 + b.shift) * 4u;
#pragma unroll
            for (int i = 0; i < R; i += 4) {
                typedef uint32_t u4 __attribute__((ext_vector_type(4)));
                const u4 w = __builtin_amdgcn_raw_buffer_load_b128(b.rs, off + 4u * i, 0, 0);
                v[i] = __uint_as_float(w.x);
                v[i + 1] = __uint_as_float(w.y);
                v[i + 2] = __uint_as_float(w.z);
                v[i + 3] = __uint_as_float(w.w);
            }
            return;
        }
    }
#pragma unroll
    for (int j = 0; j < R; j++) v[j] = span_load<T>(b, d0 + j);
}

// One row of R window-end positions per lane: entering and leaving values.
template <int R> struct Row1 {
    float a[R], b[R], ao[R], bo[R];
};

// Two waves per SIMD for the float kernel; the integer kernels (larger
// per-lane state) are left to the compiler.
template <int M> constexpr int corr1d_min_waves() { return M == MODE_F64 ? 2 : 1; }

// RING: the values leaving the window come from a per-wave LDS ring of the
// last ring_g*8 positions instead of a second read from memory.  Position p
// lives at word (p mod 8) * ring_g + (p / 8 mod ring_g): a lane owns 8
// consecutive positions starting at a multiple of 8, so for each of its 8
// elements the 64 lanes write, and (shifted back by k) read, 64 consecutive
// words.  The ring holds the raw values; missing values are masked on use.
template <int M, bool RING>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(corr1d_min_waves<M>(), 8)))
corr1d_kernel(P1D g)
{
    using T = typename Tr<M>::T;
    constexpr int R = kR1;
    constexpr bool kFloat = !Tr<M>::kInt;
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
    const int wpb = blockDim.x / kWave;
    const int64_t w = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * wpb + wv;
    if (w >= g.n_waves) return;

    const int64_t N = g.N;
    const int k = g.k;
    const int64_t p_first = w * g.seg;
    const int64_t p_last = min(p_first + g.seg, g.ON) - 1;
    const int64_t e_first = p_first * g.s + g.off + k - 1;   // window end of p_first
    const int64_t e_last = p_last * g.s + g.off + k - 1;
    const int kal = ((k + R - 1) / R) * R;
    // span positions are relative to e_base; everything below is 32-bit
    const int64_t e_base = e_first - kal;
    const int d_end = (int)(e_last - e_base);                // last window end
    const int64_t nlim64 = N - e_base;                       // positions d < nlim are < N
    const int nlim = (int)(nlim64 > 0x3FFFFFFF ? 0x3FFFFFFF : (nlim64 < -0x3FFFFFFF ? -0x3FFFFFFF : nlim64));
    const int dmin = (int)(e_base < 0 ? -e_base : 0);        // positions d >= dmin are >= 0
    const SpanBuf bx = span_buf<T>((const T*)g.x, N, e_base);
    const SpanBuf by = span_buf<T>((const T*)g.y, N, e_base);
    const int pstep = g.s;

    // ---- per-wave LDS ring (RING) ----
    extern __shared__ float ring_smem[];
    const int rg = g.ring_g;
    float* ringx = ring_smem + (size_t)wv * 2 * 8 * rg;
    float* ringy = ringx + 8 * rg;
    auto ring_at = [&](int p) __attribute__((always_inline)) {
        return (p & 7) * rg + ((p >> 3) & (rg - 1));
    };

    // ---- carry = sums over span positions [kal - k, kal - 1] ----
    Ch<M> part = ch_zero<M>();
    float mx = 0.f, my = 0.f;
    for (int i = kal - k + lane; i < kal; i += kWave) {
        float a = span_load<T>(bx, i), b = span_load<T>(by, i);
        if constexpr (RING) {
            ringx[ring_at(i)] = a;
            ringy[ring_at(i)] = b;
        }
        int m = 0;
        if constexpr (kFloat) {
            // positions outside the series read zero and are never missing
            const bool inb = i >= dmin && i < nlim;
            m = (inb && (is_missing(a, g.miss_thr) || is_missing(b, g.miss_thr))) ? 1 : 0;
            if (m) { a = 0.f; b = 0.f; }
        }
        ch_add<M>(part, ch_diff<M>(a, b, 0.f, 0.f, m, 0));
        mx = fmaxf(mx, __builtin_fabsf(a));
        my = fmaxf(my, __builtin_fabsf(b));
    }
    Ch<M> carry;
    carry.x = lane63(wave_incl_scan(part.x));
    carry.y = lane63(wave_incl_scan(part.y));
    carry.xx = lane63(wave_incl_scan(part.xx));
    carry.yy = lane63(wave_incl_scan(part.yy));
    carry.xy = lane63(wave_incl_scan(part.xy));
    carry.miss = lane63(wave_incl_scan(part.miss));
    float MX = wave_max(mx), MY = wave_max(my);
    const double gcert = g.cert_g;
    const bool has_flags = g.flags != nullptr;
    const bool fill = g.border == BORDER_FILL;

    // outputs of this wave as raw buffers (out-of-range offsets drop stores)
    const int nout = (int)(p_last - p_first + 1);
    const __amdgpu_buffer_rsrc_t rc =
        __builtin_amdgcn_make_buffer_rsrc(g.c + p_first, (short)0, nout * 4, kBufWord3_1d);
    const __amdgpu_buffer_rsrc_t rf = __builtin_amdgcn_make_buffer_rsrc(
        has_flags ? (void*)(g.flags + p_first) : (void*)g.c, (short)0, has_flags ? nout : 0,
        kBufWord3_1d);

    auto load_row = [&](int rrel, Row1<R>& r) __attribute__((always_inline)) {
        const int d0 = rrel + lane * R;
        const bool whole_in = (d0 >= dmin) && (d0 + R - 1 < nlim);
        const bool whole_out = (d0 - k >= dmin) && (d0 - k + R - 1 < nlim);
        span_load_run<T, R>(bx, d0, whole_in, r.a);
        span_load_run<T, R>(by, d0, whole_in, r.b);
        if constexpr (!RING) {
            span_load_run<T, R>(bx, d0 - k, whole_out, r.ao);
            span_load_run<T, R>(by, d0 - k, whole_out, r.bo);
        }
    };

    auto process = [&](int rrel, Row1<R>& r) __attribute__((always_inline)) {
        const int d0 = rrel + lane * R;
        if constexpr (RING) {
            // park the entering row, then read the leaving one (it may lie in
            // this row when k < 64*R; a wave's LDS accesses complete in order)
#pragma unroll
            for (int j = 0; j < R; j++) {
                ringx[ring_at(d0 + j)] = r.a[j];
                ringy[ring_at(d0 + j)] = r.b[j];
            }
#pragma unroll
            for (int j = 0; j < R; j++) {
                r.ao[j] = ringx[ring_at(d0 + j - k)];
                r.bo[j] = ringy[ring_at(d0 + j - k)];
            }
        }
        int m[R], mo[R];
        float lmx = 0.f, lmy = 0.f;
#pragma unroll
        for (int j = 0; j < R; j++) { m[j] = 0; mo[j] = 0; }
        if constexpr (kFloat) {
            // a value is missing when it is <= the threshold, NaN or +-Inf;
            // test the row's extremes first and look at single values only
            // when the wave's rows hold one
            float lo = r.a[0], hi = r.a[0];
#pragma unroll
            for (int j = 0; j < R; j++) {
                lo = fminf(lo, fminf(fminf(r.a[j], r.b[j]), fminf(r.ao[j], r.bo[j])));
                hi = fmaxf(hi, fmaxf(fmaxf(r.a[j], r.b[j]), fmaxf(r.ao[j], r.bo[j])));
            }
            // fminf/fmaxf drop NaN operands, so NaN needs its own test
            bool nan = false;
#pragma unroll
            for (int j = 0; j < R; j++)
                nan = nan | (r.a[j] != r.a[j]) | (r.b[j] != r.b[j]) | (r.ao[j] != r.ao[j]) |
                      (r.bo[j] != r.bo[j]);
            const bool clean = (lo > g.miss_thr) & (hi < __builtin_inff()) & !nan;
            if (__builtin_amdgcn_ballot_w64(!clean)) {
#pragma unroll
                for (int j = 0; j < R; j++) {
                    // positions outside the series read zero and are never missing
                    const bool in_i = d0 + j >= dmin && d0 + j < nlim;
                    const bool in_o = d0 - k + j >= dmin && d0 - k + j < nlim;
                    m[j] = (in_i && (is_missing(r.a[j], g.miss_thr) |
                                     is_missing(r.b[j], g.miss_thr))) ? 1 : 0;
                    mo[j] = (in_o && (is_missing(r.ao[j], g.miss_thr) |
                                      is_missing(r.bo[j], g.miss_thr))) ? 1 : 0;
                    r.a[j] = m[j] ? 0.f : r.a[j];
                    r.b[j] = m[j] ? 0.f : r.b[j];
                    r.ao[j] = mo[j] ? 0.f : r.ao[j];
                    r.bo[j] = mo[j] ? 0.f : r.bo[j];
                }
            }
#pragma unroll
            for (int j = 0; j < R; j++) {
                lmx = fmaxf(lmx, __builtin_fabsf(r.a[j]));
                lmy = fmaxf(lmy, __builtin_fabsf(r.b[j]));
            }
        }
        if constexpr (kFloat) {
            MX = fmaxf(MX, wave_max(lmx));
            MY = fmaxf(MY, wave_max(lmy));
        }
        // in-lane prefix of the differences
        Ch<M> P[R];
#pragma unroll
        for (int j = 0; j < R; j++) {
            P[j] = ch_diff<M>(r.a[j], r.b[j], r.ao[j], r.bo[j], m[j], mo[j]);
            if (j > 0) ch_add<M>(P[j], P[j - 1]);
        }
        // wavefront scan of the lane totals -> exclusive offsets
        const Ch<M> tot = P[R - 1];
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

        // ---- outputs ending at span positions d0 + j ----
        // window of end d: span positions [d-k+1, d]; inside the array when
        // d - k + 1 >= dmin and d < nlim (uniform test for the whole row)
        const bool row_inside = (rrel - k + 1 >= dmin) && (rrel + kWave * R - 1 < nlim);
        float cv[R];
        uint32_t flw[R / 4] = {};
        bool any_pend = false;
        uint32_t outm = 0;   // which of the R positions are output window ends
#pragma unroll
        for (int j = 0; j < R; j++) {
            const int d = d0 + j;
            const int qs = d - kal;                                 // = (p - p_first) * s
            const bool is_out = (d <= d_end) && (qs >= 0) && (pstep == 1 || (qs % pstep) == 0);
            outm |= is_out ? (1u << j) : 0u;
            Ch<M> S = base;
            ch_add<M>(S, P[j]);
            double dn;
            bool bord;
            if (row_inside) {
                dn = (double)k;
                bord = false;
            } else {
                const int lo = d - k + 1;
                bord = lo < dmin || d >= nlim;
                const int clo = lo > dmin ? lo : dmin, chi = d < nlim - 1 ? d : nlim - 1;
                dn = (double)(chi - clo + 1);
            }
            const bool fb = fill & bord;
            double Nn, Vx, Vy;
            if constexpr (kFloat) {
                Nn = __builtin_fma(dn, S.xy, -(S.x * S.y));
                Vx = __builtin_fma(dn, S.xx, -(S.x * S.x));
                Vy = __builtin_fma(dn, S.yy, -(S.y * S.y));
            } else {
                Nn = __builtin_fma(dn, S.xy, -(S.x * S.y));
                Vx = __builtin_fma(dn, S.xx, -(S.x * S.x));
                Vy = __builtin_fma(dn, S.yy, -(S.y * S.y));
            }
            const double q = Vx * Vy;
            float c;
            bool bad, pend;
            uint32_t fl;
            if constexpr (kFloat) {
                const bool cert = (Vx > gx) & (Vy > gy);
                c = clamp_unit(newton_ratio(Nn, q));
                const bool miss = S.miss > 0;
                bad = fb | miss;
                pend = (!bad) & ((!cert) | ((g.force & 1) != 0));
                fl = fb ? FL_BORDER : (miss ? FL_MISSING : 0u);
            } else {
                const double a = newton_ratio(Nn, q);
                const uint32_t lo29 = (uint32_t)__double_as_longlong(a) & 0x1FFFFFFFu;
                const bool amb = (lo29 - (0x10000000u - (1u << 15))) <= (2u << 15);
                c = (float)a;
                bad = fb | (q == 0.0);
                pend = (!bad) & (amb | ((g.force & 1) != 0));
                fl = fb ? FL_BORDER : ((Vx == 0.0 ? FL_ZVAR_X : 0u) | (Vy == 0.0 ? FL_ZVAR_Y : 0u));
            }
            asm volatile("" : "+v"(c));
            cv[j] = bad ? g.invalid : c;
            flw[j / 4] |= (bad ? fl : 0u) << (8 * (j % 4));
            any_pend = any_pend | (pend & is_out);
        }
        // rare path: two-pass recomputation (float) / exact rounding (integer)
        if (__builtin_amdgcn_ballot_w64(any_pend)) {
#pragma unroll
            for (int j = 0; j < R; j++) {
                const int d = d0 + j;
                if (!((outm >> j) & 1u)) continue;
                Ch<M> S = base;
                ch_add<M>(S, P[j]);
                const int lo = d - k + 1;
                const bool bord = lo < dmin || d >= nlim;
                if (fill && bord) continue;
                const int clo = lo > dmin ? lo : dmin, chi = d < nlim - 1 ? d : nlim - 1;
                const double dn = (double)(chi - clo + 1);
                const double Nn = __builtin_fma(dn, S.xy, -(S.x * S.y));
                const double Vx = __builtin_fma(dn, S.xx, -(S.x * S.x));
                const double Vy = __builtin_fma(dn, S.yy, -(S.y * S.y));
                if constexpr (kFloat) {
                    if (S.miss > 0) continue;
                    if ((Vx > gx) && (Vy > gy) && !(g.force & 1)) continue;
                    float c2 = 0.f;
                    const int64_t cl = e_base + clo, ch = e_base + chi;
                    const uint8_t f2 = twopass_window((const float*)g.x, (const float*)g.y, 0, 0, 0,
                                                      0, 0, 0, cl, ch, &c2);
                    cv[j] = f2 ? g.invalid : c2;
                    flw[j / 4] = (flw[j / 4] & ~(0xFFu << (8 * (j % 4)))) | ((uint32_t)f2 << (8 * (j % 4)));
                } else {
                    if (Vx == 0.0 || Vy == 0.0) continue;
                    cv[j] = rn32_certified(Nn, Vx, Vy, (g.force & 1) != 0);
                }
            }
        }
        // ---- stores: output index p - p_first = qs / s ----
        if (pstep == 1) {
            const int o0 = d0 - kal;                                  // output of position d0
            const bool whole = g.vst && (o0 >= 0) && (o0 + R - 1 < nout) && ((o0 & 3) == 0) &&
                               ((p_first & 3) == 0);
            if (whole) {
#pragma unroll
                for (int j = 0; j < R; j += 4) {
                    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
                    const u4 v = {__float_as_uint(cv[j]), __float_as_uint(cv[j + 1]),
                                  __float_as_uint(cv[j + 2]), __float_as_uint(cv[j + 3])};
                    __builtin_amdgcn_raw_buffer_store_b128(v, rc, (uint32_t)(o0 + j) * 4u, 0, 0);
                }
                if (has_flags) {
#pragma unroll
                    for (int j = 0; j < R; j++)
                        __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(flw[j / 4] >> (8 * (j % 4))),
                                                             rf, (uint32_t)(o0 + j), 0, 0);
                }
                return;
            }
        }
#pragma unroll
        for (int j = 0; j < R; j++) {
            const int d = d0 + j;
            const int qs = d - kal;
            // byte offsets; positions that are not outputs of this wave get an
            // offset beyond any record count (applied after the scaling, so
            // it cannot wrap)
            const bool is_o = (outm >> j) & 1u;
            const uint32_t o = (uint32_t)(qs / pstep);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(cv[j]), rc,
                                                  is_o ? o * 4u : 0x80000000u, 0, 0);
            if (has_flags)
                __builtin_amdgcn_raw_buffer_store_b8((uint8_t)(flw[j / 4] >> (8 * (j % 4))), rf,
                                                     is_o ? o : 0x80000000u, 0, 0);
        }
    };

    // rows of R*64 window ends, the next row's loads in flight while one is
    // processed (two register sets, alternating)
    constexpr int kRow = kWave * R;
    Row1<R> A, B;
    int rrel = kal;
    load_row(rrel, A);
    while (true) {
        const int r1 = rrel + kRow;
        if (r1 <= d_end) load_row(r1, B);
        process(rrel, A);
        if (r1 > d_end) break;
        const int r2 = r1 + kRow;
        if (r2 <= d_end) load_row(r2, A);
        process(r1, B);
        if (r2 > d_end) break;
        rrel = r2;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

bool cfg_ok_1d(const swc_problem& p, const LaunchCfg& L)
{
    const int mode = mode_of(p.dtype, p.accum);
    if (mode != MODE_U8 && mode != MODE_U16 && mode != MODE_F64) return false;
    if (!(L.wpb == 1 || L.wpb == 2 || L.wpb == 4)) return false;
    if (L.TH < 1 || L.TH > (1 << 16)) return false;
    return L.R == kR1;
}

template <int M>
static hipError_t go1d(const P1D& g, int grid, int wpb, hipStream_t s)
{
    if (g.ring_g > 0) {
        const size_t smem = (size_t)wpb * 2 * 8 * g.ring_g * sizeof(float);
        return launch_kernel(&corr1d_kernel<M, true>, dim3(grid), dim3(wpb * kWave), smem, s, g);
    }
    return launch_kernel(&corr1d_kernel<M, false>, dim3(grid), dim3(wpb * kWave), 0, s, g);
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
    g.vst = ((uintptr_t)c % 16 == 0) ? 1 : 0;
    const double rows = (double)(g.seg * g.s) / (kWave * kR1) + 1.0;
    const double chain = 2.0 * (double)(g.seg * g.s + g.k) + 16.0 * rows + 64.0;
    g.cert_g = cert_factor(mode, (double)g.k, chain, (double)g.k + 3.0);
    // LDS ring of the leaving values: a power-of-two number of 8-position
    // groups covering k + one row, at most 32 KB per wave (else re-read)
    g.ring_g = 0;
    {
        int64_t need = ((int64_t)g.k + kWave * kR1 + 7) / 8, rg = 1;
        while (rg < need) rg <<= 1;
        if (rg * 8 * 2 * (int64_t)sizeof(float) <= 32 * 1024 && !(force & 4)) g.ring_g = (int)rg;
    }
    const int64_t grid64 = (g.n_waves + L.wpb - 1) / L.wpb;
    if (grid64 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    switch (mode) {
    case MODE_U8: return go1d<MODE_U8>(g, (int)grid64, L.wpb, s);
    case MODE_U16: return go1d<MODE_U16>(g, (int)grid64, L.wpb, s);
    default: return go1d<MODE_F64>(g, (int)grid64, L.wpb, s);
    }
}

}  // namespace swc
