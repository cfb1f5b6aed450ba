// Device-side building blocks of the fused sliding-window correlation
// kernels (gfx950, wave64).  Paper: Poyda & Zhizhin, arXiv 1807.06507.
//
//  * element contributions x, y, xy, x^2, y^2 (Section 1, step 1), with the
//    missing-value rule of Section 3 (values <= missing_le, NaN, Inf);
//  * accumulators for the five sliding sums (steps 2-3) in the precision
//    each input type needs: exact integers for u8/u16, FP64 for f32 (products
//    of two floats are exact in FP64), plain FP32 for the naive comparator,
//    TwoSum-compensated FP32 pairs for the compensated mode;
//  * the per-position epilogue (step 4, the one-pass formula of Section 1),
//    with the zero-denominator rule of Section 3;
//  * exactly rounded float32 output for integer inputs: an FP64 estimate
//    whose error is bounded, and an exact big-integer decision for the rare
//    estimates that fall too close to a float32 rounding midpoint;
//  * a direct two-pass evaluation of one window (Introduction formula) for
//    float windows the error bound cannot certify.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swc {

constexpr int kWave = 64;

enum Mode : int {
    MODE_U8 = 0,     // u8 input, int32 sums
    MODE_U16 = 1,    // u16 input, int32 Sx/Sy, exact-integer FP64 Sxx/Sxy/Syy
    MODE_F64 = 2,    // f32 input, FP64 sums (default)
    MODE_F32N = 3,   // f32 input, naive FP32 sums + FP32 epilogue
    MODE_F32C = 4    // f32 input, compensated FP32 sums + FP64 epilogue
};

enum : uint8_t { FL_BORDER = 1, FL_MISSING = 2, FL_ZVAR_X = 4, FL_ZVAR_Y = 8 };
enum : int { BORDER_FILL = 0, BORDER_CLIP = 1, BORDER_VALID = 2 };

// ---------------------------------------------------------------------------
// Compensated FP32 value (hi + lo), TwoSum on every update.
// ---------------------------------------------------------------------------
struct CF {
    float hi, lo;
};
__device__ __forceinline__ CF cf_zero() { return CF{0.f, 0.f}; }
// Contraction is off in every compensated step: fusing a product into the
// TwoSum (s = hi + a*a as one fma) would fold the exact product into s while
// its TwoProd tail is still added to lo, counting the tail twice.
__device__ __forceinline__ CF cf_add(CF a, float b)
{
#pragma clang fp contract(off)
    float s = a.hi + b;
    float bp = s - a.hi;
    float err = (a.hi - (s - bp)) + (b - bp);
    return CF{s, a.lo + err};
}
__device__ __forceinline__ CF cf_add(CF a, CF b)
{
#pragma clang fp contract(off)
    CF t = cf_add(a, b.hi);
    t.lo += b.lo;
    return t;
}
__device__ __forceinline__ CF cf_neg(CF a) { return CF{-a.hi, -a.lo}; }
__device__ __forceinline__ double cf_val(CF a) { return (double)a.hi + (double)a.lo; }

// ---------------------------------------------------------------------------
// Types per mode
// ---------------------------------------------------------------------------
template <int M> struct Tr;
template <> struct Tr<MODE_U8> {
    using T = uint8_t;
    using SX = int;      // sum of x, y
    using SQ = int;      // sum of squares / cross products
    static constexpr bool kMiss = false;
    static constexpr bool kInt = true;
};
template <> struct Tr<MODE_U16> {
    using T = uint16_t;
    using SX = int;
    using SQ = double;   // integer-valued, exact below 2^53
    static constexpr bool kMiss = false;
    static constexpr bool kInt = true;
};
template <> struct Tr<MODE_F64> {
    using T = float;
    using SX = double;
    using SQ = double;
    static constexpr bool kMiss = true;
    static constexpr bool kInt = false;
};
template <> struct Tr<MODE_F32N> {
    using T = float;
    using SX = float;
    using SQ = float;
    static constexpr bool kMiss = true;
    static constexpr bool kInt = false;
};
template <> struct Tr<MODE_F32C> {
    using T = float;
    using SX = CF;
    using SQ = CF;
    static constexpr bool kMiss = true;
    static constexpr bool kInt = false;
};

// Five sliding sums plus the count of missing elements.
template <int M> struct Acc {
    typename Tr<M>::SX x, y;
    typename Tr<M>::SQ xx, xy, yy;
    int miss;
};

// One element's contribution (already zeroed when missing).
template <int M> struct Elem {
    typename Tr<M>::SX x, y;
    typename Tr<M>::SQ xx, xy, yy;
    int miss;
};

template <int M> __device__ __forceinline__ void acc_zero(Acc<M>& a)
{
    if constexpr (M == MODE_F32C) {
        a.x = a.y = a.xx = a.xy = a.yy = cf_zero();
    } else {
        a.x = a.y = 0;
        a.xx = a.xy = a.yy = 0;
    }
    a.miss = 0;
}

// Missing-value rule for float data: <= threshold, NaN or +-Inf.
__device__ __forceinline__ bool is_missing(float v, float thr)
{
    return !(v > thr) || v == __builtin_inff();
}

// Element contribution from raw values.  `thr` is the missing threshold as
// float (x <= missing_le <=> x <= thr for float x, see the host side).
// `inb`: the position lies inside the array (positions outside read as zero
// and are never missing, whatever the threshold).
template <int M>
__device__ __forceinline__ Elem<M> make_elem(typename Tr<M>::T vx, typename Tr<M>::T vy, float thr,
                                             bool inb = true)
{
    Elem<M> e;
    if constexpr (M == MODE_U8) {
        int a = vx, b = vy;
        e.x = a; e.y = b;
        e.xx = a * a; e.xy = a * b; e.yy = b * b;
        e.miss = 0;
    } else if constexpr (M == MODE_U16) {
        int a = vx, b = vy;
        e.x = a; e.y = b;
        double da = (double)a, db = (double)b;
        e.xx = da * da; e.xy = da * db; e.yy = db * db;   // exact (< 2^32)
        e.miss = 0;
    } else {
        bool m = inb && (is_missing(vx, thr) || is_missing(vy, thr));
        float a = m ? 0.f : vx;
        float b = m ? 0.f : vy;
        e.miss = m ? 1 : 0;
        if constexpr (M == MODE_F64) {
            double da = (double)a, db = (double)b;
            e.x = da; e.y = db;
            e.xx = da * da; e.xy = da * db; e.yy = db * db; // exact in FP64
        } else if constexpr (M == MODE_F32N) {
            e.x = a; e.y = b;
            e.xx = a * a; e.xy = a * b; e.yy = b * b;
        } else {
            // compensated: exact products via FMA split (TwoProd); the
            // rounded products must stay rounded (no contraction into the
            // sums that consume them)
#pragma clang fp contract(off)
            float pxx = a * a, pxy = a * b, pyy = b * b;
            e.x = CF{a, 0.f};
            e.y = CF{b, 0.f};
            e.xx = CF{pxx, __builtin_fmaf(a, a, -pxx)};
            e.xy = CF{pxy, __builtin_fmaf(a, b, -pxy)};
            e.yy = CF{pyy, __builtin_fmaf(b, b, -pyy)};
        }
    }
    return e;
}

template <int M> __device__ __forceinline__ void acc_add(Acc<M>& a, const Elem<M>& e)
{
    if constexpr (M == MODE_F32C) {
        a.x = cf_add(a.x, e.x); a.y = cf_add(a.y, e.y);
        a.xx = cf_add(a.xx, e.xx); a.xy = cf_add(a.xy, e.xy); a.yy = cf_add(a.yy, e.yy);
    } else {
        a.x += e.x; a.y += e.y; a.xx += e.xx; a.xy += e.xy; a.yy += e.yy;
    }
    if constexpr (Tr<M>::kMiss) a.miss += e.miss;
}

template <int M> __device__ __forceinline__ void acc_sub(Acc<M>& a, const Elem<M>& e)
{
    if constexpr (M == MODE_F32C) {
        a.x = cf_add(a.x, cf_neg(e.x)); a.y = cf_add(a.y, cf_neg(e.y));
        a.xx = cf_add(a.xx, cf_neg(e.xx)); a.xy = cf_add(a.xy, cf_neg(e.xy));
        a.yy = cf_add(a.yy, cf_neg(e.yy));
    } else {
        a.x -= e.x; a.y -= e.y; a.xx -= e.xx; a.xy -= e.xy; a.yy -= e.yy;
    }
    if constexpr (Tr<M>::kMiss) a.miss -= e.miss;
}

// Accumulator arithmetic (sums of accumulators in the second pass).
template <int M> __device__ __forceinline__ void acc_addacc(Acc<M>& a, const Acc<M>& b)
{
    if constexpr (M == MODE_F32C) {
        a.x = cf_add(a.x, b.x); a.y = cf_add(a.y, b.y);
        a.xx = cf_add(a.xx, b.xx); a.xy = cf_add(a.xy, b.xy); a.yy = cf_add(a.yy, b.yy);
    } else {
        a.x += b.x; a.y += b.y; a.xx += b.xx; a.xy += b.xy; a.yy += b.yy;
    }
    if constexpr (Tr<M>::kMiss) a.miss += b.miss;
}
template <int M> __device__ __forceinline__ void acc_subacc(Acc<M>& a, const Acc<M>& b)
{
    if constexpr (M == MODE_F32C) {
        a.x = cf_add(a.x, cf_neg(b.x)); a.y = cf_add(a.y, cf_neg(b.y));
        a.xx = cf_add(a.xx, cf_neg(b.xx)); a.xy = cf_add(a.xy, cf_neg(b.xy));
        a.yy = cf_add(a.yy, cf_neg(b.yy));
    } else {
        a.x -= b.x; a.y -= b.y; a.xx -= b.xx; a.xy -= b.xy; a.yy -= b.yy;
    }
    if constexpr (Tr<M>::kMiss) a.miss -= b.miss;
}

// ---------------------------------------------------------------------------
// LDS row buffer: structure of arrays, one array per channel, ncol entries.
// ---------------------------------------------------------------------------
template <int M> struct LdsRow {
    typename Tr<M>::SX* x;
    typename Tr<M>::SX* y;
    typename Tr<M>::SQ* xx;
    typename Tr<M>::SQ* xy;
    typename Tr<M>::SQ* yy;
    int* miss;
    float* mx;   // per-lane history max |x| (float modes only), kWave entries
    float* my;
};

template <int M> __host__ __device__ constexpr int lds_col_bytes()
{
    return 2 * (int)sizeof(typename Tr<M>::SX) + 3 * (int)sizeof(typename Tr<M>::SQ) +
           (Tr<M>::kMiss ? 4 : 0);
}

template <int M> __host__ __device__ constexpr int lds_row_bytes(int ncol)
{
    // channels padded to 16-byte multiples, plus two kWave float arrays
    return ((lds_col_bytes<M>() * ncol + 15) & ~15) + (Tr<M>::kMiss ? 2 * kWave * 4 : 0) + 64;
}

template <int M> __device__ __forceinline__ LdsRow<M> lds_row_carve(char* base, int ncol)
{
    LdsRow<M> r;
    char* p = base;
    r.x = (typename Tr<M>::SX*)p; p += sizeof(typename Tr<M>::SX) * ncol;
    r.y = (typename Tr<M>::SX*)p; p += sizeof(typename Tr<M>::SX) * ncol;
    r.xx = (typename Tr<M>::SQ*)p; p += sizeof(typename Tr<M>::SQ) * ncol;
    r.xy = (typename Tr<M>::SQ*)p; p += sizeof(typename Tr<M>::SQ) * ncol;
    r.yy = (typename Tr<M>::SQ*)p; p += sizeof(typename Tr<M>::SQ) * ncol;
    if constexpr (Tr<M>::kMiss) {
        r.miss = (int*)p; p += 4 * ncol;
        p = (char*)(((uintptr_t)p + 15) & ~(uintptr_t)15);
        r.mx = (float*)p; p += 4 * kWave;
        r.my = (float*)p;
    } else {
        r.miss = nullptr;
        r.mx = r.my = nullptr;
    }
    return r;
}

template <int M> __device__ __forceinline__ void lds_put(const LdsRow<M>& r, int i, const Acc<M>& a)
{
    r.x[i] = a.x; r.y[i] = a.y; r.xx[i] = a.xx; r.xy[i] = a.xy; r.yy[i] = a.yy;
    if constexpr (Tr<M>::kMiss) r.miss[i] = a.miss;
}

template <int M> __device__ __forceinline__ Acc<M> lds_get(const LdsRow<M>& r, int i)
{
    Acc<M> a;
    a.x = r.x[i]; a.y = r.y[i]; a.xx = r.xx[i]; a.xy = r.xy[i]; a.yy = r.yy[i];
    if constexpr (Tr<M>::kMiss) a.miss = r.miss[i]; else a.miss = 0;
    return a;
}

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

// Order LDS traffic of one wavefront (writes by some lanes, reads by others).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Workgroup -> XCD-contiguous index.  Workgroups are dispatched round-robin
// over the 8 XCDs; renumber them so that each XCD receives a contiguous run
// of work (neighbouring tiles then share halo rows through the same L2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_remap(int bid, int nblocks)
{
    constexpr int kXcd = 8;
    if (nblocks < kXcd) return bid;
    int xcd = bid % kXcd;
    int j = bid / kXcd;
    int full = nblocks / kXcd;
    int rem = nblocks % kXcd;
    return (xcd < rem) ? xcd * (full + 1) + j : rem * (full + 1) + (xcd - rem) * full + j;
}

// ---------------------------------------------------------------------------
// Exactly rounded float32 of N / sqrt(Vx*Vy) for exact integers
// |N|, Vx, Vy < 2^53 (Vx, Vy > 0).
// ---------------------------------------------------------------------------
struct U320 {
    uint64_t w[5];
};

__device__ __forceinline__ void u128_mul(uint64_t a, uint64_t b, uint64_t& lo, uint64_t& hi)
{
    lo = a * b;
    hi = __umul64hi(a, b);
}

// r = (a1:a0) << s into 5 limbs; returns false when bits would be lost.
// Limbs are placed by selects, never by a computed index, so the value stays
// in registers.
__device__ inline bool u320_from_shifted(uint64_t a0, uint64_t a1, int s, U320& r)
{
    const int limb = s >> 6, bit = s & 63;
    // (a1:a0) << bit as three limbs v0, v1, v2
    const uint64_t v0 = a0 << bit;
    const uint64_t v1 = bit ? ((a1 << bit) | (a0 >> (64 - bit))) : a1;
    const uint64_t v2 = bit ? (a1 >> (64 - bit)) : 0;
    r.w[0] = limb == 0 ? v0 : 0;
    r.w[1] = limb == 0 ? v1 : (limb == 1 ? v0 : 0);
    r.w[2] = limb == 0 ? v2 : (limb == 1 ? v1 : (limb == 2 ? v0 : 0));
    r.w[3] = limb == 1 ? v2 : (limb == 2 ? v1 : (limb == 3 ? v0 : 0));
    r.w[4] = limb == 2 ? v2 : (limb == 3 ? v1 : (limb == 4 ? v0 : 0));
    // limbs that would land beyond the fifth
    const bool lost = (limb == 3 && v2 != 0) || (limb == 4 && (v1 | v2) != 0) ||
                      (limb >= 5 && (v0 | v1 | v2) != 0);
    return !lost;
}

// r = m * (b1:b0), m < 2^64 -> 3 limbs (stored into 5)
__device__ inline void u320_mul_64_128(uint64_t m, uint64_t b0, uint64_t b1, U320& r)
{
    uint64_t l0, h0, l1, h1;
    u128_mul(m, b0, l0, h0);
    u128_mul(m, b1, l1, h1);
    r.w[0] = l0;
    uint64_t s1 = h0 + l1;
    uint64_t c1 = s1 < h0 ? 1 : 0;
    r.w[1] = s1;
    r.w[2] = h1 + c1;
    r.w[3] = 0;
    r.w[4] = 0;
}

__device__ inline int u320_cmp(const U320& a, const U320& b)
{
    for (int i = 4; i >= 0; i--) {
        if (a.w[i] != b.w[i]) return a.w[i] > b.w[i] ? 1 : -1;
    }
    return 0;
}

// Exact decision: RN32 of |N|/sqrt(VxVy) given an estimate `a` (>= 0) whose
// error is far below half a float32 ulp.  The float32 bucket
// [trunc32(a), trunc32(a) + ulp] is split by its midpoint m; comparing the
// exact value with m decides (ties to even).
__device__ __noinline__ float rn32_exact_decide(double aN, double Vx, double Vy, double a)
{
    if (aN == 0.0) return 0.0f;
    uint64_t bits = (uint64_t)__double_as_longlong(a);
    uint64_t tb = bits & ~0x1FFFFFFFull;                 // trunc to float32 precision
    uint64_t mb = tb | 0x10000000ull;                    // bucket midpoint
    float f_lo = (float)__longlong_as_double((long long)tb);
    float f_hi = __uint_as_float(__float_as_uint(f_lo) + 1u);   // f_lo > 0
    int ebits = (int)((mb >> 52) & 0x7FF);
    uint64_t mant = (mb & ((1ull << 52) - 1)) | (1ull << 52);
    uint64_t Mp = mant >> 28;                            // 25-bit integer
    int E = ebits - 1023 - 24;                           // m = Mp * 2^E
    uint64_t n = (uint64_t)aN;
    uint64_t a0, a1;
    u128_mul(n, n, a0, a1);                              // N^2
    uint64_t v0, v1;
    u128_mul((uint64_t)Vx, (uint64_t)Vy, v0, v1);        // Vx*Vy
    U320 rhs;
    u320_mul_64_128(Mp * Mp, v0, v1, rhs);               // Mp^2 Vx Vy
    U320 lhs;
    int cmp;
    if (E < 0) {
        bool ok = u320_from_shifted(a0, a1, -2 * E, lhs);
        cmp = ok ? u320_cmp(lhs, rhs) : 1;
    } else {
        // m >= 1 cannot be exceeded by a coefficient bounded by 1
        cmp = -1;
    }
    float f;
    if (cmp > 0) f = f_hi;
    else if (cmp < 0) f = f_lo;
    else f = (__float_as_uint(f_lo) & 1u) ? f_hi : f_lo;
    return f;
}

// Certified RN32.  Estimate: r0 = v_rsq_f32(float(Vx*Vy)) (relative error
// below 2^-20 with ample slack), one FP64 Newton step (error ~1.5 e0^2 plus a
// few FP64 roundings, below 2^-39), c = N * r.  The estimate's relative error
// is therefore below 2^-38; outputs within that distance of a float32
// midpoint (the 29 discarded mantissa bits within 2^15 of 2^28) take the
// exact decision.
__device__ __forceinline__ float rn32_certified(double N, double Vx, double Vy, bool force)
{
    if (N == 0.0) return 0.0f;
    double q = Vx * Vy;
    double r = (double)__builtin_amdgcn_rsqf((float)q);
    double h = 0.5 * q;
    double e = __builtin_fma(-h * r, r, 0.5);
    r = __builtin_fma(r, e, r);
    double aN = __builtin_fabs(N);
    double a = aN * r;
    uint32_t t = (uint32_t)__double_as_longlong(a) & 0x1FFFFFFFu;
    constexpr uint32_t kMargin = 1u << 15;
    bool amb = (t - (0x10000000u - kMargin)) <= 2u * kMargin;
    float f = (float)a;
    if (amb || force) f = rn32_exact_decide(aN, Vx, Vy, a);
    return N < 0 ? -f : f;
}

// FP64 reciprocal square root of a positive normal double: hardware
// estimate plus two Newton steps (relative error ~1e-16 level).
__device__ __forceinline__ double rsqrt64(double q)
{
    double r = __builtin_amdgcn_rsq(q);
    double h = 0.5 * q;
    double e = __builtin_fma(-h * r, r, 0.5);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-h * r, r, 0.5);
    r = __builtin_fma(r, e, r);
    return r;
}

// N / sqrt(q) for q > 0 from the hardware rsqrt estimate r (relative error
// below 2^-20) and one Newton step: N r (1 + e/2) with e = 1 - q r^2.
// Relative error below 2^-38.
__device__ __forceinline__ double newton_ratio(double N, double q)
{
    const double r = __builtin_amdgcn_rsq(q);
    const double e = __builtin_fma(-(q * r), r, 1.0);
    const double a0 = N * r;
    return __builtin_fma(0.5 * a0, e, a0);
}

__device__ __forceinline__ float clamp_unit(double c)
{
    c = c > 1.0 ? 1.0 : c;
    c = c < -1.0 ? -1.0 : c;
    return (float)c;
}

// ---------------------------------------------------------------------------
// Two-pass evaluation of one window (the Introduction's classical formula),
// for float windows that the error bound cannot certify.  The window is the
// box [lo, hi] (inclusive, already clipped to the array) of a C-ordered
// array with up to three dimensions: strides (s0, s1, 1).
// Returns the flags (ZVAR bits) in bits 32..39 and c's bits in bits 0..31
// (a value rather than a pointer: the caller's result stays in registers and
// the call needs no stack).
// ---------------------------------------------------------------------------
__device__ __noinline__ uint64_t twopass_window_packed(const float* __restrict__ x,
                                                       const float* __restrict__ y, int64_t s0,
                                                       int64_t s1, int64_t lo0, int64_t hi0,
                                                       int64_t lo1, int64_t hi1, int64_t lo2,
                                                       int64_t hi2)
{
    double sx = 0.0, sy = 0.0;
    float x0 = x[lo0 * s0 + lo1 * s1 + lo2];
    float y0 = y[lo0 * s0 + lo1 * s1 + lo2];
    bool eqx = true, eqy = true;
    int64_t n = 0;
    for (int64_t a = lo0; a <= hi0; a++)
        for (int64_t b = lo1; b <= hi1; b++)
            for (int64_t c = lo2; c <= hi2; c++) {
                float vx = x[a * s0 + b * s1 + c];
                float vy = y[a * s0 + b * s1 + c];
                eqx = eqx && (vx == x0);
                eqy = eqy && (vy == y0);
                sx += (double)vx;
                sy += (double)vy;
                n++;
            }
    uint8_t fl = (eqx ? FL_ZVAR_X : 0) | (eqy ? FL_ZVAR_Y : 0);
    if (fl) return (uint64_t)fl << 32;
    double mx = sx / (double)n, my = sy / (double)n;
    double sxy = 0.0, sxx = 0.0, syy = 0.0;
    for (int64_t a = lo0; a <= hi0; a++)
        for (int64_t b = lo1; b <= hi1; b++)
            for (int64_t c = lo2; c <= hi2; c++) {
                double dx = (double)x[a * s0 + b * s1 + c] - mx;
                double dy = (double)y[a * s0 + b * s1 + c] - my;
                sxy += dx * dy;
                sxx += dx * dx;
                syy += dy * dy;
            }
    return (uint64_t)__float_as_uint(clamp_unit(sxy / __builtin_sqrt(sxx * syy)));
}

// The same with the coefficient written to *cval (inlined: *cval is the
// caller's register) and the flags returned.
__device__ __forceinline__ uint8_t twopass_window(const float* __restrict__ x,
                                                  const float* __restrict__ y, int64_t s0,
                                                  int64_t s1, int64_t lo0, int64_t hi0,
                                                  int64_t lo1, int64_t hi1, int64_t lo2,
                                                  int64_t hi2, float* cval)
{
    const uint64_t r = twopass_window_packed(x, y, s0, s1, lo0, hi0, lo1, hi1, lo2, hi2);
    *cval = __uint_as_float((uint32_t)r);
    return (uint8_t)(r >> 32);
}

// ---------------------------------------------------------------------------
// Epilogue (Section 1 formula, step 4) on window sums S of n elements.
// Window box for the fallback: [lo, hi] per axis (clipped), strides s0, s1.
// mx, my: bounds on |x|, |y| over everything that entered S's history;
// cert_g: the host's rounding-error factor G (see the design notes).
// Returns flags; writes *cval when flags == 0.
// ---------------------------------------------------------------------------
struct WinBox {
    int64_t s0, s1;
    int64_t lo0, hi0, lo1, hi1, lo2, hi2;
};

template <int M>
__device__ __forceinline__ uint8_t epilogue(const Acc<M>& S, int64_t n, float mx, float my,
                                            double cert_g, bool force, const void* xp,
                                            const void* yp, const WinBox& wb, float* cval)
{
    if constexpr (M == MODE_U8 || M == MODE_U16) {
        double dn = (double)n;
        double sx = (double)S.x, sy = (double)S.y;
        double N = __builtin_fma(dn, (double)S.xy, -(sx * sy));
        double Vx = __builtin_fma(dn, (double)S.xx, -(sx * sx));
        double Vy = __builtin_fma(dn, (double)S.yy, -(sy * sy));
        uint8_t fl = (Vx == 0.0 ? FL_ZVAR_X : 0) | (Vy == 0.0 ? FL_ZVAR_Y : 0);
        if (fl) return fl;
        *cval = rn32_certified(N, Vx, Vy, force);
        return 0;
    } else if constexpr (M == MODE_F32N) {
        float fn = (float)n;
        float N = fn * S.xy - S.x * S.y;
        float Vx = fn * S.xx - S.x * S.x;
        float Vy = fn * S.yy - S.y * S.y;
        uint8_t fl = (Vx <= 0.f ? FL_ZVAR_X : 0) | (Vy <= 0.f ? FL_ZVAR_Y : 0);
        if (fl) return fl;
        float c = N / __builtin_sqrtf(Vx * Vy);
        c = c > 1.f ? 1.f : (c < -1.f ? -1.f : c);
        *cval = c;
        return 0;
    } else {
        double sx, sy, sxx, sxy, syy;
        if constexpr (M == MODE_F64) {
            sx = S.x; sy = S.y; sxx = S.xx; sxy = S.xy; syy = S.yy;
        } else {
            sx = cf_val(S.x); sy = cf_val(S.y);
            sxx = cf_val(S.xx); sxy = cf_val(S.xy); syy = cf_val(S.yy);
        }
        double dn = (double)n;
        double N = __builtin_fma(dn, sxy, -(sx * sy));
        double Vx = __builtin_fma(dn, sxx, -(sx * sx));
        double Vy = __builtin_fma(dn, syy, -(sy * sy));
        double Mx = (double)mx, My = (double)my;
        bool cert = (Vx > cert_g * Mx * Mx) && (Vy > cert_g * My * My) && !force;
        if (!cert) {
            return twopass_window((const float*)xp, (const float*)yp, wb.s0, wb.s1, wb.lo0,
                                  wb.hi0, wb.lo1, wb.hi1, wb.lo2, wb.hi2, cval);
        }
        double r = rsqrt64(Vx * Vy);
        *cval = clamp_unit(N * r);
        return 0;
    }
}

}  // namespace swc
