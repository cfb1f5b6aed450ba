// Unfused schemes of the same 2-D operation, kept as measured baselines for
// the fused kernels (Poyda & Zhizhin, arXiv 1807.06507):
//
//  * SWC_SCHEME_UNFUSED: the paper's parallel scheme (Section 2).  Step 1 (element
//    products) and step 4 (the Section 1 formula) run one thread per element;
//    step 2 runs one thread per row and step 3 one thread per column, each
//    walking its line with a running (moving) sum.  The intermediate matrices
//    of Section 1 (the products; the row sums Ax, Ay, Axy, Ax2, Ay2; the window
//    sums Sx, Sy, Sxy, Sx2, Sy2) live in device memory between the kernels.
//  * SWC_SCHEME_CUMSUM: the cumulative-sum alternative that Section 1 mentions
//    (and reports as slower): 2-D prefix sums (integral images) of the five
//    channels, then each window sum by inclusion-exclusion of four corners.
//    Integer inputs only: uint64 prefix sums are exact modulo 2^64, and every
//    true window sum is far below 2^63, so the wrapped differences are exact.
//
// Both give the same results as the fused kernels: exact window sums for
// integer inputs (FP64 integers below 2^53, certified float32 rounding); for
// float inputs FP64 running sums with the rigorous certification test and the
// two-pass fallback, using the global |x|, |y| maxima as the bound.
#include <mutex>

#include "swc_device.hpp"
#include "swc_internal.h"

namespace swc {

namespace {

constexpr int kChUnf = 6;   // x, y, xx, yy, xy, missing count
constexpr int kChCum = 5;   // x, y, xx, yy, xy
constexpr size_t kHdrBytes = 256;

struct SchemeGeom {
    int H, W, kh, kw, oh, ow;
    int border;
    float invalid;
    int force;
    double cert_g;
};

__device__ __forceinline__ float wave_max(float v)
{
    for (int s = 1; s < kWave; s <<= 1) v = fmaxf(v, __shfl_xor(v, s));
    return v;
}

__global__ void unf_init(uint32_t* hdr)
{
    if (threadIdx.x < 2) hdr[threadIdx.x] = 0u;
}

// Step 1: element values and products, one element per thread.  Missing
// float values contribute zero and a count of one.  The largest |x|, |y|
// is accumulated for the certification test.
template <class T, bool FLOAT>
__global__ void __launch_bounds__(256)
unf_products(const T* __restrict__ x, const T* __restrict__ y, double* __restrict__ E,
             int64_t plane, float thr, uint32_t* __restrict__ hdr)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float ax = 0.f, ay = 0.f;
    if (i < plane) {
        double vx, vy, m = 0.0;
        if constexpr (FLOAT) {
            const float fx = (float)x[i], fy = (float)y[i];
            const bool miss = is_missing(fx, thr) || is_missing(fy, thr);
            vx = miss ? 0.0 : (double)fx;
            vy = miss ? 0.0 : (double)fy;
            m = miss ? 1.0 : 0.0;
            ax = (float)__builtin_fabs(vx);
            ay = (float)__builtin_fabs(vy);
        } else {
            vx = (double)x[i];
            vy = (double)y[i];
        }
        E[0 * plane + i] = vx;
        E[1 * plane + i] = vy;
        E[2 * plane + i] = vx * vx;
        E[3 * plane + i] = vy * vy;
        E[4 * plane + i] = vx * vy;
        E[5 * plane + i] = m;
    }
    if constexpr (FLOAT) {
        ax = wave_max(ax);
        ay = wave_max(ay);
        if ((threadIdx.x & (kWave - 1)) == 0) {
            // non-negative floats order like their bit patterns
            atomicMax(&hdr[0], __float_as_uint(ax));
            atomicMax(&hdr[1], __float_as_uint(ay));
        }
    }
}

// Steps 2 and 3: moving sum of width k (window [j - lo, j - lo + k - 1],
// clipped to the line) along lines of length len, element stride `stride`,
// one thread per line; all channels advance together.
template <int NCH>
__global__ void __launch_bounds__(64)
unf_moving_sum(const double* __restrict__ in, double* __restrict__ out, int64_t plane,
               int nlines, int64_t line_stride, int len, int64_t stride, int k, int lo)
{
    const int l = blockIdx.x * 64 + threadIdx.x;
    if (l >= nlines) return;
    const int64_t base = (int64_t)l * line_stride;
    const int hi = k - 1 - lo;
    double s[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ch++) s[ch] = 0.0;
    const int first = hi < len - 1 ? hi : len - 1;
    for (int t = 0; t <= first; t++)
#pragma unroll
        for (int ch = 0; ch < NCH; ch++) s[ch] += in[ch * plane + base + t * stride];
    for (int j = 0; j < len; j++) {
        const int64_t o = base + (int64_t)j * stride;
#pragma unroll
        for (int ch = 0; ch < NCH; ch++) out[ch * plane + o] = s[ch];
        const int tin = j + hi + 1, tout = j - lo;
        if (tin < len) {
#pragma unroll
            for (int ch = 0; ch < NCH; ch++) s[ch] += in[ch * plane + base + (int64_t)tin * stride];
        }
        if (tout >= 0) {
#pragma unroll
            for (int ch = 0; ch < NCH; ch++) s[ch] -= in[ch * plane + base + (int64_t)tout * stride];
        }
    }
}

// Clipped window of output (r, j) and whether it crosses the border.
struct Box {
    int r0, r1, c0, c1;
    bool crosses;
};
__device__ __forceinline__ Box window_box(const SchemeGeom& g, int r, int j)
{
    const int ylo = r + g.oh, yhi = ylo + g.kh - 1;
    const int xlo = j + g.ow, xhi = xlo + g.kw - 1;
    Box b;
    b.crosses = ylo < 0 || yhi >= g.H || xlo < 0 || xhi >= g.W;
    b.r0 = ylo > 0 ? ylo : 0;
    b.r1 = yhi < g.H - 1 ? yhi : g.H - 1;
    b.c0 = xlo > 0 ? xlo : 0;
    b.c1 = xhi < g.W - 1 ? xhi : g.W - 1;
    return b;
}

// Step 4 on exact integer window sums (values below 2^53).
__device__ __forceinline__ uint8_t final_int(double n, double sx, double sy, double sxx,
                                             double syy, double sxy, bool force, float* cv)
{
    const double N = __builtin_fma(n, sxy, -(sx * sy));
    const double Vx = __builtin_fma(n, sxx, -(sx * sx));
    const double Vy = __builtin_fma(n, syy, -(sy * sy));
    const uint8_t fl = (Vx == 0.0 ? FL_ZVAR_X : 0) | (Vy == 0.0 ? FL_ZVAR_Y : 0);
    if (fl) return fl;
    *cv = rn32_certified(N, Vx, Vy, force);
    return 0;
}

// Step 4 for the unfused scheme, one thread per output.
template <bool FLOAT>
__global__ void __launch_bounds__(256)
unf_final(const double* __restrict__ S, int64_t plane, SchemeGeom g, const float* __restrict__ xf,
          const float* __restrict__ yf, const uint32_t* __restrict__ hdr, float* __restrict__ c,
          uint8_t* __restrict__ flags)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= plane) return;
    const int r = (int)(i / g.W), j = (int)(i - (int64_t)r * g.W);
    const Box b = window_box(g, r, j);
    uint8_t fl = 0;
    float cv = 0.f;
    if (g.border == SWC_BORDER_FILL && b.crosses) {
        fl = FL_BORDER;
    } else {
        const double n = (double)(b.r1 - b.r0 + 1) * (double)(b.c1 - b.c0 + 1);
        const double sx = S[0 * plane + i], sy = S[1 * plane + i];
        const double sxx = S[2 * plane + i], syy = S[3 * plane + i], sxy = S[4 * plane + i];
        if constexpr (FLOAT) {
            if (S[5 * plane + i] > 0.5) {
                fl = FL_MISSING;
            } else {
                const double N = __builtin_fma(n, sxy, -(sx * sy));
                const double Vx = __builtin_fma(n, sxx, -(sx * sx));
                const double Vy = __builtin_fma(n, syy, -(sy * sy));
                const double mx = (double)__uint_as_float(hdr[0]);
                const double my = (double)__uint_as_float(hdr[1]);
                const bool cert = (Vx > g.cert_g * mx * mx) && (Vy > g.cert_g * my * my) &&
                                  !(g.force & 1);
                if (cert)
                    cv = clamp_unit(N * rsqrt64(Vx * Vy));
                else
                    fl = twopass_window(xf, yf, (int64_t)g.W, 1, b.r0, b.r1, b.c0, b.c1, 0, 0, &cv);
            }
        } else {
            fl = final_int(n, sx, sy, sxx, syy, sxy, (g.force & 1) != 0, &cv);
        }
    }
    if (fl) cv = g.invalid;
    c[i] = cv;
    if (flags) flags[i] = fl;
}

// Cumulative sums along each row (one thread per row), channels formed from
// the inputs on the fly: I[r][j] = sum over t <= j of the channel at (r, t).
template <class T>
__global__ void __launch_bounds__(64)
cum_rows(const T* __restrict__ x, const T* __restrict__ y, uint64_t* __restrict__ I,
         int64_t plane, int H, int W)
{
    const int r = blockIdx.x * 64 + threadIdx.x;
    if (r >= H) return;
    uint64_t s[kChCum] = {0, 0, 0, 0, 0};
    const int64_t base = (int64_t)r * W;
    for (int j = 0; j < W; j++) {
        const uint64_t vx = (uint64_t)x[base + j], vy = (uint64_t)y[base + j];
        s[0] += vx;
        s[1] += vy;
        s[2] += vx * vx;
        s[3] += vy * vy;
        s[4] += vx * vy;
#pragma unroll
        for (int ch = 0; ch < kChCum; ch++) I[ch * plane + base + j] = s[ch];
    }
}

// Cumulative sums down each column, in place (one thread per column).
__global__ void __launch_bounds__(64)
cum_cols(uint64_t* __restrict__ I, int64_t plane, int H, int W)
{
    const int j = blockIdx.x * 64 + threadIdx.x;
    if (j >= W) return;
    uint64_t s[kChCum] = {0, 0, 0, 0, 0};
    for (int r = 0; r < H; r++) {
        const int64_t o = (int64_t)r * W + j;
#pragma unroll
        for (int ch = 0; ch < kChCum; ch++) {
            s[ch] += I[ch * plane + o];
            I[ch * plane + o] = s[ch];
        }
    }
}

// Window sums from four corners of the integral images, then step 4.
__global__ void __launch_bounds__(256)
cum_final(const uint64_t* __restrict__ I, int64_t plane, SchemeGeom g, float* __restrict__ c,
          uint8_t* __restrict__ flags)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= plane) return;
    const int r = (int)(i / g.W), j = (int)(i - (int64_t)r * g.W);
    const Box b = window_box(g, r, j);
    uint8_t fl = 0;
    float cv = 0.f;
    if (g.border == SWC_BORDER_FILL && b.crosses) {
        fl = FL_BORDER;
    } else {
        double S[kChCum];
        const int64_t a11 = (int64_t)b.r1 * g.W + b.c1;
        const int64_t a01 = (int64_t)(b.r0 - 1) * g.W + b.c1;
        const int64_t a10 = (int64_t)b.r1 * g.W + (b.c0 - 1);
        const int64_t a00 = (int64_t)(b.r0 - 1) * g.W + (b.c0 - 1);
#pragma unroll
        for (int ch = 0; ch < kChCum; ch++) {
            const uint64_t* P = I + ch * plane;
            uint64_t v = P[a11];
            if (b.r0 > 0) v -= P[a01];
            if (b.c0 > 0) v -= P[a10];
            if (b.r0 > 0 && b.c0 > 0) v += P[a00];
            S[ch] = (double)(int64_t)v;
        }
        const double n = (double)(b.r1 - b.r0 + 1) * (double)(b.c1 - b.c0 + 1);
        fl = final_int(n, S[0], S[1], S[2], S[3], S[4], (g.force & 1) != 0, &cv);
    }
    if (fl) cv = g.invalid;
    c[i] = cv;
    if (flags) flags[i] = fl;
}

inline int blocks_of(int64_t n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

bool scheme_supported(const swc_problem& p, int scheme)
{
    if (scheme != SWC_SCHEME_UNFUSED && scheme != SWC_SCHEME_CUMSUM) return false;
    if (p.ndim != 2 || p.step[0] != 1 || p.step[1] != 1) return false;
    if (p.border != SWC_BORDER_FILL && p.border != SWC_BORDER_CLIP) return false;
    if (p.accum != SWC_ACC_DEFAULT) return false;
    if (scheme == SWC_SCHEME_CUMSUM && p.dtype == SWC_F32) return false;
    // lines are indexed with int; grids stay below 2^31 blocks
    if (p.shape[0] >= ((int64_t)1 << 30) || p.shape[1] >= ((int64_t)1 << 30)) return false;
    if (p.shape[0] * p.shape[1] >= ((int64_t)1 << 38)) return false;
    return true;
}

uint64_t scheme_workspace_bytes(const swc_problem& p, int scheme)
{
    const uint64_t plane = (uint64_t)p.shape[0] * (uint64_t)p.shape[1];
    if (scheme == SWC_SCHEME_UNFUSED) return kHdrBytes + 2ull * kChUnf * plane * sizeof(double);
    return (uint64_t)kChCum * plane * sizeof(uint64_t);
}

hipError_t launch_scheme(const swc_problem& p, int scheme, const void* x, const void* y,
                         float* c, uint8_t* flags, void* ws, hipStream_t s, int force)
{
    SchemeGeom g;
    g.H = (int)p.shape[0];
    g.W = (int)p.shape[1];
    g.kh = p.window[0];
    g.kw = p.window[1];
    g.oh = window_offset(p.border, p.window[0]);
    g.ow = window_offset(p.border, p.window[1]);
    g.border = p.border;
    g.invalid = p.invalid_value;
    g.force = force;
    const int64_t plane = (int64_t)g.H * g.W;
    const int nb = blocks_of(plane, 256);
    if (scheme == SWC_SCHEME_CUMSUM) {
        uint64_t* I = (uint64_t*)ws;
        g.cert_g = 0.0;
        if (p.dtype == SWC_U8)
            SWC_TRY(launch_kernel(&cum_rows<uint8_t>, dim3(blocks_of(g.H, 64)), dim3(64), 0, s,
                               (const uint8_t*)x, (const uint8_t*)y, I, plane, g.H, g.W));
        else
            SWC_TRY(launch_kernel(&cum_rows<uint16_t>, dim3(blocks_of(g.H, 64)), dim3(64), 0, s,
                               (const uint16_t*)x, (const uint16_t*)y, I, plane, g.H, g.W));
        SWC_TRY(launch_kernel(&cum_cols, dim3(blocks_of(g.W, 64)), dim3(64), 0, s, I, plane, g.H, g.W));
        return launch_kernel(&cum_final, dim3(nb), dim3(256), 0, s, (const uint64_t*)I, plane, g, c,
                           flags);
    }
    uint32_t* hdr = (uint32_t*)ws;
    double* E = (double*)((char*)ws + kHdrBytes);   // products, then window sums
    double* A = E + kChUnf * plane;                 // row sums
    const float thr = missing_threshold(p.missing_le);
    // rounding-error factor: the row pass chains up to 2W operations, the
    // column pass up to 2H, over partial sums of at most (kh+1)(kw+1) terms
    const double chain = 2.0 * g.W + 2.0 * g.H + 4.0;
    const double nterms = (double)(g.kh + 1) * (g.kw + 1);
    g.cert_g = cert_factor(MODE_F64, (double)g.kh * g.kw, chain, nterms);
    SWC_TRY(launch_kernel(&unf_init, dim3(1), dim3(64), 0, s, hdr));
    if (p.dtype == SWC_U8)
        SWC_TRY(launch_kernel(&unf_products<uint8_t, false>, dim3(nb), dim3(256), 0, s,
                           (const uint8_t*)x, (const uint8_t*)y, E, plane, thr, hdr));
    else if (p.dtype == SWC_U16)
        SWC_TRY(launch_kernel(&unf_products<uint16_t, false>, dim3(nb), dim3(256), 0, s,
                           (const uint16_t*)x, (const uint16_t*)y, E, plane, thr, hdr));
    else
        SWC_TRY(launch_kernel(&unf_products<float, true>, dim3(nb), dim3(256), 0, s,
                           (const float*)x, (const float*)y, E, plane, thr, hdr));
    // step 2: one thread per row, moving sum along the row (E -> A)
    SWC_TRY(launch_kernel(&unf_moving_sum<kChUnf>, dim3(blocks_of(g.H, 64)), dim3(64), 0, s,
                       (const double*)E, A, plane, g.H, (int64_t)g.W, g.W, (int64_t)1, g.kw, -g.ow));
    // step 3: one thread per column, moving sum down the column (A -> E)
    SWC_TRY(launch_kernel(&unf_moving_sum<kChUnf>, dim3(blocks_of(g.W, 64)), dim3(64), 0, s,
                       (const double*)A, E, plane, g.W, (int64_t)1, g.H, (int64_t)g.W, g.kh, -g.oh));
    if (p.dtype == SWC_F32)
        return launch_kernel(&unf_final<true>, dim3(nb), dim3(256), 0, s, (const double*)E, plane, g,
                             (const float*)x, (const float*)y, (const uint32_t*)hdr, c, flags);
    return launch_kernel(&unf_final<false>, dim3(nb), dim3(256), 0, s, (const double*)E, plane, g,
                           nullptr, nullptr, (const uint32_t*)hdr, c, flags);
}

}  // namespace swc

// ---- the schemes without a caller workspace ----------------------------
// For callers that cannot allocate device memory (code under graph capture,
// tight serving loops): the workspace is a fixed array in device memory.
// Each device the library runs on holds its own copy until the process ends.
// Every call on a device uses that device's copy, so calls that overlap on
// one device (different streams, or threads) race; the array keeps the last
// call's contents, and each scheme initialises what it reads (the unfused
// scheme clears its header with a kernel; the cumulative sums overwrite
// every word they read).
static __device__ __align__(256) unsigned char scratch[SWC_SCHEME_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.  In host code the array's name is
// only a stand-in: kernels and copies take this address.
hipError_t scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" swc_status swc_corr_scheme_noalloc(const swc_problem* p, int32_t scheme, const void* x,
                                              const void* y, float* c, uint8_t* flags,
                                              void* stream)
{
    swc_status st = swc_validate(p);
    if (st != SWC_OK) return st;
    if (!x || !y || !c) return SWC_ERR_NULL;
    if (!swc::scheme_supported(*p, scheme)) return SWC_ERR_UNSUPPORTED;
    if (swc::scheme_workspace_bytes(*p, scheme) > (uint64_t)SWC_SCHEME_SCRATCH_BYTES)
        return SWC_ERR_WORKSPACE;
    if (swc::fault_inject_launch()) return SWC_ERR_LAUNCH;
    if (swc::sticky_error(hipPeekAtLastError())) return SWC_ERR_DEVICE;
    void* ws = nullptr;
    hipError_t e = scratch_address(&ws);
    if (e != hipSuccess) return swc::sticky_error(e) ? SWC_ERR_DEVICE : SWC_ERR_LAUNCH;
    e = swc::launch_scheme(*p, scheme, x, y, c, flags, ws, (hipStream_t)stream,
                           swc_get_debug() & 1);
    return swc::launch_status(e);
}
