// C ABI of libswcorr.so: argument validation, output geometry, tuned launch
// parameters and dispatch to the gfx950 kernels.  See include/swcorr.h.
#include <dlfcn.h>
#include <float.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "swc_internal.h"

namespace swc {

int mode_of(int32_t dtype, int32_t accum)
{
    switch (dtype) {
    case SWC_U8: return accum == SWC_ACC_DEFAULT ? 0 : -1;
    case SWC_U16: return accum == SWC_ACC_DEFAULT ? 1 : -1;
    case SWC_F32:
        if (accum == SWC_ACC_DEFAULT) return 2;
        if (accum == SWC_ACC_NAIVE_F32) return 3;
        if (accum == SWC_ACC_COMP_F32) return 4;
        return -1;
    default: return -1;
    }
}

float missing_threshold(double t)
{
    if (isinf(t) && t < 0) return -INFINITY;
    if (t >= (double)FLT_MAX) return FLT_MAX;
    if (t <= -(double)FLT_MAX) return -FLT_MAX;   // only -Inf/NaN below it
    float f = (float)t;
    if ((double)f > t) f = nextafterf(f, -INFINITY);
    return f;
}

double cert_factor(int mode, double n, double chain, double nterms)
{
    // unit roundoff of the sliding sums.  FP64 sums: 2^-53 per operation.
    // Compensated FP32 pairs (hi, lo): every TwoSum is exact, its error term
    // is at most 2^-24 of the partial sum, so |lo| stays below 2 C 2^-24 P
    // over a chain of C operations on partial sums bounded by P (product
    // tails included), and each of the 2C roundings of lo costs at most
    // 2^-24 |lo|: in all 4 C^2 2^-48 P, i.e. a per-operation roundoff of
    // C 2^-46 in the bound below
    const double u = (mode == 4) ? chain * ldexp(1.0, -46) : ldexp(1.0, -53);
    const double rho = 4096.0;   // fast path only when |dc| <= 2/(rho-1)
    const double g = u * n * (3.0 * chain * nterms + 6.0 * n) * (1.0 + ldexp(1.0, -10));
    return rho * g;
}

swc_status launch_status(hipError_t e)
{
    if (e == hipSuccess) return SWC_OK;
    return sticky_error(e) ? SWC_ERR_DEVICE : SWC_ERR_LAUNCH;
}

}  // namespace swc

using namespace swc;

namespace {

// Window-size limits (exactness of the integer paths; kernel reach).
constexpr int64_t kMaxWindowU16 = 1448;    // n^2 (2^16-1)^2 < 2^53
constexpr int64_t kMaxWindowU8 = 33025;    // n (2^8-1)^2 < 2^31

int g_debug = 0;
bool g_fault_launch = false;
std::once_flag g_init_once;
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, swc_launch_params> g_tune;
bool g_log = false;

int kbucket(const swc_problem* p)
{
    int kmax = 1;
    for (int d = 0; d < p->ndim; d++) kmax = p->window[d] > kmax ? p->window[d] : kmax;
    if (kmax <= 3) return 3;
    if (kmax <= 5) return 5;
    if (kmax <= 7) return 7;
    if (kmax <= 9) return 9;
    if (kmax <= 15) return 15;
    if (kmax <= 31) return 31;
    if (kmax <= 63) return 63;
    return 1 << 30;
}

void load_tune_file(const char* path)
{
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#') continue;
        int dt, nd, ac, kb, R, TH, wpb, minw, ty = 0;
        if (sscanf(line, "%d %d %d %d %d %d %d %d %d", &dt, &nd, &ac, &kb, &R, &TH, &wpb, &minw,
                   &ty) >= 8) {
            swc_launch_params lp;
            memset(&lp, 0, sizeof lp);
            lp.cols_per_lane = R;
            lp.tile_rows = TH;
            lp.waves_per_block = wpb;
            lp.min_waves_per_eu = minw;
            lp.tile_rows2 = ty;
            g_tune[std::make_tuple(dt, nd, ac, kb)] = lp;
        }
    }
    fclose(f);
    if (g_log) fprintf(stderr, "[swcorr] loaded tuning table %s (%zu entries)\n", path, g_tune.size());
}

void init_once()
{
    const char* lg = getenv("SWC_LOG");
    g_log = lg && lg[0] == '1';
    const char* fe = getenv("SWC_FORCE_EXACT_FALLBACK");
    if (fe && fe[0] == '1') g_debug |= 1;
    const char* fi = getenv("SWC_FAULT_INJECT");
    g_fault_launch = fi && strcmp(fi, "launch") == 0;
    // tuning table: SWC_TUNE_TABLE, else tune_table.txt next to the library
    const char* tt = getenv("SWC_TUNE_TABLE");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (tt && tt[0]) {
        load_tune_file(tt);
    } else {
        Dl_info info;
        if (dladdr((void*)&init_once, &info) && info.dli_fname) {
            std::string so(info.dli_fname);
            size_t slash = so.find_last_of('/');
            std::string dir = slash == std::string::npos ? std::string(".") : so.substr(0, slash);
            load_tune_file((dir + "/tune_table.txt").c_str());
        }
    }
}

void ensure_init() { std::call_once(g_init_once, init_once); }

LaunchCfg default_cfg(const swc_problem* p)
{
    LaunchCfg L;
    L.minw = 0;
    if (p->ndim == 2) {
        L.R = 4;
        L.TH = 0;     // tile height chosen per launch from the resident-wave count
        L.wpb = 4;
        if (p->window[1] > 4 * 64 - 3) L.R = 8;
    } else if (p->ndim == 1) {
        L.R = 8;
        L.TH = 64;
        L.wpb = 2;
    } else {
        L.R = 4;
        L.TH = 32;
        L.wpb = 2;
        L.TY = 2;
    }
    return L;
}

LaunchCfg cfg_from_params(const swc_launch_params* lp)
{
    LaunchCfg L;
    L.R = lp->cols_per_lane;
    L.TH = lp->tile_rows;
    L.wpb = lp->waves_per_block;
    L.minw = lp->min_waves_per_eu;
    L.TY = lp->tile_rows2;
    return L;
}

bool cfg_ok(const swc_problem* p, const LaunchCfg& L)
{
    if (p->ndim == 1) return cfg_ok_1d(*p, L);
    if (p->ndim == 2) return cfg_ok_2d(*p, L);
    return cfg_ok_3d(*p, L);
}

LaunchCfg resolve_cfg(const swc_problem* p)
{
    ensure_init();
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(std::make_tuple(p->dtype, p->ndim, p->accum, kbucket(p)));
        if (it != g_tune.end()) {
            LaunchCfg L = cfg_from_params(&it->second);
            if (cfg_ok(p, L)) return L;
        }
    }
    LaunchCfg L = default_cfg(p);
    if (!cfg_ok(p, L)) {
        // widen the per-lane run until the window fits
        for (int R : {1, 2, 4, 8}) {
            L.R = R;
            if (cfg_ok(p, L)) break;
        }
    }
    return L;
}

}  // namespace

namespace swc {
bool fault_inject_launch()
{
    ensure_init();
    return g_fault_launch;
}

// Launch configuration of one pair computed outside a persistent batch.
LaunchCfg batch_pair_cfg(const swc_problem& p) { return resolve_cfg(&p); }

// Tuning-table lookup by raw key (the batch plan uses kbucket 0).
bool tune_lookup(int dtype, int ndim, int accum, int kb, swc_launch_params* out)
{
    ensure_init();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(std::make_tuple(dtype, ndim, accum, kb));
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}
}  // namespace swc

extern "C" {

int32_t swc_version(void) { return SWC_VERSION_MAJOR * 100 + SWC_VERSION_MINOR; }

const char* swc_status_str(swc_status s)
{
    switch (s) {
    case SWC_OK: return "ok";
    case SWC_ERR_NULL: return "null pointer argument";
    case SWC_ERR_NDIM: return "ndim must be 1, 2 or 3";
    case SWC_ERR_SHAPE: return "invalid shape (must be >= 1; VALID needs shape >= window)";
    case SWC_ERR_WINDOW: return "invalid window (must be >= 1 and within the supported limits)";
    case SWC_ERR_STEP: return "invalid step (must be >= 1)";
    case SWC_ERR_DTYPE: return "unknown dtype";
    case SWC_ERR_BORDER: return "unknown border policy";
    case SWC_ERR_ACCUM: return "unknown accumulation mode or not valid for the dtype";
    case SWC_ERR_WORKSPACE: return "workspace too small";
    case SWC_ERR_LAUNCH: return "kernel launch failed";
    case SWC_ERR_DEVICE: return "device error";
    case SWC_ERR_UNSUPPORTED: return "request not supported by this build";
    case SWC_ERR_PARAM: return "invalid launch parameters";
    default: return "unknown status";
    }
}

swc_status swc_validate(const swc_problem* p)
{
    if (!p) return SWC_ERR_NULL;
    if (p->ndim < 1 || p->ndim > 3) return SWC_ERR_NDIM;
    if (p->dtype < SWC_U8 || p->dtype > SWC_F32) return SWC_ERR_DTYPE;
    if (p->border < SWC_BORDER_FILL || p->border > SWC_BORDER_VALID) return SWC_ERR_BORDER;
    if (mode_of(p->dtype, p->accum) < 0) return SWC_ERR_ACCUM;
    if (p->reserved0 != 0) return SWC_ERR_UNSUPPORTED;
    if (isnan(p->missing_le)) return SWC_ERR_UNSUPPORTED;
    int64_t total = 1, n = 1;
    for (int d = 0; d < p->ndim; d++) {
        if (p->shape[d] < 1) return SWC_ERR_SHAPE;
        if (p->shape[d] > ((int64_t)1 << 40)) return SWC_ERR_SHAPE;
        total *= p->shape[d];
        if (total > ((int64_t)1 << 40)) return SWC_ERR_SHAPE;
    }
    for (int d = 0; d < p->ndim; d++) {
        if (p->window[d] < 1) return SWC_ERR_WINDOW;
        if (p->window[d] > (1 << 24)) return SWC_ERR_WINDOW;
        n *= p->window[d];
        if (n > ((int64_t)1 << 40)) return SWC_ERR_WINDOW;
    }
    for (int d = 0; d < p->ndim; d++) {
        if (p->step[d] < 1) return SWC_ERR_STEP;
    }
    if (p->border == SWC_BORDER_VALID) {
        for (int d = 0; d < p->ndim; d++)
            if (p->shape[d] < p->window[d]) return SWC_ERR_SHAPE;
    }
    if (p->dtype == SWC_U16 && n > kMaxWindowU16) return SWC_ERR_WINDOW;
    if (p->dtype == SWC_U8 && n > kMaxWindowU8) return SWC_ERR_WINDOW;
    return SWC_OK;
}

swc_status swc_output_shape(const swc_problem* p, int64_t out[3])
{
    swc_status st = swc_validate(p);
    if (st != SWC_OK) return st;
    if (!out) return SWC_ERR_NULL;
    for (int d = 0; d < 3; d++) out[d] = 1;
    for (int d = 0; d < p->ndim; d++) {
        const int64_t N = p->shape[d], k = p->window[d], s = p->step[d];
        out[d] = p->border == SWC_BORDER_VALID ? (N - k) / s + 1 : (N + s - 1) / s;
    }
    return SWC_OK;
}

void swc_set_debug(int32_t bits)
{
    ensure_init();
    g_debug = bits;
}

int32_t swc_get_debug(void)
{
    ensure_init();
    return g_debug;
}

swc_status swc_tune_set(const swc_problem* p, const swc_launch_params* lp)
{
    swc_status st = swc_validate(p);
    if (st != SWC_OK) return st;
    if (!lp) return SWC_ERR_NULL;
    LaunchCfg L = cfg_from_params(lp);
    if (!cfg_ok(p, L)) return SWC_ERR_PARAM;
    ensure_init();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[std::make_tuple(p->dtype, p->ndim, p->accum, kbucket(p))] = *lp;
    return SWC_OK;
}

swc_status swc_tune_get(const swc_problem* p, swc_launch_params* lp)
{
    swc_status st = swc_validate(p);
    if (st != SWC_OK) return st;
    if (!lp) return SWC_ERR_NULL;
    LaunchCfg L = resolve_cfg(p);
    memset(lp, 0, sizeof *lp);
    lp->cols_per_lane = L.R;
    lp->tile_rows = L.TH;
    lp->waves_per_block = L.wpb;
    lp->min_waves_per_eu = L.minw;
    lp->tile_rows2 = L.TY;
    return cfg_ok(p, L) ? SWC_OK : SWC_ERR_UNSUPPORTED;
}

swc_status swc_corr_ex(const swc_problem* p, const swc_launch_params* lp, const void* x,
                       const void* y, float* c, uint8_t* flags, void* stream)
{
    swc_status st = swc_validate(p);
    if (st != SWC_OK) return st;
    if (!x || !y || !c) return SWC_ERR_NULL;
    ensure_init();
    LaunchCfg L;
    if (lp && (lp->cols_per_lane || lp->tile_rows || lp->waves_per_block)) {
        L = cfg_from_params(lp);
        if (p->ndim == 3 && L.TY == 0) L.TY = 2;
        if (!cfg_ok(p, L)) return SWC_ERR_PARAM;
    } else {
        L = resolve_cfg(p);
        if (!cfg_ok(p, L)) return SWC_ERR_UNSUPPORTED;
    }
    int64_t osh[3];
    swc_output_shape(p, osh);
    hipStream_t s = (hipStream_t)stream;
    if (fault_inject_launch()) return SWC_ERR_LAUNCH;
    // a device fault left by earlier work makes every launch fail: report it
    // as such (without clearing it; other pending errors belong to whoever
    // caused them, and launches report their own status)
    if (sticky_error(hipPeekAtLastError())) return SWC_ERR_DEVICE;
    hipError_t e;
    // bit 0: exact fallbacks; bit 1: generic 2-D kernel / general 3-D step;
    // bit 2: 1-D re-reads leaving values instead of its LDS ring; bit 3: the
    // compensated comparator skips its certification
    const int force = g_debug & 15;
    if (p->ndim == 1) e = launch_corr1d(*p, osh, L, x, y, c, flags, s, force);
    else if (p->ndim == 2) e = launch_corr2d(*p, osh, L, x, y, c, flags, s, force);
    else e = launch_corr3d(*p, osh, L, x, y, c, flags, s, force);
    if (e != hipSuccess) {
        if (g_log) fprintf(stderr, "[swcorr] launch failed: %s\n", hipGetErrorString(e));
        return launch_status(e);
    }
    if (g_log)
        fprintf(stderr, "[swcorr] ndim=%d dtype=%d R=%d TH=%d wpb=%d\n", p->ndim, p->dtype, L.R,
                L.TH, L.wpb);
    return SWC_OK;
}

swc_status swc_corr(const swc_problem* p, const void* x, const void* y, float* c,
                    uint8_t* flags, void* stream)
{
    return swc_corr_ex(p, nullptr, x, y, c, flags, stream);
}

swc_status swc_cloud_mask(const float* c, const uint8_t* flags, int64_t n, float tau,
                          float invalid_value, uint8_t* mask, void* stream)
{
    if (n < 0) return SWC_ERR_SHAPE;
    if (isnan(tau)) return SWC_ERR_PARAM;
    if (n == 0) return SWC_OK;
    if (!c || !mask) return SWC_ERR_NULL;
    if (fault_inject_launch()) return SWC_ERR_LAUNCH;
    if (sticky_error(hipPeekAtLastError())) return SWC_ERR_DEVICE;
    hipError_t e = launch_cloud_mask(c, flags, n, tau, invalid_value, mask, (hipStream_t)stream);
    return launch_status(e);
}

swc_status swc_filter_detections(const float* c, const uint8_t* flags, int64_t n,
                                 const int64_t* idx, int64_t k, float tau, float invalid_value,
                                 uint8_t* keep, void* stream)
{
    if (n < 0 || k < 0) return SWC_ERR_SHAPE;
    if (isnan(tau)) return SWC_ERR_PARAM;
    if (k == 0) return SWC_OK;
    if (!idx || !keep || (n > 0 && !c)) return SWC_ERR_NULL;
    if (fault_inject_launch()) return SWC_ERR_LAUNCH;
    if (sticky_error(hipPeekAtLastError())) return SWC_ERR_DEVICE;
    hipError_t e = launch_filter_detections(c, flags, n, idx, k, tau, invalid_value, keep,
                                            (hipStream_t)stream);
    return launch_status(e);
}

swc_status swc_scheme_workspace(const swc_problem* p, int32_t scheme, uint64_t* bytes)
{
    swc_status st = swc_validate(p);
    if (st != SWC_OK) return st;
    if (!bytes) return SWC_ERR_NULL;
    if (!scheme_supported(*p, scheme)) return SWC_ERR_UNSUPPORTED;
    *bytes = scheme_workspace_bytes(*p, scheme);
    return SWC_OK;
}

swc_status swc_corr_scheme(const swc_problem* p, int32_t scheme, const void* x, const void* y,
                           float* c, uint8_t* flags, void* workspace, uint64_t workspace_bytes,
                           void* stream)
{
    swc_status st = swc_validate(p);
    if (st != SWC_OK) return st;
    if (!x || !y || !c || !workspace) return SWC_ERR_NULL;
    if (!scheme_supported(*p, scheme)) return SWC_ERR_UNSUPPORTED;
    if (workspace_bytes < scheme_workspace_bytes(*p, scheme) || ((uintptr_t)workspace % 8) != 0)
        return SWC_ERR_WORKSPACE;
    ensure_init();
    if (fault_inject_launch()) return SWC_ERR_LAUNCH;
    if (sticky_error(hipPeekAtLastError())) return SWC_ERR_DEVICE;
    hipError_t e = launch_scheme(*p, scheme, x, y, c, flags, workspace, (hipStream_t)stream,
                                 g_debug & 1);
    if (e != hipSuccess) {
        if (g_log) fprintf(stderr, "[swcorr] scheme launch failed: %s\n", hipGetErrorString(e));
        return launch_status(e);
    }
    return SWC_OK;
}

}  // extern "C"
