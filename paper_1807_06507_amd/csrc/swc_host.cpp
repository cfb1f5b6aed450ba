// End-to-end host-to-host runs: the input pair is cut into slabs along the
// first axis, and each slab's host-to-device copies, fused kernel and
// device-to-host copy run in order on one of `depth` streams, so that the
// copies of one slab overlap the kernel of another.  This is the measured
// counterpart of the paper's end-to-end GPU time (Section 3), which includes
// the transfers to and from the device.
//
// Slab geometry (first axis, step 1): the outputs [o0, o1) of a slab need
// the input rows of their windows.  FILL/CLIP: window of output o is
// [o - L, o - L + k - 1] with L = floor(k/2), so the slab holds input rows
// [max(0, o0 - L), min(N, o1 - 1 - L + k)) (at most o1 - o0 + k - 1 rows,
// the staging size) and its same-size output row o - i0
// is the image's output row o: every such window lies inside the slab unless
// it is clipped by the image's own edge, which is then also the slab's edge.
// VALID: output o uses [o, o + k - 1]; the slab is [o0, o1 + k - 1) and its
// output o - o0 is the image's output o.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "swc_internal.h"

struct swc_host_plan {
    swc_problem p;
    int64_t oshape[3];
    int64_t band;          // output rows (first axis) per slab
    int depth;
    int64_t in_row;        // input elements per first-axis index
    int64_t out_row;       // output elements per first-axis index
    size_t esz;
    int device;            // the device current at creation (owns the buffers)
    std::vector<hipStream_t> streams;
    std::vector<void*> dx, dy, dc, df;   // per stream: staging buffers
};

namespace {

void slab_of(const swc_host_plan& P, int64_t o0, int64_t o1, int64_t& i0, int64_t& i1)
{
    const int64_t N = P.p.shape[0], k = P.p.window[0];
    if (P.p.border == SWC_BORDER_VALID) {
        i0 = o0;
        i1 = o1 + k - 1;
    } else {
        const int64_t L = k / 2;
        i0 = o0 - L > 0 ? o0 - L : 0;
        i1 = o1 - L + k - 1 < N ? o1 - L + k - 1 : N;
    }
}

// Host-side debug output (SWC_LOG=1), as in the rest of the library.
bool log_on()
{
    static const bool on = [] {
        const char* e = getenv("SWC_LOG");
        return e && e[0] == '1';
    }();
    return on;
}

bool ok_or_log(hipError_t e, const char* what, int64_t band)
{
    if (e == hipSuccess) return true;
    if (log_on()) fprintf(stderr, "[swcorr] host run, slab %lld: %s failed: %s\n",
                          (long long)band, what, hipGetErrorString(e));
    return false;
}

void free_plan(swc_host_plan* P)
{
    for (void* v : P->dx) (void)hipFree(v);
    for (void* v : P->dy) (void)hipFree(v);
    for (void* v : P->dc) (void)hipFree(v);
    for (void* v : P->df) (void)hipFree(v);
    for (hipStream_t s : P->streams) (void)hipStreamDestroy(s);
    delete P;
}

}  // namespace

extern "C" {

swc_status swc_host_plan_create(const swc_problem* p, int64_t band_rows, int32_t depth,
                                swc_host_plan** out)
{
    swc_status st = swc_validate(p);
    if (st != SWC_OK) return st;
    if (!out) return SWC_ERR_NULL;
    *out = nullptr;
    if (p->step[0] != 1) return SWC_ERR_UNSUPPORTED;
    if (band_rows < 1 || depth < 1 || depth > 8) return SWC_ERR_PARAM;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SWC_ERR_DEVICE;
    swc_host_plan* P = new swc_host_plan();
    P->p = *p;
    P->device = dev;
    swc_output_shape(p, P->oshape);
    P->band = band_rows < P->oshape[0] ? band_rows : P->oshape[0];
    P->depth = depth;
    P->esz = p->dtype == SWC_U8 ? 1 : (p->dtype == SWC_U16 ? 2 : 4);
    P->in_row = 1;
    P->out_row = 1;
    for (int d = 1; d < p->ndim; d++) {
        P->in_row *= p->shape[d];
        P->out_row *= P->oshape[d];
    }
    // the largest slab: band outputs plus k - 1 rows of halo
    int64_t rows_in = P->band + p->window[0] - 1;
    if (rows_in > p->shape[0]) rows_in = p->shape[0];
    // a slab must itself be a valid problem for the fused kernels
    swc_problem bp = *p;
    bp.shape[0] = rows_in;
    if (swc_validate(&bp) != SWC_OK) {
        delete P;
        return SWC_ERR_PARAM;
    }
    const size_t in_bytes = (size_t)rows_in * P->in_row * P->esz;
    const size_t out_elems = (size_t)rows_in * P->out_row;
    for (int i = 0; i < depth; i++) {
        hipStream_t s = nullptr;
        void *a = nullptr, *b = nullptr, *c = nullptr, *f = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            free_plan(P);
            return SWC_ERR_DEVICE;
        }
        P->streams.push_back(s);
        const bool ok = hipMalloc(&a, in_bytes) == hipSuccess && (P->dx.push_back(a), true) &&
                        hipMalloc(&b, in_bytes) == hipSuccess && (P->dy.push_back(b), true) &&
                        hipMalloc(&c, out_elems * 4) == hipSuccess && (P->dc.push_back(c), true) &&
                        hipMalloc(&f, out_elems) == hipSuccess && (P->df.push_back(f), true);
        if (!ok) {
            (void)hipGetLastError();
            free_plan(P);
            return SWC_ERR_DEVICE;
        }
    }
    *out = P;
    return SWC_OK;
}

swc_status swc_host_run(swc_host_plan* P, const void* x, const void* y, float* c,
                        uint8_t* flags)
{
    if (!P || !x || !y || !c) return SWC_ERR_NULL;
    // the staging buffers and streams belong to the plan's device
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != P->device) return SWC_ERR_DEVICE;
    const int64_t OH = P->oshape[0];
    const size_t ib = (size_t)P->in_row * P->esz;
    const size_t ob = (size_t)P->out_row;
    int64_t b = 0;
    swc_status st = SWC_OK;
    for (int64_t o0 = 0; o0 < OH && st == SWC_OK; o0 += P->band, b++) {
        const int64_t o1 = o0 + P->band < OH ? o0 + P->band : OH;
        int64_t i0, i1;
        slab_of(*P, o0, o1, i0, i1);
        const int slot = (int)(b % P->depth);
        hipStream_t s = P->streams[slot];
        swc_problem bp = P->p;
        bp.shape[0] = i1 - i0;
        // the slab's output row of image output o0
        const int64_t r0 = P->p.border == SWC_BORDER_VALID ? 0 : o0 - i0;
        if (!ok_or_log(hipMemcpyAsync(P->dx[slot], (const char*)x + i0 * ib, (i1 - i0) * ib,
                                      hipMemcpyHostToDevice, s), "copy of x", b) ||
            !ok_or_log(hipMemcpyAsync(P->dy[slot], (const char*)y + i0 * ib, (i1 - i0) * ib,
                                      hipMemcpyHostToDevice, s), "copy of y", b)) {
            st = SWC_ERR_DEVICE;
            break;
        }
        st = swc_corr(&bp, P->dx[slot], P->dy[slot], (float*)P->dc[slot],
                      flags ? (uint8_t*)P->df[slot] : nullptr, s);
        if (st != SWC_OK) {
            if (log_on()) fprintf(stderr, "[swcorr] host run, slab %lld: swc_corr: %s\n",
                                  (long long)b, swc_status_str(st));
            break;
        }
        if (!ok_or_log(hipMemcpyAsync(c + o0 * ob, (const float*)P->dc[slot] + r0 * ob,
                                      (o1 - o0) * ob * 4, hipMemcpyDeviceToHost, s), "copy of c", b) ||
            (flags && !ok_or_log(hipMemcpyAsync(flags + o0 * ob, (const uint8_t*)P->df[slot] + r0 * ob,
                                                (o1 - o0) * ob, hipMemcpyDeviceToHost, s),
                                 "copy of flags", b))) {
            st = SWC_ERR_DEVICE;
            break;
        }
    }
    // drain every stream, also after an error, before returning
    for (hipStream_t s : P->streams)
        if (!ok_or_log(hipStreamSynchronize(s), "stream synchronize", -1) && st == SWC_OK)
            st = SWC_ERR_DEVICE;
    return st;
}

int64_t swc_host_plan_bands(const swc_host_plan* P)
{
    if (!P) return 0;
    return (P->oshape[0] + P->band - 1) / P->band;
}

void swc_host_plan_destroy(swc_host_plan* P)
{
    if (!P) return;
    for (hipStream_t s : P->streams) (void)hipStreamSynchronize(s);
    free_plan(P);
}

}  // extern "C"
