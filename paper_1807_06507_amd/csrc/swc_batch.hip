// Batched correlation of many independent 2-D pairs in persistent launches.
//
// A plan turns n problems (different shapes, windows, steps, borders) into
// lists of tiles: in a list, the tiles of pair i occupy [tile0_i, tile0_i + n_i).
// The device holds one descriptor per pair (the same tile geometry the
// single-pair register kernel uses).  One launch of a fixed, fully resident
// grid of wavefronts walks a list: each wave takes the next item from a
// counter in device memory, finds the pair by binary search over tile0 and
// runs the tile with the kernel variant of that pair's window width.  A launch reserves, for every
// wave, the LDS ring of its widest window, which caps the resident waves per
// CU; pairs are therefore grouped by that cap (at most four groups, each one
// persistent launch), so narrow windows are not held to the occupancy of the
// widest.  Within a list pairs are ordered by (window, alignment) so that
// waves running at the same time mostly share one code path.  Pairs without a
// compiled variant are computed by their own launches, issued by the same
// swc_batch_launch call (still capture-safe: no allocation, copy or
// synchronisation).
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <vector>

#include "swc_corr2d_fast.hpp"
#include "swc_internal.h"

namespace swc {

struct BatchItem {
    P2DF g;
    int64_t tile0;
    int kw;
    int vec;
    int lds;      // LDS bytes this pair's tiles need per wave
    int pad;
};

constexpr int kBatchR = 4;

template <int M, int KW>
__device__ __forceinline__ void batch_tile(const P2DF& g, int vec, int tile, char* lds)
{
    if (vec) tile2d<M, kBatchR, KW, true, false>(g, tile, lds);
    else tile2d<M, kBatchR, KW, false, false>(g, tile, lds);
}

template <int M>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(2, 8))) corr2d_batch_kernel(const BatchItem* __restrict__ items,
                                                                int n, int64_t total,
                                                                int lds_stride, int* ctr)
{
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
    char* lds = smem + (size_t)wv * lds_stride;
    // Work items are handed out in list order through a counter in device
    // memory (ctr[0]), so a wave that started late or drew cheap tiles takes
    // more of them and the waves finish together.  Waves sharing a SIMD are
    // issued oldest first; priorities fall from 3 to 0 as the list is used
    // up, so that the waves of a SIMD keep pace.  The last wave to leave
    // (ctr[1] counts them) sets both counters back to zero for the next
    // launch, so the plan needs no clearing between launches or graph
    // replays.
    const int lane = threadIdx.x & (kWave - 1);
    for (;;) {
        int got = 0;
        if (lane == 0) got = atomicAdd(&ctr[0], 1);
        const int64_t it = __builtin_amdgcn_readfirstlane(got);
        if (it >= total) break;
        const int64_t q4 = 4 * it;
        if (q4 < total) __builtin_amdgcn_s_setprio(3);
        else if (q4 < 2 * total) __builtin_amdgcn_s_setprio(2);
        else if (q4 < 3 * total) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
        // pair owning item `it` (wave-uniform)
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (items[mid].tile0 <= it) lo = mid;
            else hi = mid - 1;
        }
        const BatchItem& b = items[lo];
        const P2DF g = b.g;
        const int tile = (int)(it - b.tile0);
        switch (b.kw) {
        case 3: batch_tile<M, 3>(g, b.vec, tile, lds); break;
        case 5: batch_tile<M, 5>(g, b.vec, tile, lds); break;
        case 7: batch_tile<M, 7>(g, b.vec, tile, lds); break;
        case 9: batch_tile<M, 9>(g, b.vec, tile, lds); break;
        case 15: batch_tile<M, 15>(g, b.vec, tile, lds); break;
        default: break;
        }
    }
    if (lane == 0) {
        const int nl = (int)(gridDim.x * (blockDim.x / kWave));
        if (atomicAdd(&ctr[1], 1) == nl - 1) {
            atomicExch(&ctr[0], 0);
            atomicExch(&ctr[1], 0);
        }
    }
}

static bool batch_kw_ok(int kw) { return kw == 3 || kw == 5 || kw == 7 || kw == 9 || kw == 15; }

}  // namespace swc

using namespace swc;

// One persistent launch: a list of pairs with a common LDS stride.
struct BatchGroup {
    const BatchItem* d_items;    // into the plan's allocation
    int n_items;
    int64_t total_tiles;
    int lds_stride;
    int wpb;
    int64_t nwaves;
};

struct swc_batch_plan {
    int mode;
    std::vector<BatchGroup> groups;
    int64_t total_tiles;
    BatchItem* d_items;          // device, owned (all groups' lists, concatenated)
    int* d_ctr;                  // device, owned: next work item, waves finished
    // pairs computed by their own launches
    std::vector<swc_problem> rest_p;
    std::vector<std::array<const void*, 2>> rest_xy;
    std::vector<float*> rest_c;
    std::vector<uint8_t*> rest_f;
    std::vector<std::array<int64_t, 3>> rest_osh;
    std::vector<LaunchCfg> rest_cfg;
    int device;
};

namespace swc {
// default per-pair configuration chooser (shared with the single-pair path)
LaunchCfg batch_pair_cfg(const swc_problem& p);
bool tune_lookup(int dtype, int ndim, int accum, int kb, swc_launch_params* out);
}

namespace {

// Resident workgroups per CU of the batch kernel for a launch shape.
int batch_blocks_per_cu(int mode, int wpb, size_t smem)
{
    int n = 0;
    hipError_t e;
    if (mode == MODE_U8)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, corr2d_batch_kernel<MODE_U8>,
                                                         wpb * kWave, smem);
    else if (mode == MODE_U16)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, corr2d_batch_kernel<MODE_U16>,
                                                         wpb * kWave, smem);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, corr2d_batch_kernel<MODE_F64>,
                                                         wpb * kWave, smem);
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

extern "C" {

swc_status swc_batch_plan_create(int32_t n, const swc_problem* p, const void* const* x,
                                 const void* const* y, float* const* c, uint8_t* const* flags,
                                 const swc_launch_params* lp, swc_batch_plan** out)
{
    if (!out) return SWC_ERR_NULL;
    *out = nullptr;
    if (n < 1) return SWC_ERR_SHAPE;
    if (!p || !x || !y || !c) return SWC_ERR_NULL;
    const int mode = mode_of(p[0].dtype, p[0].accum);
    for (int i = 0; i < n; i++) {
        swc_status st = swc_validate(&p[i]);
        if (st != SWC_OK) return st;
        if (p[i].ndim != 2) return SWC_ERR_NDIM;
        if (p[i].dtype != p[0].dtype) return SWC_ERR_DTYPE;
        if (p[i].accum != p[0].accum) return SWC_ERR_ACCUM;
        if (!x[i] || !y[i] || !c[i]) return SWC_ERR_NULL;
    }
    int TH = 0, wpb = 0, minw = 0;   // 0: chosen below
    swc_launch_params tuned;
    auto given = [](const swc_launch_params* q) {
        return q && (q->tile_rows || q->waves_per_block || q->min_waves_per_eu);
    };
    if (!given(lp) && tune_lookup(p[0].dtype, 2, p[0].accum, 0, &tuned)) lp = &tuned;
    if (given(lp)) {
        if (lp->cols_per_lane && lp->cols_per_lane != kBatchR) return SWC_ERR_PARAM;
        TH = lp->tile_rows;
        wpb = lp->waves_per_block;
        minw = lp->min_waves_per_eu;
        if (TH < 0 || TH > 4096 || !(wpb == 0 || wpb == 1 || wpb == 2 || wpb == 4) ||
            minw < 0 || minw > 8)
            return SWC_ERR_PARAM;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SWC_ERR_DEVICE;
    int cus = 256;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);

    // vector row loads for pair i (the tile code's VEC variant)
    auto vec_of = [&](int i) {
        const size_t esz = p[i].dtype == SWC_U8 ? 1 : (p[i].dtype == SWC_U16 ? 2 : 4);
        const size_t va = esz * kBatchR;
        if (esz == 4) return ((uintptr_t)x[i] % 4 == 0 && (uintptr_t)y[i] % 4 == 0) ? 1 : 0;
        return ((uintptr_t)x[i] % va == 0 && (uintptr_t)y[i] % va == 0 &&
                p[i].shape[1] % kBatchR == 0) ? 1 : 0;
    };
    // LDS bytes per wave of pair i's tiles: its row ring (none for wide windows)
    auto lds_of = [&](int i) {
        return (fast2d_lds_per_wave(mode, kBatchR, p[i].window[0], p[i].window[1],
                                    vec_of(i) != 0) + 15) & ~15;
    };
    // pairs the persistent kernel takes (the others run as separate launches)
    auto eligible = [&](int i) {
        return (mode == MODE_U8 || mode == MODE_U16 || mode == MODE_F64) &&
               batch_kw_ok(p[i].window[1]) && p[i].shape[0] < (1ll << 30) &&
               p[i].shape[1] < (1ll << 28) &&   // rows are raw buffers (< 2^31 bytes)
               lds_of(i) <= 64 * 1024;
    };
    // per pair: the resident waves per CU its LDS ring allows; pairs with the
    // same cap share one persistent launch
    int lds_cu = 160 * 1024;
    hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
    auto cap_of = [&](int i) {
        const int l = lds_of(i);
        return l > 0 ? std::min(8, std::max(1, lds_cu / l)) : 8;
    };
    int64_t tile_rows_total = 0;   // sum over pairs of output rows x tile columns
    for (int i = 0; i < n; i++) {
        if (!eligible(i)) continue;
        int64_t osh[3];
        swc_output_shape(&p[i], osh);
        const bool contig = p[i].step[1] == 1 && p[i].border != SWC_BORDER_VALID;
        const int wq = contig ? fast2d_wq_aligned(kBatchR, p[i].window[1])
                              : (kWave * kBatchR - (kBatchR - 1) - p[i].window[1]) / p[i].step[1] + 1;
        tile_rows_total += osh[0] * ((osh[1] + wq - 1) / wq);
    }
    // persistent grid: a few waves per SIMD at most
    const int64_t target = (int64_t)cus * 4 * (minw > 0 ? minw : 2);
    // tile height: about four tiles per persistent wave, 16..128 rows
    if (TH == 0)
        TH = (int)std::min<int64_t>(128, std::max<int64_t>(16, tile_rows_total / (4 * target)));
    const int wpb_req = wpb == 0 ? 4 : wpb;

    swc_batch_plan* plan = new swc_batch_plan();
    plan->mode = mode;
    plan->device = dev;
    std::vector<BatchItem> items;
    std::vector<int> order(n);
    for (int i = 0; i < n; i++) order[i] = i;
    // groups by occupancy cap (lowest first); inside a group widest windows
    // first (their tiles cost the most, so the tail of the persistent loop is
    // made of cheap tiles), then by alignment so concurrent waves share code
    std::vector<int> cap(n, 8);
    for (int i = 0; i < n; i++)
        if (eligible(i)) cap[i] = cap_of(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (cap[a] != cap[b]) return cap[a] < cap[b];
        if (p[a].window[1] != p[b].window[1]) return p[a].window[1] > p[b].window[1];
        return vec_of(a) > vec_of(b);
    });
    // at most four groups: caps beyond the fourth distinct value join the last
    std::vector<int> group_of(n, 0);
    {
        int g = -1, last_cap = -1;
        for (int oi = 0; oi < n; oi++) {
            const int i = order[oi];
            if (!eligible(i)) continue;
            if (cap[i] != last_cap && g < 3) {
                ++g;
                last_cap = cap[i];
            }
            group_of[i] = g;
        }
    }
    std::vector<int> gstart;       // first item index of each group
    std::vector<int64_t> gtiles;
    std::vector<int> glds;
    int64_t tile0 = 0;
    int cur_group = -1;
    for (int oi = 0; oi < n; oi++) {
        const int i = order[oi];
        const swc_problem& q = p[i];
        int64_t osh[3];
        swc_output_shape(&q, osh);
        const bool fast = eligible(i);
        if (!fast) {
            plan->rest_p.push_back(q);
            plan->rest_xy.push_back({x[i], y[i]});
            plan->rest_c.push_back(c[i]);
            plan->rest_f.push_back(flags ? flags[i] : nullptr);
            plan->rest_osh.push_back({osh[0], osh[1], osh[2]});
            plan->rest_cfg.push_back(batch_pair_cfg(q));
            continue;
        }
        if (group_of[i] != cur_group) {
            cur_group = group_of[i];
            gstart.push_back((int)items.size());
            gtiles.push_back(0);
            glds.push_back(0);
            tile0 = 0;
        }
        BatchItem b;
        memset(&b, 0, sizeof b);
        P2DF& g = b.g;
        g.x = x[i];
        g.y = y[i];
        g.c = c[i];
        g.flags = flags ? flags[i] : nullptr;
        g.H = (int)q.shape[0];
        g.W = (int)q.shape[1];
        g.OH = (int)osh[0];
        g.OW = (int)osh[1];
        g.kh = q.window[0];
        g.sh = q.step[0];
        g.sw = q.step[1];
        g.oh = window_offset(q.border, q.window[0]);
        g.ow = window_offset(q.border, q.window[1]);
        g.border = q.border;
        g.invalid = q.invalid_value;
        g.miss_thr = missing_threshold(q.missing_le);
        g.force = 0;
        g.TH = TH;
        const bool contig = q.step[1] == 1 && g.ow == -(q.window[1] / 2);
        g.vst = (contig && g.OW % 4 == 0 && (uintptr_t)c[i] % 16 == 0 ? 1 : 0) |
                (contig && g.flags && g.OW % kBatchR == 0 &&
                 (uintptr_t)g.flags % kBatchR == 0 ? 2 : 0);
        const int span = kWave * kBatchR - (kBatchR - 1);
        g.Wq = contig ? fast2d_wq_aligned(kBatchR, q.window[1])
                      : (span - q.window[1]) / q.step[1] + 1;
        const int tiles_x = (int)((osh[1] + g.Wq - 1) / g.Wq);
        g.tiles_y = (int)((osh[0] + TH - 1) / TH);
        g.n_tiles = tiles_x * g.tiles_y;
        const double th_ext = (double)(TH - 1) * q.step[0] + q.window[0];
        // the same bound as the single-pair launch of this tile code
        g.cert_g = fast2d_cert(mode, kBatchR, q.window[0], q.window[1], th_ext);
        b.tile0 = tile0;
        b.kw = q.window[1];
        b.vec = vec_of(i);
        b.lds = lds_of(i);
        glds.back() = std::max(glds.back(), b.lds);
        tile0 += g.n_tiles;
        gtiles.back() = tile0;
        items.push_back(b);
    }
    plan->d_items = nullptr;
    plan->d_ctr = nullptr;
    // the work-list counters (zero at rest; each launch leaves them at zero)
    if (hipMalloc((void**)&plan->d_ctr, 2 * sizeof(int)) != hipSuccess) {
        delete plan;
        return SWC_ERR_DEVICE;
    }
    if (hipMemset(plan->d_ctr, 0, 2 * sizeof(int)) != hipSuccess) {
        hipFree(plan->d_ctr);
        delete plan;
        return SWC_ERR_DEVICE;
    }
    plan->total_tiles = 0;
    if (!items.empty()) {
        if (hipMalloc((void**)&plan->d_items, items.size() * sizeof(BatchItem)) != hipSuccess) {
            hipFree(plan->d_ctr);
            delete plan;
            return SWC_ERR_DEVICE;
        }
        if (hipMemcpy(plan->d_items, items.data(), items.size() * sizeof(BatchItem),
                      hipMemcpyHostToDevice) != hipSuccess) {
            hipFree(plan->d_items);
            hipFree(plan->d_ctr);
            delete plan;
            return SWC_ERR_DEVICE;
        }
    }
    for (size_t gi = 0; gi < gstart.size(); gi++) {
        BatchGroup G;
        G.d_items = plan->d_items + gstart[gi];
        G.n_items = (gi + 1 < gstart.size() ? gstart[gi + 1] : (int)items.size()) - gstart[gi];
        G.total_tiles = gtiles[gi];
        G.lds_stride = glds[gi];
        // waves per workgroup: the largest (at most the requested) whose rings fit in 64 KB
        int w = wpb_req;
        while (w > 1 && (int64_t)w * G.lds_stride > 64 * 1024) w /= 2;
        G.wpb = w;
        // a fully resident grid: never more waves than fit at once, nor than the work
        const int64_t resident =
            (int64_t)cus * batch_blocks_per_cu(mode, w, (size_t)G.lds_stride * w) * w;
        G.nwaves = std::max<int64_t>(1, std::min<int64_t>(std::min(target, resident), G.total_tiles));
        plan->groups.push_back(G);
        plan->total_tiles += G.total_tiles;
    }
    *out = plan;
    return SWC_OK;
}

swc_status swc_batch_launch(const swc_batch_plan* plan, void* stream)
{
    if (!plan) return SWC_ERR_NULL;
    // the work lists live on the plan's device
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != plan->device) return SWC_ERR_DEVICE;
    if (fault_inject_launch()) return SWC_ERR_LAUNCH;
    if (sticky_error(hipPeekAtLastError())) return SWC_ERR_DEVICE;
    hipStream_t s = (hipStream_t)stream;
    for (const BatchGroup& G : plan->groups) {
        const int grid = (int)((G.nwaves + G.wpb - 1) / G.wpb);
        const size_t smem = (size_t)G.lds_stride * G.wpb;
        const dim3 blk(G.wpb * kWave);
        hipError_t e;
        switch (plan->mode) {
        case MODE_U8:
            e = launch_kernel(&corr2d_batch_kernel<MODE_U8>, dim3(grid), blk, smem, s, G.d_items,
                              G.n_items, G.total_tiles, G.lds_stride, plan->d_ctr);
            break;
        case MODE_U16:
            e = launch_kernel(&corr2d_batch_kernel<MODE_U16>, dim3(grid), blk, smem, s, G.d_items,
                              G.n_items, G.total_tiles, G.lds_stride, plan->d_ctr);
            break;
        default:
            e = launch_kernel(&corr2d_batch_kernel<MODE_F64>, dim3(grid), blk, smem, s, G.d_items,
                              G.n_items, G.total_tiles, G.lds_stride, plan->d_ctr);
            break;
        }
        if (e != hipSuccess) return sticky_error(e) ? SWC_ERR_DEVICE : SWC_ERR_LAUNCH;
    }
    for (size_t i = 0; i < plan->rest_p.size(); i++) {
        hipError_t e = launch_corr2d(plan->rest_p[i], plan->rest_osh[i].data(), plan->rest_cfg[i],
                                     plan->rest_xy[i][0], plan->rest_xy[i][1], plan->rest_c[i],
                                     plan->rest_f[i], s, 0);
        if (e != hipSuccess) return sticky_error(e) ? SWC_ERR_DEVICE : SWC_ERR_LAUNCH;
    }
    return SWC_OK;
}

int64_t swc_batch_plan_items(const swc_batch_plan* plan)
{
    if (!plan) return 0;
    return plan->total_tiles + (int64_t)plan->rest_p.size();
}

void swc_batch_plan_destroy(swc_batch_plan* plan)
{
    if (!plan) return;
    if (plan->d_items) hipFree(plan->d_items);
    if (plan->d_ctr) hipFree(plan->d_ctr);
    delete plan;
}

}  // extern "C"
