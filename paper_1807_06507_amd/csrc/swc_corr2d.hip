// Fused 2-D sliding-window correlation (Poyda & Zhizhin, arXiv 1807.06507,
// Section 1 steps 1-4, fused into one kernel; Section 3 output conventions).
//
// Work decomposition (one wavefront = one tile):
//   * a tile is `TH` output rows x `Wq` output columns;
//   * the wave owns 64*R contiguous input columns (R per lane, vector loads),
//     the tile's columns plus the window halo, aligned down to R elements;
//   * each lane marches down the input rows of the tile (plus the k_h - 1
//     halo rows), keeping the five running column sums of its R columns in
//     registers: add the entering row, subtract the row k_h above (re-read;
//     it is an L2/L1 hit).  This is step 2 along the first dimension;
//   * when the running sums cover an output row, the wave writes them to a
//     per-wave LDS row buffer and each lane slides a k_w-wide window over
//     that buffer for its outputs (step 3 along the contiguous dimension);
//   * the epilogue (step 4) and the store follow immediately; x and y are
//     read from HBM once (halo re-reads hit L2) and c is written once.
// Tiles are numbered column-major so vertically adjacent tiles, which share
// k_h - 1 halo rows, run close in time on the same XCD.
#include "swc_corr2d_fast.hpp"
#include "swc_device.hpp"
#include "swc_internal.h"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

namespace swc {

struct P2D {
    const void* x;
    const void* y;
    float* c;
    uint8_t* flags;
    int64_t H, W, OH, OW;
    int kh, kw, sh, sw, oh, ow;
    int border;
    float invalid;
    float miss_thr;
    int force;
    double cert_g;
    int TH, Wq, tiles_x, tiles_y, n_tiles;
    int vec;
};

// Load R consecutive elements of one row starting at column c0 (zeros
// outside [0, W)).  Vector load when allowed and fully in bounds.
template <class T, int R>
__device__ __forceinline__ void load_run(const T* __restrict__ row, int64_t c0, int64_t W,
                                         bool vec, T (&v)[R])
{
    // whole run inside the row and aligned for one vector load (float rows
    // of any width may reach here with `vec` set, unaligned)
    if (vec && c0 >= 0 && c0 + R <= W && (uintptr_t)(row + c0) % (sizeof(T) * R) == 0) {
        const T* p = (const T*)__builtin_assume_aligned(row + c0, sizeof(T) * R);
        __builtin_memcpy(v, p, sizeof(T) * R);
    } else {
#pragma unroll
        for (int j = 0; j < R; j++) {
            int64_t cc = c0 + j;
            v[j] = (cc >= 0 && cc < W) ? row[cc] : (T)0;
        }
    }
}

template <int M, int R>
__global__ void __launch_bounds__(256) corr2d_kernel(P2D g)
{
    using T = typename Tr<M>::T;
    constexpr int NC = kWave * R;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // wave-uniform
    const int wpb = blockDim.x / kWave;
    const int tile = xcd_remap(blockIdx.x, gridDim.x) * wpb + wv;
    if (tile >= g.n_tiles) return;
    LdsRow<M> L = lds_row_carve<M>(smem + wv * lds_row_bytes<M>(NC), NC);

    const int tx = tile / g.tiles_y;
    const int ty = tile - tx * g.tiles_y;
    const int64_t p0 = (int64_t)ty * g.TH;
    const int64_t q0 = (int64_t)tx * g.Wq;
    const int ph = (int)min((int64_t)g.TH, g.OH - p0);
    const int qw = (int)min((int64_t)g.Wq, g.OW - q0);
    const int64_t E = q0 * g.sw + g.ow;
    const int64_t Eal = (E >= 0) ? (E / R) * R : -((-E + R - 1) / R) * R;
    const int delta = (int)(E - Eal);
    const int64_t col0 = Eal + (int64_t)lane * R;
    const T* __restrict__ X = (const T*)g.x;
    const T* __restrict__ Y = (const T*)g.y;
    const int64_t H = g.H, W = g.W;
    const int64_t i0 = p0 * g.sh + g.oh;
    const int64_t i1 = (p0 + ph - 1) * g.sh + g.oh + g.kh - 1;
    const bool vec = g.vec != 0;

    Acc<M> V[R];
#pragma unroll
    for (int j = 0; j < R; j++) acc_zero<M>(V[j]);
    float hmx = 0.f, hmy = 0.f;

    const int Ro = (qw + kWave - 1) / kWave;
    const int ob = lane * Ro;
    const int oe = min(ob + Ro, qw);

    int64_t ready = i0 + g.kh - 1;   // row at which output row p completes
    int64_t p = p0;
    for (int64_t i = i0; i <= i1; ++i) {
        // ---- step 1 + step 2: entering row ----
        {
            T ax[R], ay[R];
            if (i >= 0 && i < H) {
                load_run<T, R>(X + i * W, col0, W, vec, ax);
                load_run<T, R>(Y + i * W, col0, W, vec, ay);
            } else {
#pragma unroll
                for (int j = 0; j < R; j++) { ax[j] = 0; ay[j] = 0; }
            }
#pragma unroll
            for (int j = 0; j < R; j++) {
                const int64_t cj = col0 + j;
                const bool inb = i >= 0 && i < H && cj >= 0 && cj < W;
                Elem<M> e = make_elem<M>(ax[j], ay[j], g.miss_thr, inb);
                acc_add<M>(V[j], e);
                if constexpr (!Tr<M>::kInt) {
                    if (!e.miss) {
                        hmx = fmaxf(hmx, __builtin_fabsf((float)ax[j]));
                        hmy = fmaxf(hmy, __builtin_fabsf((float)ay[j]));
                    }
                }
            }
        }
        // ---- leaving row ----
        const int64_t io = i - g.kh;
        if (io >= i0) {
            T ax[R], ay[R];
            if (io >= 0 && io < H) {
                load_run<T, R>(X + io * W, col0, W, vec, ax);
                load_run<T, R>(Y + io * W, col0, W, vec, ay);
            } else {
#pragma unroll
                for (int j = 0; j < R; j++) { ax[j] = 0; ay[j] = 0; }
            }
#pragma unroll
            for (int j = 0; j < R; j++) {
                const int64_t cj = col0 + j;
                const bool inb = io >= 0 && io < H && cj >= 0 && cj < W;
                Elem<M> e = make_elem<M>(ax[j], ay[j], g.miss_thr, inb);
                acc_sub<M>(V[j], e);
            }
        }
        if (i != ready) continue;

        // ---- step 3: horizontal window sums through LDS ----
#pragma unroll
        for (int j = 0; j < R; j++) lds_put<M>(L, lane * R + j, V[j]);
        if constexpr (!Tr<M>::kInt) {
            L.mx[lane] = hmx;
            L.my[lane] = hmy;
        }
        wave_lds_sync();
        if (ob < oe) {
            Acc<M> S;
            acc_zero<M>(S);
            const int a0 = delta + ob * g.sw;
            for (int e = a0; e < a0 + g.kw; ++e) acc_addacc<M>(S, lds_get<M>(L, e));
            float Mx = 0.f, My = 0.f;
            if constexpr (!Tr<M>::kInt) {
                const int l_lo = a0 / R;
                const int l_hi = (delta + (oe - 1) * g.sw + g.kw - 1) / R;
                for (int l = l_lo; l <= l_hi; ++l) {
                    Mx = fmaxf(Mx, L.mx[l]);
                    My = fmaxf(My, L.my[l]);
                }
            }
            const int64_t rlo = p * g.sh + g.oh, rhi = rlo + g.kh - 1;
            const bool row_out = rlo < 0 || rhi >= H;
            const int64_t rl = max(rlo, (int64_t)0), rh = min(rhi, H - 1);
            for (int o = ob; o < oe; ++o) {
                if (o > ob) {
                    const int ap = delta + (o - 1) * g.sw;
                    if (g.sw < g.kw) {
                        for (int e = ap + g.kw; e < ap + g.kw + g.sw; ++e)
                            acc_addacc<M>(S, lds_get<M>(L, e));
                        for (int e = ap; e < ap + g.sw; ++e) acc_subacc<M>(S, lds_get<M>(L, e));
                    } else {
                        acc_zero<M>(S);
                        const int an = ap + g.sw;
                        for (int e = an; e < an + g.kw; ++e) acc_addacc<M>(S, lds_get<M>(L, e));
                    }
                }
                // ---- step 4: epilogue + store ----
                const int64_t q = q0 + o;
                const int64_t clo = q * g.sw + g.ow, chi = clo + g.kw - 1;
                uint8_t fl = 0;
                if (g.border == BORDER_FILL && (row_out || clo < 0 || chi >= W)) fl = FL_BORDER;
                const int64_t cl = max(clo, (int64_t)0), ch = min(chi, W - 1);
                const int64_t n = (rh - rl + 1) * (ch - cl + 1);
                if constexpr (Tr<M>::kMiss) {
                    if (!fl && S.miss > 0) fl = FL_MISSING;
                }
                float cv = 0.f;
                if (!fl) {
                    WinBox wb{W, 1, rl, rh, cl, ch, 0, 0};
                    fl = epilogue<M>(S, n, Mx, My, g.cert_g, (g.force & 1) != 0, g.x, g.y, wb, &cv);
                }
                if (fl) cv = g.invalid;
                const int64_t oi = p * g.OW + q;
                g.c[oi] = cv;
                if (g.flags) g.flags[oi] = fl;
            }
        }
        wave_lds_sync();
        ++p;
        ready += g.sh;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

static int wq_of(int R, int kw, int sw)
{
    const int span = kWave * R - (R - 1);   // usable ext columns after alignment
    if (span < kw) return 0;
    return (span - kw) / sw + 1;
}

template <int M> static int lds_bytes_per_wave(int R) { return lds_row_bytes<M>(kWave * R); }

static int lds_bytes_for(int mode, int R)
{
    switch (mode) {
    case MODE_U8: return lds_bytes_per_wave<MODE_U8>(R);
    case MODE_U16: return lds_bytes_per_wave<MODE_U16>(R);
    case MODE_F64: return lds_bytes_per_wave<MODE_F64>(R);
    case MODE_F32N: return lds_bytes_per_wave<MODE_F32N>(R);
    default: return lds_bytes_per_wave<MODE_F32C>(R);
    }
}

bool cfg_ok_2d(const swc_problem& p, const LaunchCfg& L)
{
    if (!(L.R == 1 || L.R == 2 || L.R == 4 || L.R == 8)) return false;
    if (!(L.wpb == 1 || L.wpb == 2 || L.wpb == 4)) return false;
    if (L.TH < 0 || L.TH > 4096) return false;   // 0: chosen per launch
    if (L.minw < 0 || L.minw > 8) return false;
    if (wq_of(L.R, p.window[1], p.step[1]) < 1) return false;
    int mode = mode_of(p.dtype, p.accum);
    if (mode < 0) return false;
    if ((int64_t)lds_bytes_for(mode, L.R) * L.wpb > 64 * 1024) return false;
    return true;
}

template <int M, int R>
static hipError_t launch_mr(const P2D& g, int wpb, int grid, size_t smem, hipStream_t s)
{
    return launch_kernel(&corr2d_kernel<M, R>, dim3(grid), dim3(wpb * kWave), smem, s, g);
}

template <int M>
static hipError_t launch_m(const P2D& g, int R, int wpb, int grid, hipStream_t s)
{
    size_t smem = (size_t)lds_bytes_per_wave<M>(R) * wpb;
    switch (R) {
    case 1: return launch_mr<M, 1>(g, wpb, grid, smem, s);
    case 2: return launch_mr<M, 2>(g, wpb, grid, smem, s);
    case 4: return launch_mr<M, 4>(g, wpb, grid, smem, s);
    default: return launch_mr<M, 8>(g, wpb, grid, smem, s);
    }
}

// Workgroups of the register-resident kernel that fit on one CU (cached per
// configuration and device).
static int fast2d_blocks_per_cu(int mode, int R, int kw, bool vec, int wpb, size_t smem)
{
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, int, int, int, size_t>, int> cache;
    int dev = 0;
    hipGetDevice(&dev);
    const auto key = std::make_tuple(dev, mode, R, kw, (int)vec, wpb, smem);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    int n = 0;
    P2DF dummy{};
    hipError_t e;
    if (mode == MODE_U8) e = launch_fast2d_modeu8(dummy, R, kw, vec, 0, wpb, smem, nullptr, &n);
    else if (mode == MODE_U16) e = launch_fast2d_modeu16(dummy, R, kw, vec, 0, wpb, smem, nullptr, &n);
    else e = launch_fast2d_modef64(dummy, R, kw, vec, 0, wpb, smem, nullptr, &n);
    if (e != hipSuccess || n < 1) n = 1;
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = n;
    return n;
}

static int device_cus()
{
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
        cus = 256;
    return cus;
}

hipError_t launch_corr2d(const swc_problem& p, const int64_t* oshape, const LaunchCfg& L,
                         const void* x, const void* y, float* c, uint8_t* flags,
                         hipStream_t s, int force)
{
    const int mode = mode_of(p.dtype, p.accum);
    P2D g;
    g.x = x;
    g.y = y;
    g.c = c;
    g.flags = flags;
    g.H = p.shape[0];
    g.W = p.shape[1];
    g.OH = oshape[0];
    g.OW = oshape[1];
    g.kh = p.window[0];
    g.kw = p.window[1];
    g.sh = p.step[0];
    g.sw = p.step[1];
    g.oh = window_offset(p.border, g.kh);
    g.ow = window_offset(p.border, g.kw);
    g.border = p.border;
    g.invalid = p.invalid_value;
    g.miss_thr = missing_threshold(p.missing_le);
    g.force = force;
    const size_t esz = p.dtype == SWC_U8 ? 1 : (p.dtype == SWC_U16 ? 2 : 4);
    const size_t va = esz * (size_t)L.R;
    // vector loads of a lane's R-element run: float rows need only 4-byte
    // alignment (a run crossing the row end reads zeros past it: raw buffer
    // loads are range-checked per dword); narrower types need whole runs
    g.vec = (esz == 4) ? ((uintptr_t)x % 4 == 0 && (uintptr_t)y % 4 == 0 ? 1 : 0)
                       : ((uintptr_t)x % va == 0 && (uintptr_t)y % va == 0 &&
                          (g.W % L.R) == 0 ? 1 : 0);

    // register-resident kernel for compiled window widths (debug bit 2 forces
    // the generic LDS kernel); 32-bit geometry and byte counts (rows are
    // addressed as raw buffers of at most 2^31 - 1 bytes)
    const bool dims32 = g.H < ((int64_t)1 << 31) - 2 * kWave * 8 &&
                        g.W * 4 < ((int64_t)1 << 31) - 2 * kWave * 8 * 4;
    // waves per workgroup: as requested, halved while the LDS rings of the
    // workgroup would exceed 64 KB (wide windows keep no ring)
    int wpb_f = L.wpb;
    const int lds_w = fast2d_lds_per_wave(mode, L.R, g.kh, g.kw, g.vec != 0);
    while (wpb_f > 1 && (size_t)wpb_f * lds_w > 64 * 1024) wpb_f /= 2;
    const size_t smem_f = (size_t)wpb_f * lds_w;
    if (!(force & 2) && dims32 && fast2d_supported(mode, L.R, g.kw) && smem_f <= 64 * 1024) {
        P2DF f;
        f.x = x;
        f.y = y;
        f.c = c;
        f.flags = flags;
        f.H = (int)g.H;
        f.W = (int)g.W;
        f.OH = (int)g.OH;
        f.OW = (int)g.OW;
        f.kh = g.kh;
        f.sh = g.sh;
        f.sw = g.sw;
        f.oh = g.oh;
        f.ow = g.ow;
        f.border = g.border;
        f.invalid = g.invalid;
        f.miss_thr = g.miss_thr;
        f.force = force;
        // whole-vector stores: unit column step, centred windows (output
        // column = input column), rows of a multiple of 4 (c) / R (flags)
        // elements, aligned bases; tiles then start on lane boundaries
        const bool contig = g.sw == 1 && g.ow == -(g.kw / 2) && (L.R % 4) == 0 &&
                            fast2d_wq_aligned(L.R, g.kw) >= 1;
        f.vst = (contig && g.OW % 4 == 0 && (uintptr_t)c % 16 == 0 ? 1 : 0) |
                (contig && flags && g.OW % L.R == 0 && (uintptr_t)flags % L.R == 0 ? 2 : 0);
        f.Wq = contig ? fast2d_wq_aligned(L.R, g.kw) : wq_of(L.R, g.kw, g.sw);
        const int64_t tiles_x = (g.OW + f.Wq - 1) / f.Wq;
        const bool vec = g.vec != 0;
        int TH = L.TH;
        if (TH <= 0) {
            // one round of resident waves: as many tile rows as the free wave
            // slots allow across the tile columns, each as tall as that needs
            // (min_waves_per_eu > 0: at most that many waves per SIMD)
            int64_t per_cu = (int64_t)wpb_f * fast2d_blocks_per_cu(mode, L.R, g.kw, vec, wpb_f, smem_f);
            if (L.minw > 0) per_cu = std::min<int64_t>(per_cu, 4 * (int64_t)L.minw);
            const int64_t slots = (int64_t)device_cus() * std::max<int64_t>(1, per_cu);
            const int64_t ty = std::max<int64_t>(1, slots / std::max<int64_t>(1, tiles_x));
            TH = (int)std::min<int64_t>(4096, std::max<int64_t>(4, (g.OH + ty - 1) / ty));
        }
        f.TH = TH;
        f.tiles_y = (int)((g.OH + TH - 1) / TH);
        const int64_t ntf = tiles_x * f.tiles_y;
        if (ntf >= (int64_t)1 << 31) return hipErrorInvalidValue;
        f.n_tiles = (int)ntf;
        // certification factor of the tile's march and sums along the row
        const double th_ext = (double)(TH - 1) * g.sh + g.kh;
        f.cert_g = fast2d_cert(mode, L.R, g.kh, g.kw, th_ext);
        const int gridf = (int)((ntf + wpb_f - 1) / wpb_f);
        if (mode == MODE_U8) return launch_fast2d_modeu8(f, L.R, g.kw, vec, gridf, wpb_f, smem_f, s);
        if (mode == MODE_U16) return launch_fast2d_modeu16(f, L.R, g.kw, vec, gridf, wpb_f, smem_f, s);
        return launch_fast2d_modef64(f, L.R, g.kw, vec, gridf, wpb_f, smem_f, s);
    }

    // generic LDS-row kernel
    g.TH = L.TH > 0 ? L.TH : 32;
    g.Wq = wq_of(L.R, g.kw, g.sw);
    g.tiles_x = (int)((g.OW + g.Wq - 1) / g.Wq);
    g.tiles_y = (int)((g.OH + g.TH - 1) / g.TH);
    const int64_t nt = (int64_t)g.tiles_x * g.tiles_y;
    if (nt >= (int64_t)1 << 31) return hipErrorInvalidValue;
    g.n_tiles = (int)nt;
    // certification factor: chain = vertical march (2 ops/row) + horizontal
    // slide; nterms = (kh+1)(kw+1)
    const double th_ext = (double)(g.TH - 1) * g.sh + g.kh;
    const double ro = (double)((g.Wq + kWave - 1) / kWave);
    const double chain = 2.0 * th_ext + g.kw + 2.0 * ro * g.sw + 2.0;
    const double nterms = (double)(g.kh + 1) * (g.kw + 1);
    g.cert_g = cert_factor(mode, (double)g.kh * g.kw, chain, nterms);
    // debug bit 3: the compensated comparator without its certification
    // (a zero threshold passes every window of positive computed variance)
    if (mode == MODE_F32C && (force & 8)) g.cert_g = 0.0;
    const int grid = (int)((nt + L.wpb - 1) / L.wpb);
    switch (mode) {
    case MODE_U8: return launch_m<MODE_U8>(g, L.R, L.wpb, grid, s);
    case MODE_U16: return launch_m<MODE_U16>(g, L.R, L.wpb, grid, s);
    case MODE_F64: return launch_m<MODE_F64>(g, L.R, L.wpb, grid, s);
    case MODE_F32N: return launch_m<MODE_F32N>(g, L.R, L.wpb, grid, s);
    default: return launch_m<MODE_F32C>(g, L.R, L.wpb, grid, s);
    }
}

}  // namespace swc
