/*
 * swcorr: sliding-window inter-channel Pearson correlation on AMD Instinct
 * MI355X (gfx950).  C ABI of libswcorr.so.
 *
 * The operation (Poyda & Zhizhin, arXiv 1807.06507):
 *   Two arrays x, y of the same shape and type (Section 3: "both sets must be
 *   the same size") are walked synchronously by a window of a given size
 *   with a given step (Introduction, problem statement).  For each window
 *   position the Pearson coefficient of the window's values is produced
 *   (Introduction, classical formula), computed here by the paper's method
 *   (Section 1): separable sliding sums of x, y, xy, x^2 and y^2, one pass per
 *   dimension (steps 1-3 and the n-dimensional remark), then the per-position
 *   one-pass formula c = (n Sxy - Sx Sy) / sqrt((n Sxx - Sx^2)(n Syy - Sy^2))
 *   (Section 1 formula, step 4).
 *
 * Output conventions (Section 3, I/O paragraph):
 *   - FILL: output has the input's size; the value of a window goes to its
 *     middle cell; windows crossing the border give `invalid_value` (-2).
 *   - any value <= missing_le (-999) inside a window gives `invalid_value`.
 *   - a window whose x (or y) values are all equal has a zero denominator
 *     (Section 3, accuracy paragraph) and gives `invalid_value`.
 *   Readings where the paper is silent (see the design notes): CLIP uses the
 *   in-bounds part of a border window (n = in-bounds count); VALID visits
 *   only windows that fit and compacts the output; for even k the window has
 *   floor(k/2) cells before its centre and k-1-floor(k/2) after; with step s,
 *   output j is centred at j*s (FILL, CLIP) or starts at j*s (VALID); NaN
 *   and +-Inf count as missing; integer inputs never have missing values.
 *
 * Arrays are C-ordered (shape[ndim-1] is contiguous).  All data pointers are
 * DEVICE pointers on the current HIP device.  `stream` is a hipStream_t
 * (NULL = the legacy default stream), passed as void* so that this header
 * does not depend on HIP headers.
 *
 * Error behaviour: every entry point validates its arguments first and
 * returns an error code without touching any memory or launching anything
 * when they are invalid.  Nothing here aborts, throws or prints (unless the
 * environment variable SWC_LOG=1 asks for host-side debug output).  A launch
 * reports its own status (SWC_ERR_LAUNCH when the runtime refuses it); a
 * device fault left pending by earlier work (an error after which the device
 * runs nothing) gives SWC_ERR_DEVICE before anything is launched.  Other
 * errors pending in the HIP runtime are left untouched for whoever caused
 * them.  With SWC_FAULT_INJECT=launch in the environment when the library
 * initialises, every entry point that would launch device work returns
 * SWC_ERR_LAUNCH instead, without touching the device (for tests of error
 * propagation).
 */
#ifndef SWCORR_H
#define SWCORR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWC_VERSION_MAJOR 0
#define SWC_VERSION_MINOR 1

typedef enum swc_status {
    SWC_OK = 0,
    SWC_ERR_NULL = 1,        /* a required pointer is NULL */
    SWC_ERR_NDIM = 2,        /* ndim not in {1,2,3} */
    SWC_ERR_SHAPE = 3,       /* shape < 1, or VALID with shape < window */
    SWC_ERR_WINDOW = 4,      /* window < 1, or above the supported limits */
    SWC_ERR_STEP = 5,        /* step < 1 */
    SWC_ERR_DTYPE = 6,       /* unknown element type */
    SWC_ERR_BORDER = 7,      /* unknown border policy */
    SWC_ERR_ACCUM = 8,       /* unknown accumulation mode, or not valid for the dtype */
    SWC_ERR_WORKSPACE = 9,   /* a caller-provided buffer is too small */
    SWC_ERR_LAUNCH = 10,     /* the kernel launch failed */
    SWC_ERR_DEVICE = 11,     /* no usable device, or a sticky device error */
    SWC_ERR_UNSUPPORTED = 12,/* valid request outside what this build implements */
    SWC_ERR_PARAM = 13       /* invalid launch parameters */
} swc_status;

typedef enum swc_dtype { SWC_U8 = 0, SWC_U16 = 1, SWC_F32 = 2 } swc_dtype;

typedef enum swc_border {
    SWC_BORDER_FILL = 0,   /* same-size output, border windows -> invalid (paper) */
    SWC_BORDER_CLIP = 1,   /* same-size output, border windows clipped */
    SWC_BORDER_VALID = 2   /* only windows that fit; output shrinks */
} swc_border;

typedef enum swc_accum {
    /* u8/u16: exact integer sums, correctly rounded float32 output.
     * f32: FP64 sliding sums of exact FP64 products, FP64 epilogue, windows
     * that a rigorous error bound cannot certify are recomputed by the
     * two-pass formula (flags always exact). */
    SWC_ACC_DEFAULT = 0,
    /* f32 only: plain FP32 sums and FP32 epilogue (comparator, no
     * certification; flags may differ). */
    SWC_ACC_NAIVE_F32 = 1,
    /* f32 only: compensated (TwoSum) FP32 sliding sums, FP64 epilogue. */
    SWC_ACC_COMP_F32 = 2
} swc_accum;

/* Per-output flag bits (optional uint8 map, same shape as c). */
#define SWC_FLAG_BORDER 1u
#define SWC_FLAG_MISSING 2u
#define SWC_FLAG_ZVAR_X 4u
#define SWC_FLAG_ZVAR_Y 8u

/* Problem descriptor.  Entries of shape/window/step beyond ndim are ignored.
 * window[d] = k_d and step[d] = s_d per dimension, in the same (C) order as
 * shape.  invalid_value is written wherever a flag is set (paper: -2).
 * missing_le: float32 values <= this are missing (paper: -999); -INFINITY
 * keeps only NaN/Inf as missing.  Layout is fixed (80 bytes). */
typedef struct swc_problem {
    int32_t ndim;
    int32_t dtype;        /* swc_dtype */
    int32_t border;       /* swc_border */
    int32_t accum;        /* swc_accum */
    int64_t shape[3];
    int32_t window[3];
    int32_t step[3];
    float invalid_value;
    int32_t reserved0;    /* must be 0 */
    double missing_le;
} swc_problem;

/* Launch parameters (tile shape); all-zero means "use the tuned default".
 *   cols_per_lane: contiguous-axis elements owned by one lane (1, 2, 4, 8;
 *                  the 1-D kernel uses 8, the 3-D and batched kernels 4)
 *   tile_rows:     output rows (2-D) / output planes (3-D) / rows of
 *                  64*cols_per_lane window positions (1-D) per wavefront;
 *                  2-D: 0 = as many rows as fill the GPU's resident
 *                  wavefront slots in one round
 *   waves_per_block: 1, 2 or 4 wavefronts per workgroup
 *   min_waves_per_eu: waves per SIMD to size the work for (0 = as many as
 *                  fit): 2-D with tile_rows 0, the resident waves the
 *                  default tile height fills; batched launches, the
 *                  persistent waves per SIMD (0 = 2)
 *   tile_rows2:    3-D only: output rows per wavefront (2 or 4; 0 = 2)  */
typedef struct swc_launch_params {
    int32_t cols_per_lane;
    int32_t tile_rows;
    int32_t waves_per_block;
    int32_t min_waves_per_eu;
    int32_t tile_rows2;
    int32_t reserved[3];
} swc_launch_params;

/* ---- host-only queries (never touch the device) ------------------------ */

/* Check a descriptor.  Returns SWC_OK or the first error found. */
swc_status swc_validate(const swc_problem *p);

/* Output shape for a valid descriptor: out[d] for d < ndim (FILL/CLIP:
 * ceil(N/s); VALID: floor((N-k)/s)+1); entries >= ndim are set to 1. */
swc_status swc_output_shape(const swc_problem *p, int64_t out[3]);

/* Static, NUL-terminated description of a status code (never NULL). */
const char *swc_status_str(swc_status s);

/* Library version as major*100 + minor. */
int32_t swc_version(void);

/* ---- single problem ---------------------------------------------------- */

/* Correlation map of one pair (Section 1 steps 1-4, fused into one kernel).
 *   x, y:  device arrays of p->shape, element type p->dtype (read only)
 *   c:     device float32 array of swc_output_shape(p) (written)
 *   flags: device uint8 array of the same shape, or NULL (written if given)
 *   stream: hipStream_t; the call is asynchronous on it, allocates nothing
 *   and does not synchronize.
 * x/y must not alias c/flags.  The caller owns all buffers and keeps them
 * alive until the stream work completes. */
swc_status swc_corr(const swc_problem *p, const void *x, const void *y, float *c,
                    uint8_t *flags, void *stream);

/* Same as swc_corr with explicit launch parameters (NULL = tuned default).
 * Used by the autotuner; returns SWC_ERR_PARAM for unsupported values. */
swc_status swc_corr_ex(const swc_problem *p, const swc_launch_params *lp, const void *x,
                       const void *y, float *c, uint8_t *flags, void *stream);

/* ---- unfused baseline schemes ------------------------------------------ */
/* The same 2-D map computed by two unfused schemes, kept as measured
 * baselines for swc_corr:
 *   SWC_SCHEME_UNFUSED: the paper's parallel scheme (Section 2): element
 *     products, then one thread per row (step 2) and one thread per column
 *     (step 3) running moving sums, then the formula per element (step 4),
 *     with every intermediate matrix of Section 1 stored in the workspace.
 *   SWC_SCHEME_CUMSUM: the cumulative-sum alternative mentioned at the end
 *     of Section 1: 2-D prefix sums of the five channels, window sums by
 *     inclusion-exclusion of four corners.  uint8/uint16 only (exact uint64
 *     prefix sums).
 * Results equal swc_corr's (same flags, same certified rounding).  Supported:
 * ndim 2, step 1, FILL or CLIP, SWC_ACC_DEFAULT; anything else returns
 * SWC_ERR_UNSUPPORTED. */
typedef enum swc_scheme { SWC_SCHEME_UNFUSED = 1, SWC_SCHEME_CUMSUM = 2 } swc_scheme;
/* Workspace bytes the scheme needs for problem p (host only):
 * UNFUSED 256 + 96 * H * W, CUMSUM 40 * H * W. */
swc_status swc_scheme_workspace(const swc_problem *p, int32_t scheme, uint64_t *bytes);
/* Run a scheme on `stream` (asynchronous; several kernels in order).
 *   x, y, c, flags: as for swc_corr (flags may be NULL)
 *   workspace: device buffer of at least swc_scheme_workspace() bytes,
 *     8-byte aligned, owned by the caller, overwritten; it must not be used
 *     by other work until the stream has finished this call.
 * Returns SWC_ERR_WORKSPACE when the workspace is too small or misaligned.
 * Allocates nothing. */
swc_status swc_corr_scheme(const swc_problem *p, int32_t scheme, const void *x, const void *y,
                           float *c, uint8_t *flags, void *workspace, uint64_t workspace_bytes,
                           void *stream);
/* The schemes without a caller workspace, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation): the workspace is a fixed array of
 * SWC_SCHEME_SCRATCH_BYTES in device memory, one per device the library runs
 * on, held until the process ends.  Same arguments, results and errors as
 * swc_corr_scheme, except: returns SWC_ERR_WORKSPACE (before touching the
 * device) when the problem needs more than SWC_SCHEME_SCRATCH_BYTES
 * (UNFUSED: H * W <= 699,048; CUMSUM: H * W <= 1,677,721).  Calls no
 * allocating routine.  All calls on one device share its array: calls that
 * may overlap on one device (other streams, other threads) race and must be
 * ordered by the caller.  The array keeps the last call's contents; each
 * call initialises what it reads.  The first call on a device looks up the
 * array's device address (no stream work). */
#define SWC_SCHEME_SCRATCH_BYTES (64ull << 20)
swc_status swc_corr_scheme_noalloc(const swc_problem *p, int32_t scheme, const void *x,
                                   const void *y, float *c, uint8_t *flags, void *stream);
/* ---- end-to-end runs from host memory ---------------------------------- */
/* A plan for host-to-host runs of problem p (any ndim, step[0] == 1): the
 * input is cut into slabs of `band_rows` outputs along the first axis (plus
 * the k-1 halo rows their windows need), and each slab's host-to-device
 * copies, fused kernel (swc_corr) and device-to-host copy are issued in
 * order on one of `depth` streams (1..8), so transfers of one slab overlap
 * the kernel of another.  This is the end-to-end setting of the paper's GPU
 * timing (Section 3: the time includes the transfers to and from the
 * device).  Creation allocates `depth` device staging sets and streams (the
 * plan owns them); returns SWC_ERR_UNSUPPORTED for step[0] != 1,
 * SWC_ERR_PARAM for band_rows < 1 or depth outside 1..8, SWC_ERR_DEVICE
 * when allocation fails. */
typedef struct swc_host_plan swc_host_plan;
swc_status swc_host_plan_create(const swc_problem *p, int64_t band_rows, int32_t depth,
                                swc_host_plan **out);
/* Run the plan: x, y are HOST arrays of p->shape; c (float32) and flags
 * (uint8, may be NULL) HOST arrays of swc_output_shape(p).  Page-locked
 * host memory (hipHostMalloc) is needed for the copies to overlap; pageable
 * memory works but serialises them.  Synchronous: returns once c and flags
 * hold the result (all streams drained, also after an error).  Results equal
 * swc_corr's on the whole array (bit-exact for integer input; float input
 * within the same bound, since the slabs are tiled differently).  The device
 * current at plan creation must be current (SWC_ERR_DEVICE otherwise). */
swc_status swc_host_run(swc_host_plan *plan, const void *x, const void *y, float *c,
                        uint8_t *flags);
/* Number of slabs per run. */
int64_t swc_host_plan_bands(const swc_host_plan *plan);
/* Free the plan's device memory and streams (NULL is ignored). */
void swc_host_plan_destroy(swc_host_plan *plan);
/* ---- the application's use of the map ---------------------------------- */
/* Night-time light detections are false where moonlight is reflected by
 * clouds; there the visible/infrared correlation is close to -1
 * (Introduction, Conclusion).  Both calls read a finished map c (device,
 * float32, n outputs) and its flag map (device uint8, or NULL: then an output
 * is valid when c differs from invalid_value).  Asynchronous on `stream`,
 * allocate nothing; n == 0 / k == 0 launch nothing.  Errors: SWC_ERR_SHAPE
 * for n < 0 or k < 0, SWC_ERR_PARAM for a NaN tau, SWC_ERR_NULL for missing
 * pointers.
 * Cloud mask: mask[i] (device uint8, n) = 1 when output i is valid and
 * c[i] < -tau (float32 comparison), else 0. */
swc_status swc_cloud_mask(const float *c, const uint8_t *flags, int64_t n, float tau,
                          float invalid_value, uint8_t *mask, void *stream);
/* Detection filter: for k detections at flat output indices idx[j] (device
 * int64), keep[j] (device uint8) = 0 when the detection sits on a cloud
 * pixel (as in the mask), 1 when it is kept, 2 when idx[j] is outside
 * [0, n) (checked on the device; nothing outside the map is read). */
swc_status swc_filter_detections(const float *c, const uint8_t *flags, int64_t n,
                                 const int64_t *idx, int64_t k, float tau, float invalid_value,
                                 uint8_t *keep, void *stream);
/* ---- tuning table ------------------------------------------------------ */

/* Register launch parameters for problems like `p` (same dtype, ndim,
 * accumulation mode and window-size bucket).  Host only.  Thread-safe. */
swc_status swc_tune_set(const swc_problem *p, const swc_launch_params *lp);

/* Parameters swc_corr would use for `p` (tuned entry or built-in default). */
swc_status swc_tune_get(const swc_problem *p, swc_launch_params *lp);

/* ---- batches of independent pairs (persistent launches) ---------------- */

typedef struct swc_batch_plan swc_batch_plan;

/* Build a plan for n pairs (problems may differ in shape, window, step and
 * border, but must share dtype and accumulation mode, and be 2-D).  The
 * arrays x[i], y[i], c[i], flags[i] (flags may be NULL, or contain NULLs)
 * are device pointers kept by the plan.  Allocates and fills the plan's
 * device-side work list and two work-list counters (synchronous, not
 * capture-safe).  The plan owns that memory; free it with
 * swc_batch_plan_destroy.  `lp` may be NULL (tuned or
 * built-in choice); in it, tile_rows = 0 lets the plan pick about four tiles
 * per persistent wavefront, and waves_per_block = 0 (or a value whose LDS
 * rings exceed 64 KB per workgroup) the largest of 4, 2, 1 that fits. */
swc_status swc_batch_plan_create(int32_t n, const swc_problem *p, const void *const *x,
                                 const void *const *y, float *const *c,
                                 uint8_t *const *flags, const swc_launch_params *lp,
                                 swc_batch_plan **out);

/* Compute every pair of the plan on `stream` (the device current at plan
 * creation must be current; SWC_ERR_DEVICE otherwise): persistent launches, one per
 * group of pairs whose LDS rings allow the same number of resident
 * wavefronts per CU (at most four), plus one ordinary launch per pair without
 * a compiled window width.  Asynchronous, allocates nothing, safe to capture
 * into a hipGraph.  The persistent waves take work items from the plan's
 * counters, which each launch leaves at zero: launches of one plan must not
 * overlap (issue them on one stream, or order them by events). */
swc_status swc_batch_launch(const swc_batch_plan *plan, void *stream);

/* Number of work items (tiles) in the plan, for reporting. */
int64_t swc_batch_plan_items(const swc_batch_plan *plan);

/* Free the plan (NULL is ignored).  The caller ensures no launch of it is
 * still in flight. */
void swc_batch_plan_destroy(swc_batch_plan *plan);

/* ---- debug switches ---------------------------------------------------- */

/* Bit 0: send every integer-input output through the exact big-integer
 * rounding decision and every float-input output through the two-pass
 * window recomputation (results must not change).  Bit 1: 2-D pairs use the
 * generic LDS-row kernel and 3-D problems the general step.  Bit 2: the 1-D
 * kernel re-reads the values leaving the window from memory instead of its
 * LDS ring.  Bit 3: the compensated float32 comparator (SWC_ACC_COMP_F32)
 * skips its certification test, so every window with a positive computed
 * variance takes the value of its compensated sums (measures those sums'
 * own accuracy; constant windows still get their flags).  Host only;
 * applies to launches issued after the call.  Bit 0 is also set from
 * SWC_FORCE_EXACT_FALLBACK=1 at library load. */
void swc_set_debug(int32_t bits);
int32_t swc_get_debug(void);

#ifdef __cplusplus
}
#endif

#endif /* SWCORR_H */
