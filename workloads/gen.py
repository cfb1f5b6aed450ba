"""Seeded generators for the benchmark configurations and for tests.

All generators use numpy's PCG64 ``default_rng(seed)``, draw in float64 and
cast at the end.  Shapes are numpy shapes (C order, last axis contiguous); a
"W x H" image is shape (H, W).

Configurations (workloads of the benchmark and of the parity tests):
  c0  (768, 1024) f32  lognormal pair with 8 "cloud" rectangles, 7x7, CLIP
  c1  (3000, 4000) u16 visible/IR-like night image pair, 7x7, FILL (headline)
  c2  (4096, 4096) f32 offset-heavy pair for the precision sweep
  c3  64 f32 pairs of mixed size and window for the batched launch
  c4  (256, 512, 512) f32 volume 7x7x7 and a 2**28-sample series, k = 1001
"""
from __future__ import annotations

import numpy as np

# name -> (generator kwargs, window, step, border)
CONFIGS = {
    "c0": dict(shape=(768, 1024), dtype="f32", window=(7, 7), step=(1, 1), border="clip", seed=0),
    "c1": dict(shape=(3000, 4000), dtype="u16", window=(7, 7), step=(1, 1), border="fill", seed=2),
    "c2": dict(shape=(4096, 4096), dtype="f32", windows=(3, 7, 15, 31), steps=(1, 2, 4),
               border="clip", seed=3),
    "c3": dict(n_pairs=64, seed=1, windows=(5, 7, 9, 15), border="clip"),
    "c4a": dict(shape=(256, 512, 512), dtype="f32", window=(7, 7, 7), step=(1, 1, 1),
                border="clip", seed=4),
    "c4b": dict(shape=(1 << 28,), dtype="f32", window=(1001,), step=(1,), border="clip", seed=5),
}


def cloud_pair(shape=(768, 1024), seed=0, n_rect=8):
    """Lognormal x; y = -0.6 x + N(0, 0.5^2) inside the union of n_rect random
    axis-aligned rectangles ("clouds"), an independent lognormal elsewhere.
    Rectangle height ~ U{H/16..H/4}, width ~ U{W/16..W/4}; top-left uniform so
    that the rectangle fits.  Draw order: x, y_ind, e, rectangles."""
    H, W = shape
    rng = np.random.default_rng(seed)
    x = rng.lognormal(0.0, 1.0, size=shape)
    y_ind = rng.lognormal(0.0, 1.0, size=shape)
    e = rng.normal(0.0, 0.5, size=shape)
    mask = np.zeros(shape, bool)
    for _ in range(n_rect):
        h = int(rng.integers(max(1, H // 16), max(1, H // 4) + 1))
        w = int(rng.integers(max(1, W // 16), max(1, W // 4) + 1))
        r0 = int(rng.integers(0, H - h + 1))
        c0 = int(rng.integers(0, W - w + 1))
        mask[r0:r0 + h, c0:c0 + w] = True
    y = np.where(mask, -0.6 * x + e, y_ind)
    return x.astype(np.float32), y.astype(np.float32)


def _smooth_gaussian(field, sigma):
    from scipy.ndimage import gaussian_filter
    return gaussian_filter(field, sigma=sigma, mode="reflect")


def paper_shaped_u16(shape=(3000, 4000), seed=2, light_density=1e-4, cloud_sigma=40.0,
                     cloud_cover=0.30):
    """Night-time visible/IR-like uint16 pair of the paper's shape class.

    Visible: Poisson(200) background plus square point lights (side 1-3 px,
    value U{20000..60000}, centre density 1e-4).  Cloud mask: N(0,1) noise
    smoothed by a Gaussian (sigma 40 px) and thresholded so 30% is cloud.
    IR: round(N(30000, 800)) minus mask * U(2000, 6000).  Visible gains
    mask * U(1000, 8000) (moonlit cloud).  Clipped to [0, 65535]."""
    H, W = shape
    rng = np.random.default_rng(seed)
    vis = rng.poisson(200.0, size=shape).astype(np.float64)
    n_lights = int(round(light_density * H * W))
    cy = rng.integers(0, H, n_lights)
    cx = rng.integers(0, W, n_lights)
    side = rng.integers(1, 4, n_lights)
    val = rng.integers(20000, 60001, n_lights)
    for i in range(n_lights):
        r0 = max(0, cy[i] - side[i] // 2)
        c0 = max(0, cx[i] - side[i] // 2)
        vis[r0:r0 + side[i], c0:c0 + side[i]] = val[i]
    noise = rng.normal(0.0, 1.0, size=shape)
    smooth = _smooth_gaussian(noise, cloud_sigma)
    mask = (smooth > np.quantile(smooth, 1.0 - cloud_cover)).astype(np.float64)
    ir = np.round(rng.normal(30000.0, 800.0, size=shape))
    ir -= mask * rng.uniform(2000.0, 6000.0, size=shape)
    vis += mask * rng.uniform(1000.0, 8000.0, size=shape)
    x = np.clip(np.round(vis), 0, 65535).astype(np.uint16)
    y = np.clip(np.round(ir), 0, 65535).astype(np.uint16)
    return x, y


def precision_pair(shape=(4096, 4096), seed=3, block=64):
    """x ~ N(1000, 1) (large offset, unit variance); per block x block tile a
    rho ~ U(-1, 1) and y = rho x + N(0,1) sqrt(1 - rho^2)."""
    H, W = shape
    rng = np.random.default_rng(seed)
    x = rng.normal(1000.0, 1.0, size=shape)
    nb = (-(-H // block), -(-W // block))
    rho_b = rng.uniform(-1.0, 1.0, size=nb)
    rho = np.repeat(np.repeat(rho_b, block, axis=0), block, axis=1)[:H, :W]
    y = rho * x + rng.normal(0.0, 1.0, size=shape) * np.sqrt(1.0 - rho * rho)
    return x.astype(np.float32), y.astype(np.float32)


def batched_pairs(n_pairs=64, seed=1, windows=(5, 7, 9, 15), max_w=4096, max_h=3072,
                  min_side=256, scale=1.0):
    """Sizes W ~ U{256..4096}, H ~ U{256..3072} and k ~ choice(windows) drawn
    from default_rng(seed); pair i is ``cloud_pair`` with seed 1000+i.
    ``scale`` < 1 shrinks every side (tests).  Returns a list of
    (x, y, k) tuples."""
    rng = np.random.default_rng(seed)
    Ws = rng.integers(min_side, max_w + 1, n_pairs)
    Hs = rng.integers(min_side, max_h + 1, n_pairs)
    ks = rng.choice(np.asarray(windows), n_pairs)
    out = []
    for i in range(n_pairs):
        h = max(8, int(Hs[i] * scale))
        w = max(8, int(Ws[i] * scale))
        x, y = cloud_pair((h, w), seed=1000 + i)
        out.append((x, y, int(ks[i])))
    return out


def volume_3d(shape=(256, 512, 512), seed=4, sigma=2.0):
    """x = N(0,1) smoothed by a Gaussian (sigma voxels) and renormalised to
    unit standard deviation; y = -0.8 x + N(0, 0.6^2)."""
    rng = np.random.default_rng(seed)
    x = _smooth_gaussian(rng.normal(0.0, 1.0, size=shape).astype(np.float32), sigma)
    x = x / x.std(dtype=np.float64)
    y = -0.8 * x + rng.normal(0.0, 0.6, size=shape)
    return x.astype(np.float32), y.astype(np.float32)


def series_1d(n=1 << 28, seed=5, phi=0.95, rho=0.5):
    """Two AR(1) series (coefficient phi) whose innovations have correlation
    rho: e ~ N(0,1), f = rho e + sqrt(1 - rho^2) g; stationary start."""
    from scipy.signal import lfilter
    rng = np.random.default_rng(seed)
    e = rng.normal(0.0, 1.0, size=n)
    g = rng.normal(0.0, 1.0, size=n)
    f = rho * e + np.sqrt(1.0 - rho * rho) * g
    del g
    s0 = rng.normal(0.0, 1.0, size=2) / np.sqrt(1.0 - phi * phi)
    x = lfilter([1.0], [1.0, -phi], e, zi=[phi * s0[0]])[0].astype(np.float32)
    del e
    y = lfilter([1.0], [1.0, -phi], f, zi=[phi * s0[1]])[0].astype(np.float32)
    return x, y


def random_pair(shape, dtype="f32", seed=0, kind="normal", rho=0.3):
    """Small generic pair for tests: ``kind`` in normal | uniform_int |
    lognormal | offset.  Integer dtypes draw over the full range."""
    rng = np.random.default_rng(seed)
    if dtype == "u8" or dtype == "u16":
        hi = 255 if dtype == "u8" else 65535
        nt = np.uint8 if dtype == "u8" else np.uint16
        x = rng.integers(0, hi + 1, size=shape)
        noise = rng.integers(0, hi + 1, size=shape)
        y = np.where(rng.random(size=shape) < 0.5, x, noise)
        return x.astype(nt), y.astype(nt)
    if kind == "lognormal":
        x = rng.lognormal(0.0, 1.0, size=shape)
        y = rho * x + rng.lognormal(0.0, 1.0, size=shape)
    elif kind == "offset":
        x = rng.normal(1000.0, 1.0, size=shape)
        y = rho * x + rng.normal(0.0, 1.0, size=shape)
    else:
        x = rng.normal(0.0, 1.0, size=shape)
        y = rho * x + rng.normal(0.0, 1.0, size=shape)
    return x.astype(np.float32), y.astype(np.float32)
