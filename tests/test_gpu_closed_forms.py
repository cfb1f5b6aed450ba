"""Statistical sanity of whole maps on the configurations' generators
(closed forms, not parity: they pin the generators and the kernels' overall
behaviour together, where the per-output parity tests pin single values).

  4096x4096 offset pair: y = rho_b x + N(0,1) sqrt(1 - rho_b^2) with rho_b drawn per
      64x64 block, so windows inside a block estimate rho_b; their mean over the block
      matches rho_b up to the small-sample bias of r (about rho (1 - rho^2) / (2n)).
  512x512x256 volume: y = -0.8 x + noise with x a smoothed field; every window is
      strongly negative (the within-window variance of x is below its global unit
      variance, so the window mean lies between -0.8 and about -0.6).
  2^28-sample AR(1) pair with innovation correlation 0.5: the series correlate at
      0.5, and the mean over all windows is 0.5 up to the bias of r at the
      windows' effective sample size.
"""
import numpy as np
import pytest

from gpu_util import gpu_corr, say
from workloads import precision_pair, volume_3d, series_1d

pytestmark = pytest.mark.gpu


def test_block_correlation_tracks_rho():
    x, y = precision_pair((4096, 4096), seed=3)
    c, fl = gpu_corr(x, y, (7, 7), 1, "clip")
    # the generator's block rho values, redrawn in the generator's order
    rng = np.random.default_rng(3)
    rng.normal(1000.0, 1.0, size=(4096, 4096))
    rho_b = rng.uniform(-1.0, 1.0, size=(64, 64))
    pick = np.random.default_rng(7).integers(0, 64, size=(40, 2))
    worst_s = worst_p = 0.0
    for bi, bj in pick:
        win = c[bi * 64 + 3:bi * 64 + 61, bj * 64 + 3:bj * 64 + 61]   # windows inside the block
        bx = x[bi * 64:bi * 64 + 64, bj * 64:bj * 64 + 64].astype(np.float64).ravel()
        by = y[bi * 64:bi * 64 + 64, bj * 64:bj * 64 + 64].astype(np.float64).ravel()
        r_block = float(np.corrcoef(bx, by)[0, 1])                  # the block's own sample
        rho = rho_b[bi, bj]
        bias = rho * (1 - rho * rho) / (2 * 49)                     # small-sample bias of r
        worst_s = max(worst_s, abs(float(win.mean()) - (r_block - bias)))
        worst_p = max(worst_p, abs(float(win.mean()) - (rho - bias)))
    say(f"[closed] 40 blocks: worst |mean c - block r| = {worst_s:.4f}, "
        f"|mean c - rho| = {worst_p:.4f}")
    assert worst_s < 0.03
    assert worst_p < 0.08


def test_volume_windows_negative():
    x, y = volume_3d((128, 256, 256), seed=4)
    c, fl = gpu_corr(x, y, (7, 7, 7), 1, "clip")
    m = float(c.mean())
    say(f"[closed] volume mean c = {m:.4f}, fraction negative = {(c < 0).mean():.5f}")
    assert -0.8 < m < -0.5
    assert (c < 0).mean() > 0.999


def test_series_mean_correlation():
    x, y = series_1d(1 << 24, seed=5)
    c, fl = gpu_corr(x, y, (1001,), 1, "clip")
    m = float(c.mean())
    say(f"[closed] series mean c = {m:.4f}")
    assert abs(m - 0.5) < 0.03
