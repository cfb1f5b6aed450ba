"""GPU parity of the fused 3-D kernel (the n-dimensional summation of
Section 1) against the CPU oracle, through the C ABI.

Integer inputs bit-exact; float inputs |dc| <= 2^-24 with identical flags.
Covers every border policy, odd window widths 3-9 with mixed window depths and
heights (even ones too), steps, volumes smaller than the window, missing values
and constant blocks; the 3-D configuration's generator at 64x128x128 on every
output and at its full 256x512x512 size on sampled outputs.
"""
import numpy as np
import pytest

from gpu_util import compare, say
from workloads import random_pair, volume_3d

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("border", ["fill", "clip", "valid"])
def test_parity_3d_shapes(dtype, border):
    for shape, window, step in [((9, 20, 300), (3, 5, 7), 1), ((12, 33, 70), (7, 7, 7), 1),
                                ((6, 17, 260), (4, 2, 5), 1), ((10, 21, 90), (3, 3, 3), (2, 3, 1)),
                                ((5, 9, 40), (5, 3, 9), (1, 1, 2)), ((3, 4, 5), (3, 3, 3), 1)]:
        if border == "valid" and any(s < k for s, k in zip(shape, window)):
            continue
        x, y = random_pair(shape, dtype, seed=sum(shape) + sum(window))
        compare(x, y, window, step, border, tag="3d")


@pytest.mark.parametrize("params", [(4, 1, 1, 0, 2), (4, 7, 2, 0, 2), (4, 32, 4, 0, 4),
                                    (4, 64, 1, 0, 2)])
def test_parity_3d_launch_params(params):
    for dtype in ("u16", "f32"):
        x, y = random_pair((20, 30, 300), dtype, seed=7)
        compare(x, y, (7, 7, 7), 1, "clip", params=params, tag="3d-params")


def test_parity_3d_missing_and_constant():
    x, y = random_pair((14, 24, 100), "f32", seed=2, kind="lognormal")
    x[3, 4, 5] = -999.0
    y[7, 10, 60] = np.nan
    x[9:14, 0:12, 20:45] = 1.5
    y[0:6, 15:24, 70:100] = -3.0
    for border in ("clip", "fill"):
        compare(x, y, (5, 5, 5), 1, border, tag="3d-specials")


def test_parity_3d_tiny_volumes():
    for dtype in ("u16", "f32"):
        x, y = random_pair((2, 3, 4), dtype, seed=1)
        compare(x, y, (7, 7, 7), 1, "clip", tag="3d-tiny")
        compare(x, y, (7, 7, 7), 1, "fill", tag="3d-tiny")


def test_parity_volume_config_reduced():
    """Smoothed-normal volume pair (y = -0.8 x + noise), 7x7x7, CLIP, at
    64x128x128: every output."""
    x, y = volume_3d((64, 128, 128), seed=4)
    d = compare(x, y, (7, 7, 7), 1, "clip", tag="c4a-reduced")
    say(f"c4a reduced max|dc| = {d:.3e}")


def test_parity_volume_config_full_sampled():
    """Full 256x512x512 volume: 20000 sampled outputs plus the first planes'
    border region, compared one by one."""
    x, y = volume_3d((256, 512, 512), seed=4)
    n = x.size
    rng = np.random.default_rng(0)
    idx = np.unique(np.concatenate([rng.integers(0, n, 20000), np.arange(3000)]))
    d = compare(x, y, (7, 7, 7), 1, "clip", indices=idx, tag="c4a-full")
    say(f"c4a full (sampled) max|dc| = {d:.3e}")


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("border", ["fill", "clip", "valid"])
def test_parity_3d_square_yx_windows(dtype, border):
    """Square (y, x) windows with unit y step and rows a multiple of 4 long
    (the specialised step): every x window width, z windows and steps that
    differ, and agreement with the general step (debug bit 1)."""
    import paper_1807_06507_amd as swc
    from gpu_util import gpu_corr
    for shape, window, step in [((11, 19, 64), (3, 3, 3), 1), ((9, 14, 132), (5, 5, 5), (1, 1, 2)),
                                ((13, 22, 200), (3, 7, 7), (2, 1, 1)), ((10, 17, 96), (9, 9, 9), 1),
                                ((8, 9, 40), (1, 5, 5), (3, 1, 3))]:
        if border == "valid" and any(s < k for s, k in zip(shape, window)):
            continue
        x, y = random_pair(shape, dtype, seed=sum(shape) * 3 + sum(window))
        compare(x, y, window, step, border, tag="3d-square")
        a, fa = gpu_corr(x, y, window, step, border)
        swc.set_debug(2)
        try:
            b, fb = gpu_corr(x, y, window, step, border)
        finally:
            swc.set_debug(0)
        assert np.array_equal(fa, fb)
        if dtype != "f32":
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_parity_3d_missing_enters_mid_march():
    """Missing values that first enter a tile's window after many clean
    planes (and leave it again), on the specialised step."""
    x, y = random_pair((40, 16, 128), "f32", seed=12, kind="lognormal")
    x[25, 7, 33] = -1000.0
    y[31, 2, 90] = np.inf
    x[38, 15, 127] = np.nan
    for border in ("clip", "fill"):
        compare(x, y, (7, 7, 7), 1, border, tag="3d-missing-late", params=(4, 40, 1, 0, 2))
        compare(x, y, (5, 5, 5), 1, border, tag="3d-missing-late")


def test_parity_3d_missing_dense_square():
    """About one value in fifty missing, from the first plane on, on the
    specialised step (rows a multiple of 4 long) for every compiled window
    width, whole-wave and half-wave tiles: the steps that carry missing
    counts against the oracle, output by output."""
    x, y = random_pair((20, 18, 128), "f32", seed=21, kind="lognormal")
    rng = np.random.default_rng(5)
    x[rng.random(x.shape) < 0.02] = -1000.0
    y[rng.random(y.shape) < 0.01] = np.nan
    for k in (3, 5, 7, 9):
        for border in ("clip", "fill"):
            compare(x, y, (k, k, k), 1, border, tag="3d-missing-dense")
    compare(x, y, (7, 7, 7), 1, "clip", tag="3d-missing-dense", params=(4, 8, 1, 0, 2))
    # 256-wide rows take the half-wave tiles (three halves instead of two waves)
    x, y = random_pair((12, 10, 256), "f32", seed=22, kind="lognormal")
    x[rng.random(x.shape) < 0.02] = -1000.0
    y[rng.random(y.shape) < 0.01] = np.inf
    for k in (5, 7):
        compare(x, y, (k, k, k), 1, "clip", tag="3d-missing-dense-halves")
