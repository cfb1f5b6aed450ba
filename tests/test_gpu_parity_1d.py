"""GPU parity of the 1-D kernel (moving sums of Section 1 in one dimension)
against the CPU oracle, through the C ABI.

Integer inputs: bit-exact c and flags.  Float inputs: identical flags and
|dc| <= 2^-24.  Windows from 1 to 2000 (1448 for uint16, its exact limit) (below and above one 512-sample row),
steps, all border policies, missing values, constant runs; the long-series
configuration (AR(1) pair, k = 1001) at 2^20 samples on every output and at
its full 2^28 samples on a sample of outputs.
"""
import numpy as np
import pytest

from gpu_util import compare, say
from workloads import random_pair, series_1d

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("border", ["fill", "clip", "valid"])
def test_parity_1d_windows(dtype, border):
    for n, k, s in [(1, 1, 1), (5, 3, 1), (100, 7, 1), (3000, 64, 1), (5000, 511, 1),
                    (5000, 513, 2), (9000, 1001, 1), (4000, 2000, 3), (777, 8, 4), (2, 5, 1)]:
        if dtype == "u16" and k > 1448:
            k = 1448            # the exact u16 path's window-size limit
        if border == "valid" and n < k:
            continue
        x, y = random_pair((n,), dtype, seed=n + k)
        compare(x, y, (k,), (s,), border, tag="1d")


def test_parity_1d_missing_and_constant():
    x, y = random_pair((6000,), "f32", seed=3, kind="lognormal")
    x[100] = -999.0
    y[2500] = np.nan
    x[4000] = np.inf
    x[1000:1500] = 2.0          # constant run longer than the window
    y[3000:3100] = -4.0
    for k in (3, 101, 1001):
        compare(x, y, (k,), 1, "clip", tag="1d-specials")
        compare(x, y, (k,), 1, "fill", tag="1d-specials")


def test_parity_1d_missing_enters_late():
    """Missing values that first enter a wave's span after many clean rows
    (the leaving values are looked at one by one only from then on), in the
    initial window of a span, and a threshold of 0 (zeros missing; positions
    outside the series are not): every output, ring and re-read paths, and
    several waves per series (short spans)."""
    import paper_1807_06507_amd as swc
    x, y = random_pair((90000,), "f32", seed=8, kind="lognormal")
    x[40000] = -5000.0
    y[61234:61240] = np.nan
    x[88000] = -np.inf
    for k in (5, 101, 1001):
        for params in (None, (8, 4, 1)):
            compare(x, y, (k,), 1, "clip", params=params, tag="1d-missing-late")
        compare(x, y, (k,), 1, "fill", tag="1d-missing-late")
    swc.set_debug(4)
    try:
        compare(x, y, (1001,), 1, "clip", tag="1d-missing-late-reread")
    finally:
        swc.set_debug(0)
    z = x.copy()
    z[30000:30010] = 0.0
    compare(z, y, (101,), 1, "fill", params=(8, 4, 1), missing_le=0.0, tag="1d-missing-thr0")


@pytest.mark.parametrize("dtype", ["u8", "u16"])
def test_parity_1d_integer_constant_runs(dtype):
    rng = np.random.default_rng(11)
    hi = 255 if dtype == "u8" else 65535
    nt = np.uint8 if dtype == "u8" else np.uint16
    x = rng.integers(0, hi + 1, 20000).astype(nt)
    y = rng.integers(0, hi + 1, 20000).astype(nt)
    x[5000:7000] = hi
    y[12000:12600] = 3
    for k in (5, 512, 1001):
        compare(x, y, (k,), 1, "clip", tag="1d-int")


def test_parity_1d_launch_params():
    x, y = random_pair((50000,), "f32", seed=5)
    for params in [(8, 1, 1), (8, 3, 2), (8, 16, 1), (8, 64, 2)]:
        compare(x, y, (1001,), 1, "clip", params=params, tag="1d-params")
        compare(x, y, (17,), 1, "fill", params=params, tag="1d-params")


def test_parity_long_series_reduced():
    """AR(1) pair (phi = 0.95, innovation correlation 0.5), k = 1001, CLIP,
    2^20 samples: every output."""
    x, y = series_1d(1 << 20, seed=5)
    d = compare(x, y, (1001,), 1, "clip", tag="c4b-2^20")
    say(f"c4b reduced max|dc| = {d:.3e}")


def test_parity_long_series_full_sampled():
    """The full 2^28-sample series: 20000 sampled outputs plus the first and
    last 500 (border region), compared with the oracle one by one."""
    x, y = series_1d(1 << 28, seed=5)
    n = x.size
    rng = np.random.default_rng(0)
    idx = np.unique(np.concatenate([rng.integers(0, n, 20000), np.arange(500),
                                    np.arange(n - 500, n)]))
    d = compare(x, y, (1001,), 1, "clip", indices=idx, tag="c4b-full")
    say(f"c4b full (sampled) max|dc| = {d:.3e}")


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_parity_1d_ring_and_reread_paths(dtype):
    """Leaving values from the per-wave LDS ring (windows up to ~3500) and
    re-read from memory (debug bit 2, and windows too wide for the ring):
    both match the oracle; integer results are identical bit for bit."""
    import paper_1807_06507_amd as swc
    from gpu_util import gpu_corr
    x, y = random_pair((70001,), dtype, seed=44)
    for k in (1, 7, 100, 511, 512, 513, 1001, 3000, 3600):
        if dtype == "u16" and k > 1448:
            continue
        for border in ("clip", "fill"):
            compare(x, y, (k,), 1, border, tag="1d-ring")
            a, fa = gpu_corr(x, y, (k,), 1, border)
            swc.set_debug(4)
            try:
                b, fb = gpu_corr(x, y, (k,), 1, border)
            finally:
                swc.set_debug(0)
            assert np.array_equal(fa, fb)
            if dtype != "f32":
                assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    xs, ys = random_pair((30000,), dtype, seed=45)
    compare(xs, ys, (257,), (3,), "clip", tag="1d-ring-step")
