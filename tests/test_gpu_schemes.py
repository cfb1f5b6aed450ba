"""GPU parity of the unfused baseline schemes against the CPU oracle (through
the C ABI): the paper's four-phase parallel scheme (Section 2) and the
cumulative-sum (integral image) alternative of Section 1.

Same bar as the fused kernels: integer inputs bit-exact c and flags; float
inputs identical flags and |dc| <= 2^-24.  Shapes span many threads' lines
with ragged sizes; edge cases cover windows larger than the grid, even
windows, constant patches, missing values and both same-size borders.  At
the paper-shaped full size (4000x3000 u16, 7x7, FILL) both schemes must give
exactly the fused kernel's bits (all three are correctly rounded).
"""
import numpy as np
import pytest

from gpu_util import compare, gpu_corr, say
from workloads import random_pair, cloud_pair, paper_shaped_u16

pytestmark = pytest.mark.gpu

SHAPES = [((37, 300), (7, 7)), ((130, 517), (3, 5)), ((64, 257), (4, 6)), ((33, 65), (1, 1)),
          ((50, 700), (9, 15)), ((2, 3), (5, 7)), ((1, 1), (3, 3)), ((50, 1), (7, 1))]


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("border", ["fill", "clip"])
def test_unfused_parity(dtype, border):
    for shape, window in SHAPES:
        x, y = random_pair(shape, dtype, seed=hash((shape, window)) % 1000)
        compare(x, y, window, 1, border, tag="unfused", scheme="unfused")


@pytest.mark.parametrize("dtype", ["u8", "u16"])
@pytest.mark.parametrize("border", ["fill", "clip"])
def test_cumsum_parity(dtype, border):
    for shape, window in SHAPES:
        x, y = random_pair(shape, dtype, seed=hash((shape, window)) % 1000 + 1)
        compare(x, y, window, 1, border, tag="cumsum", scheme="cumsum")


@pytest.mark.parametrize("scheme", ["unfused", "cumsum"])
def test_schemes_integer_extremes_and_constants(scheme):
    rng = np.random.default_rng(5)
    x = rng.choice(np.array([0, 1, 65534, 65535]), size=(90, 333)).astype(np.uint16)
    y = rng.integers(0, 65536, size=(90, 333)).astype(np.uint16)
    x[10:30, 40:90] = 65535
    y[50:60, 100:200] = 0
    x[70:80, 250:300] = 7
    y[70:80, 250:300] = 9
    for border in ("fill", "clip"):
        compare(x, y, (5, 5), 1, border, tag="extremes", scheme=scheme)
        compare(x, y, (7, 3), 1, border, tag="extremes", scheme=scheme)


def test_unfused_float_missing_constant_and_offset():
    x, y = random_pair((120, 400), "f32", seed=9, kind="lognormal")
    x[5, 7] = -999.0
    x[60, 300] = -1e30
    y[33, 100] = np.nan
    y[90, 390] = np.inf
    x[20:40, 150:230] = 2.5
    y[20:40, 200:260] = -7.25
    for border in ("fill", "clip"):
        compare(x, y, (7, 7), 1, border, tag="unfused-specials", scheme="unfused")
    # heavy cancellation (x ~ N(1000, 1)): certification or the two-pass fallback
    xo, yo = random_pair((200, 300), "f32", seed=1, kind="offset", rho=0.7)
    for window in ((3, 3), (7, 7), (15, 15)):
        compare(xo, yo, window, 1, "clip", tag="unfused-offset", scheme="unfused")


def test_unfused_small_cloud_pair():
    """The small configuration: 1024x768 f32 cloud pair, 7x7, step 1, CLIP."""
    x, y = cloud_pair((768, 1024), seed=0)
    d = compare(x, y, (7, 7), 1, "clip", tag="c0-unfused", scheme="unfused")
    say(f"c0 unfused max|dc| = {d:.3e}")


def test_schemes_full_size_equal_fused():
    """4000x3000 u16, 7x7, FILL: every output of both schemes equals the fused
    kernel's bits and flags; a sample of outputs also matches the oracle."""
    x, y = paper_shaped_u16((3000, 4000), seed=2)
    a, fa = gpu_corr(x, y, (7, 7), 1, "fill")
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(x.size, size=4000, replace=False))
    for scheme in ("unfused", "cumsum"):
        say(f"[full] scheme={scheme}")
        b, fb = gpu_corr(x, y, (7, 7), 1, "fill", scheme=scheme)
        assert np.array_equal(fa, fb)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        compare(x, y, (7, 7), 1, "fill", tag=f"full-sampled-{scheme}", indices=idx, scheme=scheme)


def test_schemes_reject_unsupported():
    import torch
    import paper_1807_06507_amd as swc
    x = torch.zeros((16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(Exception):
        swc.corr_scheme(x, x, (3, 3), "cumsum")           # float input
    with pytest.raises(Exception):
        swc.corr_scheme(x, x, (3, 3), "unfused", border="valid")
    x3 = torch.zeros((4, 8, 8), dtype=torch.uint8, device="cuda")
    with pytest.raises(Exception):
        swc.corr_scheme(x3, x3, (3, 3, 3), "unfused")     # 3-D
