"""GPU parity of the fused 2-D kernel against the CPU oracle (through the C ABI).

Integer inputs: bit-exact c and flags.  Float inputs: identical flags and
|dc| <= 2^-24 against the oracle's FP64 two-pass value.  Sizes span several
tiles with ragged tails; edge cases cover tiny grids, windows larger than the
grid, even windows, steps, every border policy, missing values, constant
patches and every launch-parameter family.
"""
import numpy as np
import pytest

from gpu_util import compare, say
from workloads import random_pair, cloud_pair, paper_shaped_u16

pytestmark = pytest.mark.gpu

BORDERS = ["fill", "clip", "valid"]


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("border", BORDERS)
def test_parity_basic_shapes(dtype, border):
    for shape, window, step in [((37, 300), (7, 7), 1), ((130, 517), (3, 5), 1),
                                ((64, 257), (4, 6), 1), ((71, 150), (7, 7), (2, 3)),
                                ((40, 90), (5, 5), (4, 4)), ((33, 65), (1, 1), 1),
                                ((50, 700), (9, 15), 1)]:
        x, y = random_pair(shape, dtype, seed=hash((shape, window)) % 1000)
        compare(x, y, window, step, border, tag="basic")


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_parity_tiny_and_degenerate(dtype):
    for shape, window, border in [((1, 1), (1, 1), "fill"), ((1, 1), (3, 3), "clip"),
                                  ((2, 3), (5, 7), "fill"), ((2, 3), (5, 7), "clip"),
                                  ((5, 3), (5, 3), "valid"), ((1, 50), (1, 7), "clip"),
                                  ((50, 1), (7, 1), "clip"), ((3, 4), (2, 2), "valid")]:
        x, y = random_pair(shape, dtype, seed=3)
        compare(x, y, window, 1, border, tag="tiny")


@pytest.mark.parametrize("dtype", ["u8", "u16"])
def test_parity_integer_extremes_and_constants(dtype):
    rng = np.random.default_rng(5)
    hi = 255 if dtype == "u8" else 65535
    nt = np.uint8 if dtype == "u8" else np.uint16
    x = rng.choice(np.array([0, 1, hi - 1, hi]), size=(90, 333)).astype(nt)
    y = rng.integers(0, hi + 1, size=(90, 333)).astype(nt)
    x[10:30, 40:90] = hi          # constant patch in x
    y[50:60, 100:200] = 0         # constant patch in y
    x[70:80, 250:300] = 7
    y[70:80, 250:300] = 9         # both constant
    for border in BORDERS:
        compare(x, y, (5, 5), 1, border, tag="extremes")
        compare(x, y, (7, 3), (1, 2), border, tag="extremes")
    # exact linear relation: c = +-1 exactly
    x2 = rng.integers(0, hi // 4, size=(60, 200)).astype(nt)
    y2 = (hi - 3 * x2.astype(np.int64)).astype(nt)
    compare(x2, y2, (7, 7), 1, "clip", tag="linear")


def test_parity_float_missing_and_constant():
    rng = np.random.default_rng(9)
    x, y = random_pair((120, 400), "f32", seed=9, kind="lognormal")
    x[5, 7] = -999.0
    x[60, 300] = -1e30
    y[33, 100] = np.nan
    y[90, 390] = np.inf
    x[100, 20] = -np.inf
    x[20:40, 150:230] = 2.5
    y[20:40, 200:260] = -7.25
    x[70:90, 10:60] = 0.0
    for border in BORDERS:
        for window, step in (((7, 7), 1), ((3, 9), (2, 1)), ((6, 4), 1)):
            compare(x, y, window, step, border, tag="float-specials")


def test_parity_float_missing_enters_mid_march():
    """Float rows are parked in the LDS ring as read; a leaving row's missing
    positions are found again only once a missing value has entered the
    tile.  Missing values that first appear deep in a tile's march (one tile
    per column band, 256-row tiles), leave its windows again, and a threshold
    of 0 (zeros then missing, while the ring's initial zeros and positions
    outside the array are not): every output against the oracle, for every
    window width the ring serves."""
    x, y = random_pair((200, 300), "f32", seed=31, kind="lognormal")
    x[90, 40] = -1000.0
    y[120, 200:204] = np.nan
    x[150, 290] = -np.inf
    for k in (3, 5, 7, 9):
        compare(x, y, (k, k), 1, "clip", params=(4, 256, 1), tag="float-missing-late")
        compare(x, y, (k, k), 1, "fill", tag="float-missing-late")
    z = x.copy()
    z[100:103, 50:60] = 0.0
    compare(z, y, (7, 7), 1, "clip", params=(4, 256, 1), missing_le=0.0, tag="float-missing-late-thr0")
    compare(z, y, (9, 9), 1, "fill", params=(4, 256, 1), missing_le=0.0, tag="float-missing-late-thr0")


def test_parity_offset_data_cancellation():
    """x ~ N(1000, 1): the sums cancel heavily; still within 2^-24."""
    for window in ((3, 3), (7, 7), (15, 15), (31, 31)):
        x, y = random_pair((200, 300), "f32", seed=1, kind="offset", rho=0.7)
        compare(x, y, window, 1, "clip", tag="offset")


@pytest.mark.parametrize("params", [(1, 1, 1), (1, 13, 2), (2, 7, 4), (4, 32, 4), (4, 5, 1),
                                    (8, 16, 2), (8, 64, 1)])
def test_parity_launch_params(params):
    for dtype in ("u16", "f32", "u8"):
        x, y = random_pair((150, 700), dtype, seed=17)
        compare(x, y, (7, 7), 1, "fill", params=params, tag="params")
        compare(x, y, (5, 9), (2, 1), "clip", params=params, tag="params")


def test_integer_determinism_across_params():
    import paper_1807_06507_amd as swc
    from gpu_util import gpu_corr
    x, y = random_pair((300, 900), "u16", seed=23)
    ref = None
    for params in [(1, 8, 4), (2, 16, 2), (4, 32, 4), (8, 24, 1), None]:
        c, fl = gpu_corr(x, y, (7, 7), 1, "fill", params=params)
        if ref is None:
            ref = (c, fl)
        assert np.array_equal(c.view(np.uint32), ref[0].view(np.uint32))
        assert np.array_equal(fl, ref[1])
        c2, _ = gpu_corr(x, y, (7, 7), 1, "fill", params=params)
        assert np.array_equal(c2.view(np.uint32), c.view(np.uint32))


def test_forced_exact_fallbacks_do_not_change_results():
    import paper_1807_06507_amd as swc
    from gpu_util import gpu_corr
    for dtype in ("u16", "u8", "f32"):
        x, y = random_pair((80, 300), dtype, seed=31)
        a, fa = gpu_corr(x, y, (7, 7), 1, "clip")
        swc.set_debug(1)
        try:
            b, fb = gpu_corr(x, y, (7, 7), 1, "clip")
        finally:
            swc.set_debug(0)
        assert np.array_equal(fa, fb)
        if dtype != "f32":
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        else:
            assert np.max(np.abs(a.astype(np.float64) - b)) <= 2.0 ** -23
        compare(x, y, (7, 7), 1, "clip", tag="forced")


def test_comparator_modes_run():
    x, y = random_pair((100, 300), "f32", seed=4)
    dn = compare(x, y, (7, 7), 1, "clip", accum="naive", tag="naive")
    dc = compare(x, y, (7, 7), 1, "clip", accum="comp", tag="comp")
    say(f"naive max|dc|={dn:.3e} comp max|dc|={dc:.3e}")


def test_parity_config_small_cloud_pair():
    """The small configuration: 1024x768 f32 cloud pair, 7x7, step 1, CLIP."""
    x, y = cloud_pair((768, 1024), seed=0)
    d = compare(x, y, (7, 7), 1, "clip", tag="c0")
    say(f"c0 max|dc| = {d:.3e}")


def test_parity_config_paper_shaped_full():
    """The paper-shaped configuration at full size (4000x3000 u16, 7x7, FILL):
    every output, bit-exact."""
    import paper_1807_06507_amd as swc
    from gpu_util import gpu_corr
    x, y = paper_shaped_u16((3000, 4000), seed=2)
    compare(x, y, (7, 7), 1, "fill", tag="c1-full")
    # every output through the exact big-integer decision: identical bits,
    # so the certified FP64 estimate never rounded differently (12M samples)
    a, fa = gpu_corr(x, y, (7, 7), 1, "fill")
    swc.set_debug(1)
    try:
        b, fb = gpu_corr(x, y, (7, 7), 1, "fill")
    finally:
        swc.set_debug(0)
    assert np.array_equal(fa, fb)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_register_and_lds_kernels_agree(dtype):
    """The register-resident kernel (compiled window widths) and the generic
    LDS kernel give identical integer results and flags, and both match the
    oracle."""
    import paper_1807_06507_amd as swc
    from gpu_util import gpu_corr
    for shape, window, step, border, params in [
            ((300, 1000), (7, 7), 1, "fill", (4, 32, 4)),
            ((211, 777), (3, 9), (1, 2), "clip", (4, 16, 2)),
            ((97, 1290), (5, 15), 1, "valid", (8, 24, 1)),
            ((64, 64), (9, 5), (3, 1), "clip", (4, 7, 4))]:
        x, y = random_pair(shape, dtype, seed=41)
        a, fa = gpu_corr(x, y, window, step, border, params=params)
        swc.set_debug(2)
        try:
            b, fb = gpu_corr(x, y, window, step, border, params=params)
        finally:
            swc.set_debug(0)
        assert np.array_equal(fa, fb)
        if dtype != "f32":
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        compare(x, y, window, step, border, params=params, tag="fast-kernel")


@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_prepared_launch_equals_direct_call(dtype):
    """A prepared launch (arguments marshalled once) gives the same map as the
    direct call, on every repeat, with flags."""
    import torch
    import paper_1807_06507_amd as swc
    from gpu_util import to_dev
    x, y = random_pair((301, 1000), dtype, seed=43)
    xd, yd = to_dev(x), to_dev(y)
    ref, fref = swc.corr(xd, yd, (7, 7), 1, "clip", return_flags=True)
    p = swc.make_problem(x.shape, xd.dtype, (7, 7), 1, "clip")
    out = torch.full(ref.shape, 5.0, dtype=torch.float32, device="cuda")
    fl = torch.full(ref.shape, 77, dtype=torch.uint8, device="cuda")
    go = swc.prepare(p, xd, yd, out, fl)
    for _ in range(3):
        go()
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32))
        assert torch.equal(fl, fref)
        out.fill_(5.0)
        fl.fill_(77)


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
def test_maps_with_and_without_flag_map_agree(dtype):
    """Launches that write a flag map and launches that do not (float input
    has separate code for each) give bit-identical coefficient maps,
    including border, missing and constant windows, in vector-store and
    per-column tiles."""
    import torch
    import paper_1807_06507_amd as swc
    from gpu_util import to_dev
    for shape, window, step, border in [((130, 1000), (7, 7), 1, "fill"),
                                        ((97, 517), (5, 3), 1, "clip"),
                                        ((64, 301), (7, 7), (2, 3), "valid")]:
        x, y = random_pair(shape, dtype, seed=47)
        if dtype == "f32":
            x[5, 40] = -1000.0
            y[60, 200] = np.nan
            x[20:40, 100:160] = 3.0
        else:
            x[20:40, 100:160] = 9
        xd, yd = to_dev(x), to_dev(y)
        a, fl = swc.corr(xd, yd, window, step, border, return_flags=True)
        b = swc.corr(xd, yd, window, step, border)
        torch.cuda.synchronize()
        say(f"flags/no-flags {dtype} {shape} {window} {step} {border}")
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))
        assert int((fl != 0).sum()) > 0
