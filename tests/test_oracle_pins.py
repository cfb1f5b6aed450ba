"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself:
  * an exact rational brute force (tests/exactref.py) on tiny inputs;
  * library special cases (numpy.corrcoef, scipy.stats.pearsonr, pandas
    rolling correlation, scipy.ndimage box sums fed into the paper's
    one-pass sums formula of Section 1);
  * closed-form invariants of the Pearson coefficient;
  * hand-derived golden cases (tests/golden/hand_cases.json);
  * exactly constructed float32 rounding midpoints.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import exactref
from workloads import random_pair

HERE = os.path.dirname(os.path.abspath(__file__))


def _flat(a):
    return np.asarray(a).ravel()


def _check_against_exact(x, y, window, step, border, tol64=1e-12):
    c32, c64, fl = oracle.corr(x, y, window, step, border)
    e32, e64, efl = exactref.exact_corr(x, y, window, step, border)
    assert c32.size == e32.size
    np.testing.assert_array_equal(_flat(fl), efl)
    ok = efl == 0
    assert np.all(np.abs(_flat(c64)[ok] - e64[ok]) <= tol64)
    if x.dtype.kind == "u":
        np.testing.assert_array_equal(_flat(c32).view(np.uint32), e32.view(np.uint32))
    else:
        # float input: c32 = float32(c64); the exact value rounds to within 1 ulp
        d = np.abs(_flat(c32)[ok].astype(np.float64) - e64[ok])
        assert np.all(d <= np.spacing(np.abs(e32[ok])) + 1e-15)
    # flagged outputs carry the invalid value
    assert np.all(_flat(c32)[~ok] == np.float32(-2.0))


SHAPES = {1: [(1,), (5,), (13,)], 2: [(1, 1), (3, 4), (6, 9), (9, 7)],
          3: [(2, 3, 4), (4, 5, 3)]}


@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("border", ["fill", "clip", "valid"])
def test_oracle_matches_exact_bruteforce(ndim, dtype, border):
    rng = np.random.default_rng(100 * ndim + len(dtype) + len(border))
    for shape in SHAPES[ndim]:
        for trial in range(3):
            window = tuple(int(v) for v in rng.integers(1, 5, ndim))
            step = tuple(int(v) for v in rng.integers(1, 4, ndim))
            if border == "valid" and any(s < k for s, k in zip(shape, window)):
                window = tuple(min(k, s) for k, s in zip(window, shape))
            if dtype == "f32":
                x = rng.normal(size=shape).astype(np.float32)
                y = (0.5 * x + rng.normal(size=shape)).astype(np.float32)
            else:
                hi = 4 if trial == 0 else (255 if dtype == "u8" else 65535)
                nt = np.uint8 if dtype == "u8" else np.uint16
                x = rng.integers(0, hi + 1, size=shape).astype(nt)
                y = rng.integers(0, hi + 1, size=shape).astype(nt)
            _check_against_exact(x, y, window, step, border)


def test_oracle_float_specials_bruteforce():
    """Missing values (<= -999 inclusive, NaN, +-Inf) and constant patches."""
    rng = np.random.default_rng(7)
    x = rng.normal(size=(7, 8)).astype(np.float32)
    y = rng.normal(size=(7, 8)).astype(np.float32)
    x[1, 1] = -999.0          # exactly the threshold: missing
    x[5, 6] = -998.9          # above the threshold: a valid value
    y[3, 0] = np.nan
    y[6, 7] = np.inf
    x[0, 5] = -np.inf
    x[4:7, 2:5] = 3.25        # constant patch (3x3)
    y[4:7, 2:5] = -1.5
    for border in ("fill", "clip", "valid"):
        for window, step in (((3, 3), (1, 1)), ((2, 3), (2, 1)), ((3, 2), (1, 3))):
            _check_against_exact(x, y, window, step, border)


def test_oracle_shapes_smaller_than_window():
    x, y = random_pair((2, 3), "f32", seed=3)
    _check_against_exact(x, y, (5, 7), (1, 1), "clip")
    c32, _, fl = oracle.corr(x, y, (5, 7), 1, "fill")
    assert np.all(fl == exactref.BORDER) and np.all(c32 == -2.0)
    with pytest.raises(ValueError):
        oracle.corr(x, y, (5, 7), 1, "valid")


def test_output_shape_rule():
    assert oracle.output_shape((3000, 4000), (7, 7), 1, "fill") == (3000, 4000)
    assert oracle.output_shape((4096, 4096), (31, 31), 4, "clip") == (1024, 1024)
    assert oracle.output_shape((7,), (3,), 2, "fill") == (4,)
    assert oracle.output_shape((10, 9), (3, 4), (2, 3), "valid") == (4, 2)
    assert oracle.output_shape((5,), (5,), 3, "valid") == (1,)


# --------------------------------------------------------------------------
# Library special cases
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(50,), (9, 11), (4, 5, 6)])
def test_full_window_equals_numpy_and_scipy(shape):
    from scipy.stats import pearsonr
    x, y = random_pair(shape, "f32", seed=11)
    _, c64, fl = oracle.corr(x, y, shape, 1, "valid")
    assert fl.size == 1 and fl.ravel()[0] == 0
    ref = np.corrcoef(x.ravel().astype(np.float64), y.ravel().astype(np.float64))[0, 1]
    assert abs(c64.ravel()[0] - ref) < 1e-12
    assert abs(c64.ravel()[0] - pearsonr(x.ravel().astype(np.float64),
                                         y.ravel().astype(np.float64))[0]) < 1e-12


@pytest.mark.parametrize("k", [3, 4, 7, 10])
def test_1d_clip_equals_pandas_rolling(k):
    """pandas' centred rolling window puts one more cell before the centre
    for even k, like the reading taken here."""
    import pandas as pd
    x, y = random_pair((300,), "f32", seed=k)
    _, c64, fl = oracle.corr(x, y, k, 1, "clip")
    ref = pd.Series(x.astype(np.float64)).rolling(k, center=True, min_periods=2).corr(
        pd.Series(y.astype(np.float64))).to_numpy()
    assert np.all(fl == 0)
    np.testing.assert_allclose(c64, ref, rtol=0, atol=1e-9)


def _box_sum(a, window):
    """Box sum over a centred window with zero padding (scipy uniform_filter
    averages over the full window size; multiply back)."""
    from scipy.ndimage import uniform_filter
    return uniform_filter(a, size=window, mode="constant", cval=0.0) * float(np.prod(window))


@pytest.mark.parametrize("shape,window", [((40, 37), (7, 7)), ((33, 20), (4, 5)),
                                          ((12, 14, 16), (3, 5, 4))])
def test_box_sums_via_scipy_equal_oracle(shape, window):
    """Section 1: the coefficient from box sums of x, y, xy, x^2, y^2 (the
    one-pass sums formula) equals the two-pass oracle on well-conditioned
    data (CLIP: n = in-bounds count)."""
    x, y = random_pair(shape, "f32", seed=5)
    x64, y64 = x.astype(np.float64), y.astype(np.float64)
    n = _box_sum(np.ones(shape), window)
    sx, sy = _box_sum(x64, window), _box_sum(y64, window)
    sxy, sxx, syy = _box_sum(x64 * y64, window), _box_sum(x64 * x64, window), _box_sum(y64 * y64, window)
    n = np.round(n)
    num = n * sxy - sx * sy
    den = np.sqrt(n * sxx - sx * sx) * np.sqrt(n * syy - sy * sy)
    ref = num / den
    _, c64, fl = oracle.corr(x, y, window, 1, "clip")
    assert np.all(fl == 0)
    np.testing.assert_allclose(c64, ref, rtol=0, atol=1e-9)


# --------------------------------------------------------------------------
# Invariants
# --------------------------------------------------------------------------

def test_exact_linear_relation_gives_sign():
    rng = np.random.default_rng(1)
    x = rng.integers(0, 20000, size=(20, 30)).astype(np.uint16)
    y_pos = (3 * x.astype(np.int64) + 7).astype(np.uint16)
    y_neg = (60001 - 3 * x.astype(np.int64)).astype(np.uint16)
    for y, s in ((y_pos, 1.0), (y_neg, -1.0)):
        c32, c64, fl = oracle.corr(x, y, (5, 5), 1, "clip")
        ok = fl == 0
        assert ok.sum() > 500
        assert np.all(c32[ok] == np.float32(s))
        assert np.all(np.abs(c64[ok] - s) < 1e-12)


def test_symmetry_and_affine_invariance_integer_exact():
    x, y = random_pair((25, 31), "u16", seed=4)
    x = (x // 4).astype(np.uint16)
    y = (y // 4).astype(np.uint16)
    c_xy, _, f_xy = oracle.corr(x, y, (5, 3), 1, "clip")
    c_yx, _, f_yx = oracle.corr(y, x, (5, 3), 1, "clip")
    np.testing.assert_array_equal(c_xy.view(np.uint32), c_yx.view(np.uint32))
    sw = {0: 0, 4: 8, 8: 4, 12: 12}
    np.testing.assert_array_equal(np.vectorize(sw.get)(f_xy), f_yx)
    # c(a x + b, g y + d) = sign(a g) c(x, y), exactly for integer maps
    xa = (3 * x.astype(np.int64) + 11).astype(np.uint16)
    yg = (65535 - 2 * y.astype(np.int64)).astype(np.uint16)
    c_t, _, f_t = oracle.corr(xa, yg, (5, 3), 1, "clip")
    np.testing.assert_array_equal(f_t, f_xy)
    ok = f_xy == 0
    np.testing.assert_array_equal(c_t[ok].view(np.uint32), (-c_xy[ok]).view(np.uint32))


def test_bounds_and_self_correlation():
    x, y = random_pair((64, 64), "f32", seed=9, kind="lognormal")
    c32, c64, fl = oracle.corr(x, y, (7, 7), 1, "clip")
    ok = fl == 0
    assert np.all(np.abs(c64[ok]) <= 1.0)
    c32s, c64s, fls = oracle.corr(x, x, (7, 7), 1, "clip")
    assert np.all(np.abs(c64s[fls == 0] - 1.0) < 1e-12)


def test_translation_equivariance_with_step():
    """Shifting the input by a multiple of the step shifts the output grid."""
    x, y = random_pair((40, 44), "f32", seed=12)
    s0, s1, a, b = 2, 3, 2, 3
    full, _, ff = oracle.corr(x, y, (5, 5), (s0, s1), "fill")
    sh, _, fs = oracle.corr(x[a * s0:, b * s1:], y[a * s0:, b * s1:], (5, 5), (s0, s1), "fill")
    reg = full[a:a + sh.shape[0], b:b + sh.shape[1]]
    freg = ff[a:a + sh.shape[0], b:b + sh.shape[1]]
    inside = fs == 0
    assert inside.sum() > 50
    assert np.all(freg[inside] == 0)
    np.testing.assert_array_equal(reg[inside].view(np.uint32), sh[inside].view(np.uint32))


def test_transpose_equivariance():
    x, y = random_pair((17, 23), "u8", seed=13)
    a, _, fa = oracle.corr(x, y, (3, 5), (1, 2), "clip")
    b, _, fb = oracle.corr(x.T.copy(), y.T.copy(), (5, 3), (2, 1), "clip")
    np.testing.assert_array_equal(a.T.view(np.uint32), b.view(np.uint32))
    np.testing.assert_array_equal(fa.T, fb)


def test_constant_patch_flags_exactly_windows_inside():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(30, 30)).astype(np.float32)
    y = rng.normal(size=(30, 30)).astype(np.float32)
    x[10:20, 5:15] = 4.0
    _, _, fl = oracle.corr(x, y, (5, 5), 1, "fill")
    expect = np.zeros((30, 30), bool)
    expect[12:18, 7:13] = True          # centres whose 5x5 window lies in the patch
    assert np.array_equal((fl & exactref.ZVAR_X) != 0, expect)
    assert not np.any(fl & exactref.ZVAR_Y)


def test_single_missing_flags_exactly_covering_windows():
    x, y = random_pair((21, 19), "f32", seed=2)
    y[8, 11] = -1000.0
    _, _, fl = oracle.corr(x, y, (3, 5), 1, "clip")
    expect = np.zeros((21, 19), bool)
    expect[7:10, 9:14] = True
    assert np.array_equal(fl == exactref.MISSING, expect)


def test_fill_frame_width_even_and_odd():
    x, y = random_pair((12, 15), "f32", seed=8)
    _, _, fl = oracle.corr(x, y, (4, 5), 1, "fill")
    b = fl == exactref.BORDER
    # k=4: 2 cells before, 1 after; k=5: 2 and 2
    expect = np.ones((12, 15), bool)
    expect[2:12 - 1, 2:15 - 2] = False
    assert np.array_equal(b, expect)


# --------------------------------------------------------------------------
# Exactly rounded float32 (integer input)
# --------------------------------------------------------------------------

def _rn32_exact_fraction(P, Q, R):
    c2 = Fraction(P * P, Q * R)
    return exactref.rn32_from_exact((P > 0) - (P < 0), c2)


def test_rn32_constructed_midpoints_and_ties():
    """Choose Q = R = 2^m so that c = P / 2^m is a dyadic rational, and place
    it exactly on, just below and just above float32 rounding midpoints."""
    rng = np.random.default_rng(0)
    checked = 0
    for _ in range(300):
        f = np.float32(rng.uniform(0.01, 1.0))
        up = np.nextafter(f, np.float32(2.0))
        mid = (Fraction(float(f)) + Fraction(float(up))) / 2
        m = 60
        P0 = mid * 2 ** m
        assert P0.denominator == 1
        P0 = int(P0)
        for dP in (-1, 0, 1):
            P = P0 + dP
            got = oracle.rn32_ratio(P, 2 ** m, 2 ** m)
            want = _rn32_exact_fraction(P, 2 ** m, 2 ** m)
            assert got.view(np.uint32) == want.view(np.uint32)
            if dP == 0:   # exact tie: the even neighbour
                even = f if (f.view(np.uint32) & 1) == 0 else up
                assert got == even
            checked += 1
            got_n = oracle.rn32_ratio(-P, 2 ** m, 2 ** m)
            assert got_n == -got
    assert checked == 900


def test_rn32_random_operands():
    rng = np.random.default_rng(1)
    for _ in range(2000):
        Q = int(rng.integers(1, 2 ** 62))
        R = int(rng.integers(1, 2 ** 62))
        lim = math.isqrt(Q * R)
        P = int(rng.integers(-min(lim, 2 ** 62), min(lim, 2 ** 62) + 1))
        got = oracle.rn32_ratio(P, Q, R)
        want = _rn32_exact_fraction(P, Q, R)
        assert got.view(np.uint32) == want.view(np.uint32)


def test_integer_c32_within_half_ulp_of_c64():
    x, y = random_pair((60, 70), "u16", seed=21)
    c32, c64, fl = oracle.corr(x, y, (7, 7), 1, "fill")
    ok = fl == 0
    assert np.all(np.abs(c32[ok].astype(np.float64) - c64[ok]) <= 2.0 ** -24)


# --------------------------------------------------------------------------
# Golden hand-derived cases
# --------------------------------------------------------------------------

def _token_value(tok):
    if tok in ("1", "-1"):
        return 0, int(tok), Fraction(1)
    if tok == "B":
        return exactref.BORDER, 0, None
    if tok == "M":
        return exactref.MISSING, 0, None
    if tok.startswith("Z"):
        return int(tok[1:]), 0, None
    sign = -1 if tok.startswith("-") else 1
    p, q = tok.lstrip("-r").split("/")
    return 0, sign, Fraction(int(p), int(q))


def test_golden_hand_cases():
    with open(os.path.join(HERE, "golden", "hand_cases.json")) as f:
        cases = json.load(f)["cases"]
    nt = {"u8": np.uint8, "u16": np.uint16, "f32": np.float32}
    for case in cases:
        shape = tuple(case["shape"])
        x = np.array(case["x"], dtype=nt[case["dtype"]]).reshape(shape)
        y = np.array(case["y"], dtype=nt[case["dtype"]]).reshape(shape)
        c32, c64, fl = oracle.corr(x, y, case["window"], case["step"], case["border"])
        exp = [_token_value(t) for t in case["expect"]]
        assert c32.size == len(exp), case["name"]
        for i, (ef, es, ec2) in enumerate(exp):
            assert fl.ravel()[i] == ef, (case["name"], i)
            if ef:
                assert c32.ravel()[i] == np.float32(-2.0)
                continue
            want64 = es * math.sqrt(float(ec2))
            assert abs(c64.ravel()[i] - want64) < 1e-15, (case["name"], i)
            want32 = exactref.rn32_from_exact(es, ec2)
            if case["dtype"] != "f32":
                assert c32.ravel()[i].view(np.uint32) == want32.view(np.uint32), (case["name"], i)
            else:
                assert abs(float(c32.ravel()[i]) - want64) <= np.spacing(np.float32(abs(want64)))


def test_cloud_mask_pins():
    """The application's cloud test (Introduction: under clouds the visible
    and infrared channels move in opposite directions, c close to -1):
    an exactly anti-linear patch gives c = -1 and is masked for every
    tau < 1, never for tau = 1; a co-linear patch is never masked; border
    outputs (FILL) and constant windows are never masked."""
    rng = np.random.default_rng(41)
    x = rng.integers(100, 2000, size=(40, 60)).astype(np.uint16)
    y = rng.integers(100, 2000, size=(40, 60)).astype(np.uint16)
    x[5:25, 10:30] = rng.integers(1000, 5000, size=(20, 20))
    y[5:25, 10:30] = (30000 - 3 * x[5:25, 10:30].astype(np.int64)).astype(np.uint16)
    x[5:25, 35:55] = rng.integers(1000, 5000, size=(20, 20))
    y[5:25, 35:55] = (7 + 2 * x[5:25, 35:55].astype(np.int64)).astype(np.uint16)
    y[30:38, 0:20] = 4444                                   # constant y patch
    c32, _, fl = oracle.corr(x, y, (5, 5), 1, "fill")
    inner_anti = (slice(7, 23), slice(12, 28))              # windows inside the patch
    inner_co = (slice(7, 23), slice(37, 53))
    assert np.all(c32[inner_anti] == np.float32(-1.0))
    assert np.all(c32[inner_co] == np.float32(1.0))
    for tau in (0.0, 0.5, 0.9, 0.999):
        m = oracle.cloud_mask(c32, fl, tau)
        assert np.all(m[inner_anti] == 1)
        assert np.all(m[inner_co] == 0)
        assert np.all(m[fl != 0] == 0)
        assert np.all(m[:2, :] == 0) and np.all(m[:, -2:] == 0)
    assert np.all(oracle.cloud_mask(c32, fl, 1.0) == 0)
    assert np.all(fl[32:36, 2:18] & oracle.FLAG_ZVAR_Y)
