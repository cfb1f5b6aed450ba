"""Exact rational brute force for tiny inputs (a pin for the oracle).

Independent of ``oracle/``: pure Python with ``fractions.Fraction``.  Every
input value is converted exactly (a float32 is a dyadic rational), the window
of each output is enumerated with Python ranges, and the classical two-pass
coefficient of the paper's Introduction is evaluated without any rounding:
means, deviations and the three deviation sums are exact rationals, so the
result is known as ``sign`` and ``c**2`` (a rational).  From that this module
derives the exactly rounded float32 (ties to even) and a float64 value.

Window convention (paper, Section 3 I/O paragraph, "middle cell"): for window
k the output at centre i covers [i - k//2, i - k//2 + k - 1]; FILL marks
windows that leave the array, CLIP keeps their in-bounds part, VALID starts
windows at the output position times the step.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction

import numpy as np

BORDER, MISSING, ZVAR_X, ZVAR_Y = 1, 2, 4, 8


def _out_len(n, k, s, border):
    if border == "valid":
        return (n - k) // s + 1 if n >= k else 0
    return -(-n // s)


def _range(p, n, k, s, border):
    """Inclusive window bounds for output p along one axis, and whether the
    window leaves the array."""
    if border == "valid":
        a = p * s
        b = a + k - 1
    else:
        a = p * s - k // 2
        b = a + k - 1
    out = a < 0 or b > n - 1
    return max(a, 0), min(b, n - 1), out


def _is_missing(v, is_float, missing_le):
    if not is_float:
        return False
    return (not math.isfinite(v)) or v <= missing_le


def exact_window_results(x, y, window, step, border, missing_le=-999.0):
    """Yield (flags, sign, c2) for every output in C order.  ``c2`` is the
    exact rational square of the coefficient (None when flagged)."""
    x = np.asarray(x)
    y = np.asarray(y)
    nd = x.ndim
    is_float = x.dtype.kind == "f"
    oshape = [_out_len(x.shape[d], window[d], step[d], border) for d in range(nd)]
    for p in itertools.product(*[range(m) for m in oshape]):
        bounds = [_range(p[d], x.shape[d], window[d], step[d], border) for d in range(nd)]
        if border == "fill" and any(b[2] for b in bounds):
            yield BORDER, 0, None
            continue
        cells = list(itertools.product(*[range(b[0], b[1] + 1) for b in bounds]))
        xv = [float(x[c]) for c in cells]
        yv = [float(y[c]) for c in cells]
        if any(_is_missing(a, is_float, missing_le) or _is_missing(b, is_float, missing_le)
               for a, b in zip(xv, yv)):
            yield MISSING, 0, None
            continue
        fl = 0
        if all(v == xv[0] for v in xv):
            fl |= ZVAR_X
        if all(v == yv[0] for v in yv):
            fl |= ZVAR_Y
        if fl:
            yield fl, 0, None
            continue
        fx = [Fraction(v) for v in xv]
        fy = [Fraction(v) for v in yv]
        n = len(fx)
        mx = sum(fx) / n
        my = sum(fy) / n
        sxy = sum((a - mx) * (b - my) for a, b in zip(fx, fy))
        sxx = sum((a - mx) ** 2 for a in fx)
        syy = sum((b - my) ** 2 for b in fy)
        sign = (sxy > 0) - (sxy < 0)
        yield 0, sign, (sxy * sxy) / (sxx * syy)


def rn32_from_exact(sign, c2):
    """Round-to-nearest-even float32 of sign*sqrt(c2), decided exactly."""
    if sign == 0:
        return np.float32(0.0)
    f = np.float32(math.sqrt(float(c2)))
    for _ in range(8):
        up = np.nextafter(f, np.float32(np.inf))
        dn = np.nextafter(f, np.float32(0.0))
        mh = (Fraction(float(f)) + Fraction(float(up))) / 2
        ml = (Fraction(float(dn)) + Fraction(float(f))) / 2
        if c2 > mh * mh:
            f = up
            continue
        if c2 < ml * ml:
            f = dn
            continue
        if c2 == mh * mh:
            f = f if (f.view(np.uint32) & 1) == 0 else up
        elif c2 == ml * ml:
            f = f if (f.view(np.uint32) & 1) == 0 else dn
        break
    return np.float32(sign * f)


def exact_corr(x, y, window, step, border, missing_le=-999.0, invalid=-2.0):
    """Returns (c32_exact, c64_exact_approx, flags) as flat numpy arrays.
    c32 is the exactly rounded float32 of the exact coefficient; c64 is the
    exact coefficient rounded through float (error < 1e-15)."""
    c32, c64, fl = [], [], []
    for flags, sign, c2 in exact_window_results(x, y, window, step, border, missing_le):
        fl.append(flags)
        if flags:
            c32.append(np.float32(invalid))
            c64.append(invalid)
        else:
            c32.append(rn32_from_exact(sign, c2))
            c64.append(sign * math.sqrt(float(c2)))
    return (np.array(c32, np.float32), np.array(c64, np.float64), np.array(fl, np.uint8))
