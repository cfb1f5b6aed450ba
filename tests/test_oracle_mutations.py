"""Planted-mistake check for the oracle's pins (CPU only).

Each mutation below is a plausible slip in ``oracle/oracle.c`` (a dropped or
swapped term, an off-by-one in the window or border, a wrong tie rule).  The
test builds the mutated source into a throw-away library and runs a compact
battery of the same pins used in test_oracle_pins.py against it; every
mutation must be caught by at least one pin.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import exactref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = {
    "even_k_anchor": ("int64_t l = k / 2;", "int64_t l = (k - 1) / 2;"),
    "sxy_transposed_operand": ("sxy += dx * dy;", "sxy += dx * dx;"),
    "mean_y_from_x": ("my = sy / (double)n;", "my = sx / (double)n;"),
    "border_off_by_one": ("hi[d] > J->shape[d] - 1) {", "hi[d] > J->shape[d]) {"),
    "tie_rounds_up": ("if (s == 0) { f = f32_is_even(f) ? f : up; break; }",
                      "if (s == 0) { f = up; break; }"),
    "missing_strict": ("xs[i] <= J->missing_le", "xs[i] < J->missing_le"),
    "int_dev_y_uses_sx": ("load_as_int(J->y, J->dtype, ix[i]) - Sy;",
                          "load_as_int(J->y, J->dtype, ix[i]) - Sx;"),
    "output_len_floor": ("out[d] = (N + s - 1) / s;", "out[d] = N / s;"),
    "denominator_sxx_twice": ("double c = sxy / sqrt(sxx * syy);",
                              "double c = sxy / sqrt(sxx * sxx);"),
    "valid_start_centred": ("lo[d] = p[d] * s;\n            hi[d] = lo[d] + k - 1;",
                            "lo[d] = p[d] * s - k / 2;\n            hi[d] = lo[d] + k - 1;"),
    "zvar_y_checks_x": ("if (ys[i] != ys[0]) eqy = 0;", "if (xs[i] != xs[0]) eqy = 0;"),
    "nan_not_missing": ("if (!isfinite(xs[i]) || !isfinite(ys[i]) ||", "if ("),
}


def _battery(lib):
    """Return True when every pin in the compact battery passes."""
    rng = np.random.default_rng(42)
    try:
        cases = []
        for dtype in ("u16", "f32"):
            for border in ("fill", "clip", "valid"):
                shape = (6, 7)
                if dtype == "f32":
                    x = rng.normal(size=shape).astype(np.float32)
                    y = (0.4 * x + rng.normal(size=shape)).astype(np.float32)
                    x[2, 3] = -999.0
                    y[4, 1] = np.nan
                    y[0:3, 4:7] = 1.0
                else:
                    x = rng.integers(0, 5, size=shape).astype(np.uint16)
                    y = rng.integers(0, 65536, size=shape).astype(np.uint16)
                for window, step in (((3, 4), (1, 1)), ((2, 3), (2, 1))):
                    cases.append((x, y, window, step, border))
        for x, y, window, step, border in cases:
            c32, c64, fl = oracle.corr(x, y, window, step, border, lib=lib)
            e32, e64, efl = exactref.exact_corr(x, y, window, step, border)
            if c32.size != e32.size or not np.array_equal(fl.ravel(), efl):
                return False
            ok = efl == 0
            if not np.all(np.abs(c64.ravel()[ok] - e64[ok]) <= 1e-12):
                return False
            if x.dtype.kind == "u" and not np.array_equal(c32.ravel().view(np.uint32),
                                                          e32.view(np.uint32)):
                return False
        # exact rounding ties (Q = R = 2^60, P on a midpoint)
        for f in np.float32([0.3, 0.7, 0.123, 0.9]):
            up = np.nextafter(f, np.float32(2))
            P = int((float(f) + float(up)) / 2 * 2 ** 60)
            got = oracle.rn32_ratio(P, 2 ** 60, 2 ** 60, lib=lib)
            even = f if (f.view(np.uint32) & 1) == 0 else up
            if got != even:
                return False
        if oracle.output_shape((7,), (3,), 2, "fill", lib=lib) != (4,):
            return False
    except (ValueError, RuntimeError):
        return False
    return True


def test_unmutated_oracle_passes_battery():
    assert _battery(oracle._load())


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    if shutil.which("gcc") is None:
        pytest.skip("gcc missing")
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique/present"
    tmp = tempfile.mkdtemp(prefix="oracle_mut_")
    try:
        msrc = os.path.join(tmp, "oracle_mut.c")
        with open(msrc, "w") as f:
            f.write(src.replace(old, new))
        out = os.path.join(tmp, "liboracle_mut.so")
        subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-o", out, msrc, "-lm"],
                       check=True)
        lib = oracle._load(out)
        assert not _battery(lib), f"pins did not catch mutation {name}"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
