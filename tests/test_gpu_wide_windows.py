"""Wide windows on the register 2-D kernel and the batched kernel, against the
oracle (through the C ABI).

* Certification reach (float input).  A window 15 or 31 columns wide spans
  two to four lanes on each side of the lane that computes it.  Its FP64 sums
  carry the rounding residue of every value that ever passed through those
  columns' running sums, so the error bound that certifies a window as
  non-constant must use the largest such value over all of those lanes.
  The cases plant values of 1e6 early in a tile's march, in columns that a
  later constant-x patch's windows reach from two or more lanes away; the
  oracle flags those windows ZVAR_X (Section 3, all-equal windows), and so
  must the GPU.
* The prefix form (windows reaching more than two lanes): its sums are
  differences of prefixes over the whole wave, so the bound takes the
  wave's largest value; a case plants 1e6 far left of a constant patch.
* Every compiled wide variant (R = 4 and 8 columns per lane, k_w = 15 and 31,
  u8 / u16 / f32) on several tiles with ragged tails, borders, missing values
  and constant patches: bit-exact for integers, flags identical and
  |dc| <= 2^-24 for float.
* The float launch without a flag map runs its own code (no flags formed or
  stored); it is compared with the oracle directly: c within 2^-24 where the
  oracle gives a coefficient, exactly -2 where it flags the window.
"""
import numpy as np
import pytest

from gpu_util import F32_TOL, compare, say, to_dev
from workloads import random_pair, precision_pair

import oracle

pytestmark = pytest.mark.gpu


def _spike_then_constant(k, seed, W=420):
    """Float pair: x ~ N(0, 1) with values of 1e6 in rows 2..4 of the columns
    a constant-x patch (rows from 2k+8) starts and ends with; y ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    H = 5 * k + 40
    x = rng.standard_normal((H, W)).astype(np.float32)
    y = rng.standard_normal((H, W)).astype(np.float32)
    r0, r1 = 2 * k + 8, 4 * k + 30
    c0, c1 = 100, 100 + 3 * k + 20
    x[r0:r1, c0:c1] = 5.0
    x[2:5, c0:c0 + k // 2 + 4] = 1e6
    x[2:5, c1 - k // 2 - 4:c1] = 1e6
    return x, y, (r0, r1, c0, c1)


def _noflag_compare(x, y, window, step, border, params=None, indices=None, tag=""):
    """Launch without a flag map; c must match the oracle (-2 exactly where
    the oracle flags the window)."""
    import torch
    import paper_1807_06507_amd as swc
    say(f"[no-flag-map] {tag} shape={x.shape} window={window} step={step} border={border} "
        f"params={params}")
    c = swc.corr(to_dev(x), to_dev(y), window, step, border, params=params)
    torch.cuda.synchronize()
    c = c.cpu().numpy()
    if indices is None:
        _, o64, ofl = oracle.corr(x, y, window, step, border)
        cc = c
    else:
        _, o64, ofl = oracle.corr(x, y, window, step, border, indices=indices)
        cc = c.ravel()[indices]
    bad = ofl != 0
    assert np.all(cc[bad] == np.float32(-2.0)), f"{int(np.count_nonzero(cc[bad] != -2))} " \
        "flagged windows got a coefficient"
    assert np.all(cc[~bad] != np.float32(-2.0))
    d = float(np.max(np.abs(cc[~bad].astype(np.float64) - o64[~bad]))) if (~bad).any() else 0.0
    assert d <= F32_TOL, d
    return d


@pytest.mark.parametrize("k,R", [(15, 4), (31, 4), (15, 8), (31, 8)])
def test_certification_reaches_every_window_lane(k, R):
    x, y, (r0, r1, c0, c1) = _spike_then_constant(k, seed=k + R)
    # one tile covers the spikes and the whole patch, so the same running
    # column sums carry the residue into the constant windows
    params = (R, 256, 1)
    _, _, ofl = oracle.corr(x, y, (k, k), 1, "clip")
    nzx = int(np.count_nonzero(ofl & 4))
    assert nzx > 0, "the patch must produce constant-x windows"
    for border in ("clip", "fill"):
        compare(x, y, (k, k), 1, border, params=params, tag=f"cert-reach k={k} R={R}")
        _noflag_compare(x, y, (k, k), 1, border, params=params, tag=f"cert-reach k={k} R={R}")
    # default launch parameters (tile height from the resident-wave count)
    compare(x, y, (k, k), 1, "clip", tag=f"cert-reach k={k} default")


def test_certification_prefix_form_wave_wide():
    """Windows reaching more than two lanes (k = 31 at R = 4) take their sums
    as differences of prefixes over every column of the wave to their left.
    Values of 1e6 far to the left of a constant-x patch, in the same rows,
    then leave rounding in the patch's sums although no patch window holds
    them: the bound must take the wave's largest value, and the oracle's
    ZVAR_X flags must come back."""
    k = 31
    rng = np.random.default_rng(7)
    H, W = 160, 300
    x = rng.standard_normal((H, W)).astype(np.float32)
    y = rng.standard_normal((H, W)).astype(np.float32)
    r0, r1, c0, c1 = 40, 120, 150, 230
    x[r0:r1, c0:c1] = 5.0
    x[r0 - 20:r1 + 20, 40:52] = 1e6
    _, _, ofl = oracle.corr(x, y, (k, k), 1, "clip")
    assert int(np.count_nonzero(ofl & 4)) > 0, "the patch must produce constant-x windows"
    for border in ("clip", "fill"):
        compare(x, y, (k, k), 1, border, params=(4, 256, 1), tag="prefix-cert")
        _noflag_compare(x, y, (k, k), 1, border, params=(4, 256, 1), tag="prefix-cert")
    compare(x, y, (k, k), 1, "clip", tag="prefix-cert default")


def test_certification_reach_batched():
    """The batched kernel shares the tile code: k = 15 pairs with the spike
    and patch, mixed with narrower windows, one persistent plan."""
    import torch
    import paper_1807_06507_amd as swc
    cases = []
    for i, k in enumerate((15, 15, 9, 7)):
        x, y, _ = _spike_then_constant(k, seed=100 + i, W=300 + 37 * i)
        cases.append((x, y, k))
    pairs = [dict(x=to_dev(x), y=to_dev(y), window=(k, k), border="clip") for x, y, k in cases]
    for params in ((4, 256, 1), None):
        plan = swc.BatchPlan(pairs, return_flags=True, params=params)
        plan.launch()
        torch.cuda.synchronize()
        for (x, y, k), c, fl in zip(cases, plan.outputs, plan.flags):
            _, o64, ofl = oracle.corr(x, y, (k, k), 1, "clip")
            c, fl = c.cpu().numpy(), fl.cpu().numpy()
            mism = int(np.count_nonzero(fl != ofl))
            say(f"[batch cert-reach] k={k} params={params} flag mismatches={mism}")
            assert mism == 0
            ok = ofl == 0
            assert np.all(c[~ok] == np.float32(-2.0))
            assert float(np.max(np.abs(c[ok].astype(np.float64) - o64[ok]))) <= F32_TOL
        plan.close()


def _patched(shape, dtype, seed):
    x, y = random_pair(shape, dtype, seed=seed)
    if dtype == "f32":
        x[7, 40] = -999.0
        y[50, 500] = np.nan
        x[20:70, 100:160] = 3.0
        y[90:150, 300:380] = -1.5
    else:
        x[20:70, 100:160] = 9
        y[90:150, 300:380] = 0
    return x, y


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("R", [4, 8])
def test_parity_wide_compiled_variants(dtype, R):
    for k in (15, 31):
        # (column steps above 1: outputs no longer start on lane boundaries,
        # so halo lanes hold outputs whose windows end inside the wave)
        for shape, step, border, th in [((173, 1001), 1, "fill", 48),
                                        ((140, 1504), 1, "clip", 64),
                                        ((150, 777), (2, 1), "valid", 32),
                                        ((131, 1003), (1, 3), "fill", 40),
                                        ((120, 999), 2, "clip", 24)]:
            x, y = _patched(shape, dtype, seed=k + R + shape[1])
            compare(x, y, (k, k), step, border, params=(R, th, 2), tag=f"wide k={k} R={R}")
        # a rectangular window with the wide axis along the rows; several
        # waves per workgroup (the generic kernel's LDS row buffers, which
        # the launch parameters must also fit, allow 4 at R = 4 and 2 at R = 8)
        wpb = 4 if R == 4 else 2
        x, y = _patched((160, 900), dtype, seed=5 * k + R)
        compare(x, y, (5, k), 1, "clip", params=(R, 40, wpb), tag=f"wide 5x{k} R={R}")
        if dtype == "f32":
            _noflag_compare(x, y, (5, k), 1, "clip", params=(R, 40, wpb), tag=f"5x{k} R={R}")


@pytest.mark.parametrize("k", [3, 7, 15, 31])
def test_float_no_flag_map_full_size(k):
    """The float launch without a flag map at the precision pair's full size
    (4096x4096, x ~ N(1000, 1)), default launch parameters, CLIP, on sampled
    outputs."""
    x, y = precision_pair((4096, 4096), seed=3)
    x[1000:1100, 2000:2100] = 1000.5      # a constant patch
    n = 4096 * 4096
    rng = np.random.default_rng(k)
    idx = np.unique(np.concatenate([rng.integers(0, n, 4000), np.arange(400),
                                    (np.arange(1020, 1080)[:, None] * 4096 +
                                     np.arange(2020, 2080)[None, :]).ravel()[::7]]))
    d = _noflag_compare(x, y, (k, k), 1, "clip", indices=idx, tag=f"c2 k={k}")
    say(f"[no-flag-map] 4096x4096 k={k} max|dc|={d:.3e}")
