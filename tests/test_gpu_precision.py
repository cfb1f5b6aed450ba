"""Precision sweep on the large-offset float32 pair (x ~ N(1000, 1), per-block
rho): the sliding-sum formulation (Section 1, steps 1-4, and its one-pass
formula) evaluated four ways on the GPU and compared with the oracle's two-pass
FP64 value (the Introduction's classical formula).

  default   FP64 sliding sums with a certified fast path, two-pass rescan
            otherwise: |dc| <= 2^-24 is asserted at every (k, s);
  comp      compensated float32 sums (TwoSum / TwoProd pairs) with a certified
            fast path: a window passes only when its computed variances exceed
            rho = 4096 times their rounding-error bound, so |dc| <= 2/(rho-1)
            plus the float32 output rounding, asserted at every (k, s);
  comp-raw  the same sums without the certification (debug bit 3): the
            accuracy of the compensated sums themselves, reported;
  naive     plain float32 sums: reported only (cancellation leaves errors of
            order 1 on this input).

Each (k, s) case compares sampled outputs of the full 4096x4096 map one by
one against the oracle, so the whole sweep stays within a minute or two.
"""
import numpy as np
import pytest

from gpu_util import COMP_BOUND, F32_TOL, gpu_corr, say
from workloads import precision_pair

import oracle
import paper_1807_06507_amd as swc

pytestmark = pytest.mark.gpu

_X = {}


def _pair():
    if "p" not in _X:
        _X["p"] = precision_pair((4096, 4096), seed=3)
    return _X["p"]


def _sample(oshape, seed):
    n = int(np.prod(oshape))
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.integers(0, n, 6000), np.arange(min(n, 600))]))


def _maxdiff(c, fl, o64, ofl, idx):
    cs, fs = c.ravel()[idx], fl.ravel()[idx]
    ok = (fs == 0) & (ofl == 0)
    if not ok.any():
        return 0.0, 0
    d = np.abs(cs[ok].astype(np.float64) - o64[ok])
    return float(d.max()), int(np.count_nonzero(fs != ofl))


@pytest.mark.parametrize("k", [3, 7, 15, 31])
def test_precision_sweep(k):
    x, y = _pair()
    rows = []
    for s in (1, 2, 4):
        c, fl = gpu_corr(x, y, (k, k), s, "clip")
        idx = _sample(c.shape, 100 * k + s)
        _, o64, ofl = oracle.corr(x, y, (k, k), s, "clip", indices=idx)
        d_def, fmis = _maxdiff(c, fl, o64, ofl, idx)
        assert fmis == 0, f"k={k} s={s}: {fmis} flag mismatches"
        assert d_def <= F32_TOL, (k, s, d_def)
        cc, flc = gpu_corr(x, y, (k, k), s, "clip", accum="comp")
        d_comp, fmis_c = _maxdiff(cc, flc, o64, ofl, idx)
        assert fmis_c == 0, f"k={k} s={s}: comp {fmis_c} flag mismatches"
        assert d_comp <= COMP_BOUND, (k, s, d_comp)
        swc.set_debug(8)
        try:
            cr, flr = gpu_corr(x, y, (k, k), s, "clip", accum="comp")
        finally:
            swc.set_debug(0)
        d_raw, _ = _maxdiff(cr, flr, o64, ofl, idx)
        cn, fln = gpu_corr(x, y, (k, k), s, "clip", accum="naive")
        d_naive, _ = _maxdiff(cn, fln, o64, ofl, idx)
        rows.append((s, d_def, d_comp, d_raw, d_naive))
    for s, a, b, r, n in rows:
        say(f"[precision] k={k:2d} s={s} default={a:.3e} comp={b:.3e} comp-raw={r:.3e} "
            f"naive={n:.3e}")
