"""Missing-value thresholds at or above zero (a caller's convention, e.g.
"0 means no data"): positions outside the array are not data, so they must
never count as missing, whatever the threshold.  Each kernel family (1-D,
2-D register and generic, 3-D specialised and general, batched, unfused
scheme) against the oracle with thresholds 0 and 0.05 on positive data that
also holds some values at or below the threshold."""
import numpy as np
import pytest

from gpu_util import compare
from workloads import random_pair

pytestmark = pytest.mark.gpu


def _positive(shape, seed, thr):
    x, y = random_pair(shape, "f32", seed=seed, kind="lognormal")
    rng = np.random.default_rng(seed + 100)
    idx = rng.integers(0, x.size, size=max(1, x.size // 2000))
    x.reshape(-1)[idx] = thr                     # exactly at the threshold: missing
    return x, y


@pytest.mark.parametrize("thr", [0.0, 0.05])
@pytest.mark.parametrize("border", ["clip", "fill", "valid"])
def test_threshold_2d(thr, border):
    import paper_1807_06507_amd as swc
    x, y = _positive((70, 300), 31, thr)
    compare(x, y, (7, 7), 1, border, missing_le=thr, tag="thr-2d")
    compare(x, y, (5, 9), (1, 2), border, missing_le=thr, tag="thr-2d-step")
    compare(x[:, :297], y[:, :297], (7, 7), 1, border, missing_le=thr, tag="thr-2d-ragged")
    swc.set_debug(2)                               # generic LDS kernel
    try:
        compare(x, y, (7, 7), 1, border, missing_le=thr, tag="thr-2d-generic")
    finally:
        swc.set_debug(0)


@pytest.mark.parametrize("thr", [0.0, 0.05])
@pytest.mark.parametrize("border", ["clip", "fill"])
def test_threshold_1d_3d(thr, border):
    x, y = _positive((20000,), 32, thr)
    compare(x, y, (101,), 1, border, missing_le=thr, tag="thr-1d")
    x3, y3 = _positive((12, 20, 64), 33, thr)
    compare(x3, y3, (5, 5, 5), 1, border, missing_le=thr, tag="thr-3d-square")
    x4, y4 = _positive((12, 20, 70), 34, thr)
    compare(x4, y4, (3, 5, 7), 1, border, missing_le=thr, tag="thr-3d-general")
    compare(x3, y3, (5, 5, 5), 1, border, missing_le=thr, tag="thr-3d-whole",
            params=(4, 8, 1, 0, 2))


def test_threshold_scheme_and_batch():
    import torch
    import paper_1807_06507_amd as swc
    import oracle
    from gpu_util import to_dev
    x, y = _positive((90, 130), 35, 0.0)
    compare(x, y, (7, 7), 1, "clip", missing_le=0.0, tag="thr-unfused", scheme="unfused")
    pairs = [_positive((60 + 7 * i, 100 + 9 * i), 40 + i, 0.0) for i in range(4)]
    plan = swc.BatchPlan([dict(x=to_dev(a), y=to_dev(b), window=(7, 7), step=1, border="clip")
                          for a, b in pairs], missing_le=0.0)
    plan.launch()
    torch.cuda.synchronize()
    for (a, b), out in zip(pairs, plan.outputs):
        o32, o64, ofl = oracle.corr(a, b, (7, 7), 1, "clip", missing_le=0.0)
        c = out.cpu().numpy()
        ok = ofl == 0
        assert np.all(c[~ok] == np.float32(-2.0))
        assert np.abs(c[ok].astype(np.float64) - o64[ok]).max() <= 2.0 ** -24
    plan.close()
