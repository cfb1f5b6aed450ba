"""End-to-end runs from host memory (slabs along the first axis, copies and
kernels pipelined over several streams) against the CPU oracle and against
the device path on the whole array.

Integer inputs: bit-exact c and flags, and identical to swc_corr on the whole
array.  Float inputs: identical flags and |dc| <= 2^-24 against the oracle.
Cases: 1-D, 2-D and 3-D; every border; slabs that are a single row, that do
not divide the output, and that cover the whole array; steps along the other
axes; pinned and pageable host memory.
"""
import numpy as np
import pytest

from gpu_util import F32_TOL, gpu_corr, say
from workloads import random_pair, paper_shaped_u16

import oracle

pytestmark = pytest.mark.gpu


def _host_run(x, y, window, step, border, band, depth, pinned=True):
    import torch
    import paper_1807_06507_amd as swc
    plan = swc.HostPlan(x.shape, x.dtype, window, step, border, band_rows=band, depth=depth)
    xt = torch.from_numpy(np.ascontiguousarray(x))
    yt = torch.from_numpy(np.ascontiguousarray(y))
    if pinned:
        xt, yt = xt.pin_memory(), yt.pin_memory()
    fl = torch.empty(plan.oshape, dtype=torch.uint8, pin_memory=pinned)
    c, fl = plan.run(xt, yt, flags=fl)
    nb = plan.bands
    plan.close()
    return c.numpy(), fl.numpy(), nb


def _check(x, y, window, step, border, band, depth, pinned=True):
    say(f"[host] shape={x.shape} dtype={x.dtype} window={window} step={step} border={border} "
        f"band={band} depth={depth} pinned={pinned}")
    c, fl, nb = _host_run(x, y, window, step, border, band, depth, pinned)
    o32, o64, ofl = oracle.corr(x, y, window, step, border)
    assert c.shape == o32.shape
    assert np.array_equal(fl, ofl)
    ok = ofl == 0
    assert np.all(c[~ok] == np.float32(-2.0))
    if x.dtype.kind == "u":
        assert np.array_equal(c[ok].view(np.uint32), o32[ok].view(np.uint32))
        a, fa = gpu_corr(x, y, window, step, border)
        assert np.array_equal(a.view(np.uint32), c.view(np.uint32))
        assert np.array_equal(fa, fl)
    else:
        d = np.abs(c[ok].astype(np.float64) - o64[ok])
        assert (float(d.max()) if d.size else 0.0) <= F32_TOL
    return nb


@pytest.mark.parametrize("dtype", ["u8", "u16", "f32"])
@pytest.mark.parametrize("border", ["fill", "clip", "valid"])
def test_host_pipeline_2d(dtype, border):
    x, y = random_pair((203, 317), dtype, seed=21)
    assert _check(x, y, (7, 5), 1, border, band=50, depth=3) >= 4
    _check(x, y, (7, 5), (1, 2), border, band=1, depth=2)        # one output row per slab
    _check(x, y, (3, 9), 1, border, band=1000, depth=1)          # one slab
    _check(x, y, (6, 4), 1, border, band=37, depth=4, pinned=False)


@pytest.mark.parametrize("dtype", ["u16", "f32"])
def test_host_pipeline_1d_and_3d(dtype):
    x, y = random_pair((20000,), dtype, seed=22)
    _check(x, y, (101,), 1, "clip", band=3000, depth=3)
    _check(x, y, (64,), 1, "valid", band=777, depth=2)
    x3, y3 = random_pair((40, 33, 70), dtype, seed=23)
    _check(x3, y3, (5, 3, 7), 1, "fill", band=7, depth=3)
    _check(x3, y3, (3, 5, 5), (1, 2, 1), "clip", band=9, depth=2)


def test_host_pipeline_full_size_paper_shaped():
    """4000x3000 u16, 7x7, FILL through host memory: identical to the device
    path on the whole array (every output)."""
    x, y = paper_shaped_u16((3000, 4000), seed=2)
    c, fl, nb = _host_run(x, y, (7, 7), 1, "fill", band=500, depth=3)
    a, fa = gpu_corr(x, y, (7, 7), 1, "fill")
    assert nb == 6
    assert np.array_equal(a.view(np.uint32), c.view(np.uint32))
    assert np.array_equal(fa, fl)


def test_host_plan_rejects_bad_arguments():
    import paper_1807_06507_amd as swc
    with pytest.raises(Exception):
        swc.HostPlan((100, 100), "uint8", (3, 3), (2, 1), "fill")    # step along axis 0
    with pytest.raises(Exception):
        swc.HostPlan((100, 100), "uint8", (3, 3), 1, "fill", band_rows=0)
    with pytest.raises(Exception):
        swc.HostPlan((100, 100), "uint8", (3, 3), 1, "fill", depth=9)
