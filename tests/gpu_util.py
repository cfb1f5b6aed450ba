"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
(via the thin binding) and compare with the CPU oracle on the same seeded
inputs."""
import os
import sys

import numpy as np

import oracle

# f32 tolerance: |c_gpu - c64_oracle| <= 2^-24 (float32 output rounding is at
# most 2^-25 for |c| <= 1; the FP64 sliding sums add far less on these inputs)
F32_TOL = 2.0 ** -24
# comparator modes.  Naive float32 sums: a sanity bound only.  Compensated
# float32 sums with the certification test: every certified window has both
# computed variances above rho = 4096 times their rounding-error bound, so its
# relative errors in N, Vx, Vy stay below 1/rho and |dc| <= 2/(rho - 1); the
# output rounding adds 2^-24 (uncertified windows are recomputed two-pass).
NAIVE_TOL = 0.5
COMP_BOUND = 2.0 / 4095.0 + 2.0 ** -24
# on the well-conditioned inputs of the parity tests the compensated sums
# stay far inside that bound
COMP_TOL = 1e-4


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.cuda()


def gpu_corr(x, y, window, step=1, border="fill", accum="default", params=None,
             missing_le=-999.0, invalid=-2.0, scheme=None):
    import torch
    import paper_1807_06507_amd as swc
    xd, yd = to_dev(x), to_dev(y)
    if scheme is not None:
        assert step in (1, (1, 1)) and accum == "default" and params is None
        c, fl = swc.corr_scheme(xd, yd, window, scheme, border, invalid=invalid,
                                missing_le=missing_le, return_flags=True)
    else:
        c, fl = swc.corr(xd, yd, window, step, border, invalid=invalid, missing_le=missing_le,
                         return_flags=True, accum=accum, params=params)
    torch.cuda.synchronize()
    return c.cpu().numpy(), fl.cpu().numpy()


def compare(x, y, window, step=1, border="fill", accum="default", params=None, tag="",
            indices=None, tol=None, scheme=None, missing_le=-999.0):
    """Run both sides, assert parity, return max |dc| over valid outputs.
    ``scheme`` selects one of the unfused baseline schemes instead of the
    fused kernels."""
    say(f"[parity] {tag} shape={x.shape} dtype={x.dtype} window={window} step={step} "
        f"border={border} accum={accum} params={params} scheme={scheme}")
    c, fl = gpu_corr(x, y, window, step, border, accum, params, scheme=scheme,
                     missing_le=missing_le)
    if indices is None:
        o32, o64, ofl = oracle.corr(x, y, window, step, border, missing_le=missing_le)
        c_cmp, fl_cmp = c, fl
    else:
        o32, o64, ofl = oracle.corr(x, y, window, step, border, missing_le=missing_le,
                                    indices=indices)
        c_cmp, fl_cmp = c.ravel()[indices], fl.ravel()[indices]
    assert c_cmp.shape == o32.shape, (c_cmp.shape, o32.shape)
    if accum != "default":
        ok = (ofl == 0) & (fl_cmp == 0)
        d = np.abs(c_cmp[ok].astype(np.float64) - o64[ok])
        dmax = float(d.max()) if d.size else 0.0
        lim = NAIVE_TOL if accum.startswith("naive") else COMP_TOL
        assert dmax <= lim, dmax
        return dmax
    mism = np.flatnonzero(fl_cmp.ravel() != ofl.ravel())
    assert mism.size == 0, f"{mism.size} flag mismatches, first {mism[:5]}: " \
        f"gpu {fl_cmp.ravel()[mism[:5]]} oracle {ofl.ravel()[mism[:5]]}"
    bad = ofl != 0
    assert np.all(c_cmp[bad] == np.float32(-2.0))
    ok = ~bad
    if x.dtype.kind == "u":
        diff = np.flatnonzero(c_cmp[ok].view(np.uint32) != o32[ok].view(np.uint32))
        assert diff.size == 0, f"{diff.size} bit mismatches, e.g. gpu {c_cmp[ok][diff[:5]]} " \
            f"oracle {o32[ok][diff[:5]]}"
        return 0.0
    d = np.abs(c_cmp[ok].astype(np.float64) - o64[ok])
    dmax = float(d.max()) if d.size else 0.0
    assert dmax <= (tol if tol is not None else F32_TOL), dmax
    return dmax
