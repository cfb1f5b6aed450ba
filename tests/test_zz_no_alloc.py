"""The scheme entry point without a caller workspace (swc_corr_scheme_noalloc,
for callers that cannot allocate device memory) against swc_corr_scheme with
a caller workspace, both called through the C ABI with ctypes.

Both run the same kernels on the same inputs, so the outputs must be
identical bit for bit (coefficients and flags).  Each case makes two calls in
a row on the fixed device workspace, the second on a smaller input, so the
second call starts from what the first left behind.  The float case puts its
largest magnitudes in the first input only: the unfused scheme's header of
global maxima must be cleared between calls for the second to match.
"""
import ctypes

import numpy as np
import pytest

from gpu_util import say, to_dev
from workloads import random_pair

pytestmark = pytest.mark.gpu


def _run(lib, swc, entry, p, scheme, xd, yd):
    import torch
    oshape = swc.output_shape(p)
    c = torch.full(oshape, 7.0, dtype=torch.float32, device=xd.device)
    fl = torch.full(oshape, 0xEE, dtype=torch.uint8, device=xd.device)
    stream = torch.cuda.current_stream(xd.device)
    h = ctypes.c_void_p(int(stream.cuda_stream))
    args = [ctypes.byref(p), swc.SCHEMES[scheme], ctypes.c_void_p(xd.data_ptr()),
            ctypes.c_void_p(yd.data_ptr()), ctypes.c_void_p(c.data_ptr()),
            ctypes.c_void_p(fl.data_ptr())]
    if entry == "noalloc":
        code = lib.swc_corr_scheme_noalloc(*args, h)
    else:
        ws = torch.empty(swc.scheme_workspace_bytes(p, scheme), dtype=torch.uint8,
                         device=xd.device)
        code = lib.swc_corr_scheme(*args, ctypes.c_void_p(ws.data_ptr()),
                                   ctypes.c_uint64(ws.numel()), h)
    assert code == 0, swc.status_str(code)
    torch.cuda.synchronize()
    return c.cpu().numpy(), fl.cpu().numpy()


CASES = [
    # scheme, dtype, window, border, first shape, second (smaller) shape
    ("unfused", "f32", (7, 7), "clip", (600, 1100), (233, 411)),
    ("unfused", "u16", (5, 9), "fill", (512, 1000), (97, 301)),
    ("cumsum", "u16", (7, 7), "fill", (1000, 1500), (300, 517)),
    ("cumsum", "u8", (3, 15), "clip", (800, 900), (64, 200)),
]


@pytest.mark.parametrize("scheme,dtype,window,border,shape1,shape2", CASES)
def test_noalloc_matches_workspace_entry(scheme, dtype, window, border, shape1, shape2):
    import paper_1807_06507_amd as swc
    lib = swc._load()
    for i, shape in enumerate((shape1, shape2)):
        x, y = random_pair(shape, dtype, seed=11 + i)
        if dtype == "f32":
            if i == 0:
                x[3:9, 5:40] = 3e4      # the largest values of the two calls
            x[40:60, 100:140] = 2.5     # constant patch
            y[20, 30] = -999.0          # missing value
        else:
            x[40:60, 100:140] = 9
        p = swc.make_problem(shape, x.dtype, window, 1, border)
        say(f"[noalloc] call {i + 1}: {scheme} {dtype} shape={shape} window={window} "
            f"border={border}")
        xd, yd = to_dev(x), to_dev(y)
        c_ref, f_ref = _run(lib, swc, "workspace", p, scheme, xd, yd)
        c_na, f_na = _run(lib, swc, "noalloc", p, scheme, xd, yd)
        assert np.array_equal(f_na, f_ref), f"{int(np.count_nonzero(f_na != f_ref))} flags differ"
        assert np.array_equal(c_na.view(np.uint32), c_ref.view(np.uint32)), \
            f"{int(np.count_nonzero(c_na.view(np.uint32) != c_ref.view(np.uint32)))} values differ"


def test_noalloc_rejects_problems_beyond_its_workspace():
    """A problem needing more than the fixed workspace returns
    SWC_ERR_WORKSPACE before anything is launched (outputs untouched)."""
    import torch
    import paper_1807_06507_amd as swc
    lib = swc._load()
    shape = (700, 1000)     # 96 B per element for the unfused scheme: 67.2 MB > 64 MiB
    p = swc.make_problem(shape, torch.float32, (7, 7), 1, "clip")
    assert swc.scheme_workspace_bytes(p, "unfused") > swc.SCHEME_SCRATCH_BYTES
    xd = torch.zeros(shape, dtype=torch.float32, device="cuda")
    c = torch.full(shape, 5.0, dtype=torch.float32, device="cuda")
    h = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    code = lib.swc_corr_scheme_noalloc(ctypes.byref(p), swc.SCHEMES["unfused"],
                                       ctypes.c_void_p(xd.data_ptr()),
                                       ctypes.c_void_p(xd.data_ptr()),
                                       ctypes.c_void_p(c.data_ptr()), None, h)
    assert swc.STATUS.get(code) == "SWC_ERR_WORKSPACE"
    torch.cuda.synchronize()
    assert bool(torch.all(c == 5.0))
