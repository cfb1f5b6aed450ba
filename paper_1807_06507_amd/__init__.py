"""Sliding-window inter-channel Pearson correlation on MI355X (gfx950).

Thin ctypes binding of ``libswcorr.so`` (C ABI in ``include/swcorr.h``):
argument marshalling only.  Every step of the computation runs in the HIP
kernels of the library; torch supplies device memory and streams.  There is
no CPU fallback: if the library is missing the import of the binding fails.

    import torch, paper_1807_06507_amd as swc
    c = swc.corr(x, y, window=7)                     # FILL, step 1 (paper)
    c, flags = swc.corr(x, y, (7, 7), border="clip", return_flags=True)
"""
from __future__ import annotations

import ctypes
import os
import threading

__all__ = [
    "Problem", "LaunchParams", "corr", "corr_into", "prepare", "output_shape", "validate",
    "status_str", "tune_set", "tune_get", "set_debug", "get_debug", "BatchPlan", "library_path",
    "SwcError", "FLAG_BORDER", "FLAG_MISSING", "FLAG_ZVAR_X", "FLAG_ZVAR_Y",
    "HostPlan", "corr_scheme", "scheme_workspace_bytes", "SCHEMES", "cloud_mask",
    "filter_detections",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
# SWC_LIBRARY selects another build of the same library (e.g. a variant
# compiled with different tuning macros); the default is the in-tree build.
_LIB_PATH = os.environ.get("SWC_LIBRARY") or os.path.join(_HERE, "libswcorr.so")

U8, U16, F32 = 0, 1, 2
BORDERS = {"fill": 0, "clip": 1, "valid": 2}
ACCUMS = {"default": 0, "naive": 1, "naive_f32": 1, "comp": 2, "comp_f32": 2}
FLAG_BORDER, FLAG_MISSING, FLAG_ZVAR_X, FLAG_ZVAR_Y = 1, 2, 4, 8

STATUS = {
    0: "SWC_OK", 1: "SWC_ERR_NULL", 2: "SWC_ERR_NDIM", 3: "SWC_ERR_SHAPE", 4: "SWC_ERR_WINDOW",
    5: "SWC_ERR_STEP", 6: "SWC_ERR_DTYPE", 7: "SWC_ERR_BORDER", 8: "SWC_ERR_ACCUM",
    9: "SWC_ERR_WORKSPACE", 10: "SWC_ERR_LAUNCH", 11: "SWC_ERR_DEVICE",
    12: "SWC_ERR_UNSUPPORTED", 13: "SWC_ERR_PARAM",
}


class SwcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("dtype", ctypes.c_int32), ("border", ctypes.c_int32),
        ("accum", ctypes.c_int32), ("shape", ctypes.c_int64 * 3), ("window", ctypes.c_int32 * 3),
        ("step", ctypes.c_int32 * 3), ("invalid_value", ctypes.c_float),
        ("reserved0", ctypes.c_int32), ("missing_le", ctypes.c_double),
    ]


class LaunchParams(ctypes.Structure):
    _fields_ = [
        ("cols_per_lane", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
        ("waves_per_block", ctypes.c_int32), ("min_waves_per_eu", ctypes.c_int32),
        ("tile_rows2", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3),
    ]

    def as_tuple(self):
        return (self.cols_per_lane, self.tile_rows, self.waves_per_block, self.min_waves_per_eu,
                self.tile_rows2)


assert ctypes.sizeof(Problem) == 80
assert ctypes.sizeof(LaunchParams) == 32

_lock = threading.Lock()
_lib = None


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            raise ImportError(
                f"{_LIB_PATH} is missing: build it with `python -m paper_1807_06507_amd.build` "
                "(there is no CPU fallback)")
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(Problem)
        LP = ctypes.POINTER(LaunchParams)
        vp = ctypes.c_void_p
        lib.swc_validate.argtypes = [P]
        lib.swc_output_shape.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
        lib.swc_status_str.argtypes = [ctypes.c_int]
        lib.swc_status_str.restype = ctypes.c_char_p
        lib.swc_version.restype = ctypes.c_int32
        lib.swc_corr.argtypes = [P, vp, vp, vp, vp, vp]
        lib.swc_corr_ex.argtypes = [P, LP, vp, vp, vp, vp, vp]
        lib.swc_tune_set.argtypes = [P, LP]
        lib.swc_tune_get.argtypes = [P, LP]
        lib.swc_set_debug.argtypes = [ctypes.c_int32]
        lib.swc_get_debug.restype = ctypes.c_int32
        lib.swc_batch_plan_create.argtypes = [ctypes.c_int32, P, ctypes.POINTER(vp),
                                              ctypes.POINTER(vp), ctypes.POINTER(vp),
                                              ctypes.POINTER(vp), LP, ctypes.POINTER(vp)]
        lib.swc_batch_launch.argtypes = [vp, vp]
        lib.swc_batch_plan_items.argtypes = [vp]
        lib.swc_batch_plan_items.restype = ctypes.c_int64
        lib.swc_batch_plan_destroy.argtypes = [vp]
        lib.swc_batch_plan_destroy.restype = None
        lib.swc_scheme_workspace.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]
        lib.swc_corr_scheme.argtypes = [P, ctypes.c_int32, vp, vp, vp, vp, vp, ctypes.c_uint64, vp]
        lib.swc_corr_scheme_noalloc.argtypes = [P, ctypes.c_int32, vp, vp, vp, vp, vp]
        lib.swc_host_plan_create.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(vp)]
        lib.swc_host_run.argtypes = [vp, vp, vp, vp, vp]
        lib.swc_host_plan_bands.argtypes = [vp]
        lib.swc_host_plan_bands.restype = ctypes.c_int64
        lib.swc_host_plan_destroy.argtypes = [vp]
        lib.swc_host_plan_destroy.restype = None
        lib.swc_cloud_mask.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_float, ctypes.c_float,
                                       vp, vp]
        lib.swc_filter_detections.argtypes = [vp, vp, ctypes.c_int64, vp, ctypes.c_int64,
                                              ctypes.c_float, ctypes.c_float, vp, vp]
        for fn in ("swc_host_plan_create", "swc_host_run", "swc_cloud_mask",
                   "swc_filter_detections"):
            getattr(lib, fn).restype = ctypes.c_int
        for fn in ("swc_validate", "swc_output_shape", "swc_corr", "swc_corr_ex", "swc_tune_set",
                   "swc_tune_get", "swc_batch_plan_create", "swc_batch_launch",
                   "swc_scheme_workspace", "swc_corr_scheme"):
            getattr(lib, fn).restype = ctypes.c_int
        _lib = lib
        return lib


def status_str(code: int) -> str:
    return _load().swc_status_str(int(code)).decode()


def _check(code):
    if code != 0:
        raise SwcError(code, status_str(code))


def _per_dim(v, ndim, name):
    if isinstance(v, int):
        return [int(v)] * ndim
    v = [int(t) for t in v]
    if len(v) != ndim:
        raise ValueError(f"{name} needs {ndim} entries, got {len(v)}")
    return v


_DT = {"uint8": U8, "u8": U8, "uint16": U16, "u16": U16, "float32": F32, "f32": F32}


def _dtype_code(dt) -> int:
    name = str(dt).replace("torch.", "").replace("numpy.", "")
    if name not in _DT:
        raise ValueError(f"unsupported dtype {dt} (uint8, uint16 or float32)")
    return _DT[name]


def make_problem(shape, dtype, window, step=1, border="fill", accum="default",
                 invalid=-2.0, missing_le=-999.0) -> Problem:
    ndim = len(shape)
    if ndim not in (1, 2, 3):
        raise ValueError("ndim must be 1, 2 or 3")
    p = Problem()
    p.ndim = ndim
    p.dtype = _dtype_code(dtype) if not isinstance(dtype, int) else dtype
    if border not in BORDERS:
        raise ValueError(f"border must be one of {sorted(BORDERS)}")
    p.border = BORDERS[border]
    if accum not in ACCUMS:
        raise ValueError(f"accum must be one of {sorted(ACCUMS)}")
    p.accum = ACCUMS[accum]
    w = _per_dim(window, ndim, "window")
    s = _per_dim(step, ndim, "step")
    for d in range(3):
        p.shape[d] = int(shape[d]) if d < ndim else 1
        p.window[d] = w[d] if d < ndim else 1
        p.step[d] = s[d] if d < ndim else 1
    p.invalid_value = float(invalid)
    p.reserved0 = 0
    p.missing_le = float(missing_le)
    return p


def validate(p: Problem) -> int:
    return int(_load().swc_validate(ctypes.byref(p)))


def output_shape(p: Problem):
    out = (ctypes.c_int64 * 3)()
    _check(_load().swc_output_shape(ctypes.byref(p), out))
    return tuple(int(out[d]) for d in range(p.ndim))


def _params(params):
    if params is None:
        return None
    if isinstance(params, LaunchParams):
        return params
    lp = LaunchParams()
    lp.cols_per_lane, lp.tile_rows, lp.waves_per_block = (int(v) for v in params[:3])
    lp.min_waves_per_eu = int(params[3]) if len(params) > 3 else 0
    lp.tile_rows2 = int(params[4]) if len(params) > 4 else 0
    return lp


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(int(stream.cuda_stream))


def _check_tensor(t, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def corr_into(p: Problem, x, y, out, flags=None, params=None, stream=None):
    """Launch on preallocated device tensors (no allocation, asynchronous)."""
    _check_tensor(x, "x")
    _check_tensor(y, "y")
    _check_tensor(out, "out")
    if flags is not None:
        _check_tensor(flags, "flags")
    h = _stream_handle(stream, x.device)
    lp = _params(params)
    lib = _load()
    fptr = ctypes.c_void_p(flags.data_ptr()) if flags is not None else None
    code = lib.swc_corr_ex(ctypes.byref(p), ctypes.byref(lp) if lp is not None else None,
                           ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                           ctypes.c_void_p(out.data_ptr()), fptr, h)
    _check(code)
    return out


def prepare(p: Problem, x, y, out, flags=None, params=None, stream=None):
    """Check and marshal the arguments of ``corr_into`` once; returns a
    callable that launches the same call again (asynchronously, on the same
    stream) with no per-call Python work beyond the C call itself.  The
    callable keeps the tensors alive."""
    _check_tensor(x, "x")
    _check_tensor(y, "y")
    _check_tensor(out, "out")
    if flags is not None:
        _check_tensor(flags, "flags")
    lib = _load()
    lp = _params(params)
    args = (ctypes.byref(p), ctypes.byref(lp) if lp is not None else None,
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
            ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(flags.data_ptr()) if flags is not None else None,
            _stream_handle(stream, x.device))
    fn = lib.swc_corr_ex
    keep = (p, lp, x, y, out, flags)

    def launch():
        code = fn(*args)
        if code != 0:
            _check(code)
        return keep[4]
    return launch


def corr(x, y, window, step=1, border="fill", invalid=-2.0, missing_le=-999.0,
         return_flags=False, accum="default", out=None, flags_out=None, params=None,
         stream=None):
    """Sliding-window correlation map of two equal-shape device tensors
    (uint8, uint16 or float32; 1-D, 2-D or 3-D).  Returns a float32 tensor
    (and a uint8 flag tensor when ``return_flags``)."""
    import torch
    _check_tensor(x, "x")
    _check_tensor(y, "y")
    if x.shape != y.shape or x.dtype != y.dtype:
        raise ValueError("x and y must have the same shape and dtype")
    if x.device != y.device:
        raise ValueError("x and y must be on the same device")
    p = make_problem(tuple(x.shape), x.dtype, window, step, border, accum, invalid, missing_le)
    code = validate(p)
    if code != 0:
        raise ValueError(f"{STATUS.get(code)}: {status_str(code)}")
    oshape = output_shape(p)
    if out is None:
        out = torch.empty(oshape, dtype=torch.float32, device=x.device)
    elif tuple(out.shape) != oshape or out.dtype != torch.float32:
        raise ValueError(f"out must be float32 of shape {oshape}")
    fl = None
    if return_flags or flags_out is not None:
        fl = flags_out if flags_out is not None else torch.empty(oshape, dtype=torch.uint8,
                                                                 device=x.device)
        if tuple(fl.shape) != oshape or fl.dtype != torch.uint8:
            raise ValueError(f"flags must be uint8 of shape {oshape}")
    corr_into(p, x, y, out, fl, params, stream)
    return (out, fl) if return_flags else out


SCHEMES = {"unfused": 1, "cumsum": 2}


def scheme_workspace_bytes(p: Problem, scheme: str) -> int:
    """Workspace bytes an unfused baseline scheme needs for problem ``p``."""
    n = ctypes.c_uint64(0)
    _check(_load().swc_scheme_workspace(ctypes.byref(p), SCHEMES[scheme], ctypes.byref(n)))
    return int(n.value)


def corr_scheme(x, y, window, scheme="unfused", border="fill", invalid=-2.0, missing_le=-999.0,
                return_flags=False, workspace=None, stream=None):
    """The same 2-D map by one of the unfused baseline schemes: "unfused"
    (the paper's four-phase parallel scheme with intermediates in device
    memory) or "cumsum" (integral images; uint8/uint16).  Step 1 only.
    ``workspace`` (a uint8 device tensor) is allocated when not given."""
    import torch
    _check_tensor(x, "x")
    _check_tensor(y, "y")
    if x.shape != y.shape or x.dtype != y.dtype:
        raise ValueError("x and y must have the same shape and dtype")
    if scheme not in SCHEMES:
        raise ValueError(f"scheme must be one of {sorted(SCHEMES)}")
    p = make_problem(tuple(x.shape), x.dtype, window, 1, border, "default", invalid, missing_le)
    code = validate(p)
    if code != 0:
        raise ValueError(f"{STATUS.get(code)}: {status_str(code)}")
    nbytes = scheme_workspace_bytes(p, scheme)
    if workspace is None:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    _check_tensor(workspace, "workspace")
    oshape = output_shape(p)
    out = torch.empty(oshape, dtype=torch.float32, device=x.device)
    fl = torch.empty(oshape, dtype=torch.uint8, device=x.device) if return_flags else None
    h = _stream_handle(stream, x.device)
    code = _load().swc_corr_scheme(
        ctypes.byref(p), SCHEMES[scheme], ctypes.c_void_p(x.data_ptr()),
        ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(out.data_ptr()),
        ctypes.c_void_p(fl.data_ptr()) if fl is not None else None,
        ctypes.c_void_p(workspace.data_ptr()), ctypes.c_uint64(workspace.numel()), h)
    _check(code)
    return (out, fl) if return_flags else out


# bytes of the fixed device workspace of corr_scheme_noalloc (64 MiB)
SCHEME_SCRATCH_BYTES = 64 << 20


def corr_scheme_noalloc(x, y, window, scheme="unfused", border="fill", invalid=-2.0,
                        missing_le=-999.0, out=None, flags=None, stream=None):
    """corr_scheme with the library's fixed device workspace instead of a
    caller one (for callers that cannot allocate: pass ``out`` (and
    ``flags``) to allocate nothing here either).  Problems needing more than
    SCHEME_SCRATCH_BYTES raise; calls that overlap on one device race."""
    import torch
    _check_tensor(x, "x")
    _check_tensor(y, "y")
    if x.shape != y.shape or x.dtype != y.dtype:
        raise ValueError("x and y must have the same shape and dtype")
    if scheme not in SCHEMES:
        raise ValueError(f"scheme must be one of {sorted(SCHEMES)}")
    p = make_problem(tuple(x.shape), x.dtype, window, 1, border, "default", invalid, missing_le)
    code = validate(p)
    if code != 0:
        raise ValueError(f"{STATUS.get(code)}: {status_str(code)}")
    oshape = output_shape(p)
    if out is None:
        out = torch.empty(oshape, dtype=torch.float32, device=x.device)
    _check_tensor(out, "out")
    if tuple(out.shape) != tuple(oshape) or out.dtype != torch.float32:
        raise ValueError(f"out must be float32 of shape {tuple(oshape)}")
    if flags is not None:
        _check_tensor(flags, "flags")
        if tuple(flags.shape) != tuple(oshape) or flags.dtype != torch.uint8:
            raise ValueError(f"flags must be uint8 of shape {tuple(oshape)}")
    h = _stream_handle(stream, x.device)
    code = _load().swc_corr_scheme_noalloc(
        ctypes.byref(p), SCHEMES[scheme], ctypes.c_void_p(x.data_ptr()),
        ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(out.data_ptr()),
        ctypes.c_void_p(flags.data_ptr()) if flags is not None else None, h)
    _check(code)
    return out if flags is None else (out, flags)


class HostPlan:
    """End-to-end runs from host memory: slabs along the first axis, each
    copied in, computed and copied out on one of ``depth`` streams.  Inputs
    and outputs are CPU tensors (pinned for overlap); the plan owns its
    device staging buffers."""

    def __init__(self, shape, dtype, window, step=1, border="fill", band_rows=512, depth=3,
                 invalid=-2.0, missing_le=-999.0):
        self.problem = make_problem(tuple(shape), dtype, window, step, border, "default",
                                    invalid, missing_le)
        code = validate(self.problem)
        if code != 0:
            raise ValueError(f"{STATUS.get(code)}: {status_str(code)}")
        self.oshape = output_shape(self.problem)
        self._lib = _load()
        h = ctypes.c_void_p()
        _check(self._lib.swc_host_plan_create(ctypes.byref(self.problem), int(band_rows),
                                              int(depth), ctypes.byref(h)))
        self._h = h

    @property
    def bands(self) -> int:
        return int(self._lib.swc_host_plan_bands(self._h))

    def run(self, x, y, out=None, flags=None):
        """x, y: contiguous CPU tensors of the plan's shape and dtype.
        Returns (c, flags) CPU tensors (flags None unless given)."""
        import torch
        for t, n in ((x, "x"), (y, "y")):
            if not isinstance(t, torch.Tensor) or t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{n} must be a contiguous CPU tensor")
            if tuple(t.shape) != tuple(self.problem.shape[:self.problem.ndim]):
                raise ValueError(f"{n} has the wrong shape")
            if _dtype_code(t.dtype) != self.problem.dtype:
                raise ValueError(f"{n} has the wrong dtype")
        if out is None:
            out = torch.empty(self.oshape, dtype=torch.float32, pin_memory=x.is_pinned())
        if tuple(out.shape) != self.oshape or out.dtype != torch.float32 or out.is_cuda \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous float32 CPU tensor of the output shape")
        if flags is not None and (tuple(flags.shape) != self.oshape or flags.dtype != torch.uint8
                                  or flags.is_cuda or not flags.is_contiguous()):
            raise ValueError("flags must be a contiguous uint8 CPU tensor of the output shape")
        code = self._lib.swc_host_run(
            self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
            ctypes.c_void_p(out.data_ptr()),
            ctypes.c_void_p(flags.data_ptr()) if flags is not None else None)
        _check(code)
        return out, flags

    def close(self):
        if getattr(self, "_h", None):
            self._lib.swc_host_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cloud_mask(c, flags=None, tau=0.5, invalid=-2.0, out=None, stream=None):
    """uint8 device mask of the valid outputs with c < -tau (the cloud test of
    the paper's application)."""
    import torch
    _check_tensor(c, "c")
    if c.dtype != torch.float32:
        raise ValueError("c must be float32")
    if flags is not None:
        _check_tensor(flags, "flags")
        if flags.shape != c.shape or flags.dtype != torch.uint8:
            raise ValueError("flags must be uint8 of c's shape")
    if out is None:
        out = torch.empty(c.shape, dtype=torch.uint8, device=c.device)
    _check_tensor(out, "out")
    if out.shape != c.shape or out.dtype != torch.uint8:
        raise ValueError("out must be uint8 of c's shape")
    h = _stream_handle(stream, c.device)
    _check(_load().swc_cloud_mask(ctypes.c_void_p(c.data_ptr()),
                                  ctypes.c_void_p(flags.data_ptr()) if flags is not None else None,
                                  c.numel(), float(tau), float(invalid),
                                  ctypes.c_void_p(out.data_ptr()), h))
    return out


def filter_detections(c, idx, flags=None, tau=0.5, invalid=-2.0, stream=None):
    """For detections at flat output indices ``idx`` (int64 device tensor):
    0 = on a cloud pixel (reject), 1 = keep, 2 = index outside the map."""
    import torch
    _check_tensor(c, "c")
    _check_tensor(idx, "idx")
    if c.dtype != torch.float32 or idx.dtype != torch.int64:
        raise ValueError("c must be float32 and idx int64")
    if flags is not None:
        _check_tensor(flags, "flags")
        if flags.shape != c.shape or flags.dtype != torch.uint8:
            raise ValueError("flags must be uint8 of c's shape")
    keep = torch.empty(idx.shape, dtype=torch.uint8, device=c.device)
    h = _stream_handle(stream, c.device)
    _check(_load().swc_filter_detections(
        ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(flags.data_ptr()) if flags is not None else None,
        c.numel(), ctypes.c_void_p(idx.data_ptr()), idx.numel(), float(tau), float(invalid),
        ctypes.c_void_p(keep.data_ptr()), h))
    return keep


def tune_set(p: Problem, params) -> None:
    _check(_load().swc_tune_set(ctypes.byref(p), ctypes.byref(_params(params))))


def tune_get(p: Problem):
    lp = LaunchParams()
    _check(_load().swc_tune_get(ctypes.byref(p), ctypes.byref(lp)))
    return lp.as_tuple()


def set_debug(bits: int) -> None:
    _load().swc_set_debug(int(bits))


def get_debug() -> int:
    return int(_load().swc_get_debug())


class BatchPlan:
    """Many independent 2-D pairs computed by one persistent launch.

    ``pairs`` is a list of dicts with keys x, y (device tensors), window,
    and optional step, border, out, flags.  Shares dtype and accum."""

    def __init__(self, pairs, accum="default", invalid=-2.0, missing_le=-999.0, params=None,
                 return_flags=False):
        import torch
        if not pairs:
            raise ValueError("empty batch")
        lib = _load()
        n = len(pairs)
        probs = (Problem * n)()
        xs = (ctypes.c_void_p * n)()
        ys = (ctypes.c_void_p * n)()
        cs = (ctypes.c_void_p * n)()
        fs = (ctypes.c_void_p * n)()
        self.outputs, self.flags = [], []
        self._keep = []
        for i, pr in enumerate(pairs):
            x, y = pr["x"], pr["y"]
            _check_tensor(x, "x")
            _check_tensor(y, "y")
            if x.shape != y.shape or x.dtype != y.dtype:
                raise ValueError(f"pair {i}: x and y differ in shape/dtype")
            probs[i] = make_problem(tuple(x.shape), x.dtype, pr["window"], pr.get("step", 1),
                                    pr.get("border", "clip"), accum, invalid, missing_le)
            osh = output_shape(probs[i])
            out = pr.get("out")
            if out is None:
                out = torch.empty(osh, dtype=torch.float32, device=x.device)
            fl = pr.get("flags")
            if fl is None and return_flags:
                fl = torch.empty(osh, dtype=torch.uint8, device=x.device)
            self.outputs.append(out)
            self.flags.append(fl)
            self._keep += [x, y]
            xs[i], ys[i], cs[i] = x.data_ptr(), y.data_ptr(), out.data_ptr()
            fs[i] = fl.data_ptr() if fl is not None else None
        lp = _params(params)
        handle = ctypes.c_void_p()
        _check(lib.swc_batch_plan_create(n, probs, xs, ys, cs, fs,
                                         ctypes.byref(lp) if lp is not None else None,
                                         ctypes.byref(handle)))
        self._h = handle
        self._lib = lib
        self.device = pairs[0]["x"].device

    @property
    def items(self) -> int:
        return int(self._lib.swc_batch_plan_items(self._h))

    def launch(self, stream=None):
        _check(self._lib.swc_batch_launch(self._h, _stream_handle(stream, self.device)))
        return self.outputs

    def capture_graph(self, stream=None):
        """Capture one launch into a torch CUDA graph; returns the graph."""
        import torch
        g = torch.cuda.CUDAGraph()
        s = stream or torch.cuda.Stream(device=self.device)
        with torch.cuda.graph(g, stream=s):
            self.launch(stream=torch.cuda.current_stream(self.device))
        return g

    def close(self):
        if getattr(self, "_h", None):
            self._lib.swc_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
