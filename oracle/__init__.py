"""CPU reference ("oracle") for the sliding-window Pearson correlation.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It shares no
code with the GPU path.  The arithmetic lives in ``oracle.c`` (plain C, FP64,
window by window, the classical two-pass formula of the paper's Introduction);
this module only compiles it with gcc and marshals numpy arrays.

``corr`` returns ``(c32, c64, flags)``:
  c64   FP64 two-pass coefficient (or the invalid value where flagged);
  c32   float32 result: exactly rounded (ties to even) for u8/u16 input,
        ``float(c64)`` for float32 input;
  flags bit 1 BORDER, 2 MISSING, 4 ZVAR_X, 8 ZVAR_Y (0 = valid).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

DTYPES = {np.dtype(np.uint8): 0, np.dtype(np.uint16): 1, np.dtype(np.float32): 2}
BORDERS = {"fill": 0, "clip": 1, "valid": 2}
FLAG_BORDER, FLAG_MISSING, FLAG_ZVAR_X, FLAG_ZVAR_Y = 1, 2, 4, 8


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile oracle.c (or ``src``) into liboracle.so (or ``out``) with gcc
    and OpenMP.  Returns the path."""
    if not force and os.path.exists(out):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _bind(lib):
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_output_shape.argtypes = [ctypes.c_int, i64p, i32p, i32p, ctypes.c_int, i64p]
    lib.oracle_output_shape.restype = ctypes.c_int
    lib.oracle_corr.argtypes = [
        ctypes.c_int, i64p, i32p, i32p, ctypes.c_int, ctypes.c_int,
        ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
        i64p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
        ctypes.c_int,
    ]
    lib.oracle_corr.restype = ctypes.c_int
    lib.oracle_rn32_ratio.argtypes = [ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64]
    lib.oracle_rn32_ratio.restype = ctypes.c_float
    lib.oracle_has_openmp.restype = ctypes.c_int
    return lib


def _load(path=None):
    """The default compiled oracle, or (``path`` given) another build of it,
    e.g. a deliberately broken variant in the mutation test."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _bind(ctypes.CDLL(_LIB))
        return _lib


def _per_dim(v, ndim, name):
    if np.isscalar(v):
        return [int(v)] * ndim
    v = [int(t) for t in v]
    if len(v) != ndim:
        raise ValueError(f"{name} needs {ndim} entries, got {len(v)}")
    return v


def _arr(ctype, vals):
    return (ctype * 3)(*(list(vals) + [1] * (3 - len(vals))))


def output_shape(shape, window, step=1, border="fill", lib=None):
    ndim = len(shape)
    lib = lib or _load()
    w = _per_dim(window, ndim, "window")
    s = _per_dim(step, ndim, "step")
    out = (ctypes.c_int64 * 3)()
    rc = lib.oracle_output_shape(ndim, _arr(ctypes.c_int64, shape), _arr(ctypes.c_int32, w),
                                 _arr(ctypes.c_int32, s), BORDERS[border], out)
    if rc != 0:
        raise ValueError("invalid problem")
    return tuple(int(out[d]) for d in range(ndim))


def corr(x, y, window, step=1, border="fill", invalid=-2.0, missing_le=-999.0,
         indices=None, threads=0, lib=None):
    """Evaluate the oracle.  ``indices`` (optional) lists flat output indices
    (C order of the output shape); then 1-D arrays of that length come back."""
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y)
    if x.shape != y.shape or x.dtype != y.dtype:
        raise ValueError("x and y must have the same shape and dtype")
    if x.dtype not in DTYPES:
        raise ValueError(f"unsupported dtype {x.dtype}")
    ndim = x.ndim
    w = _per_dim(window, ndim, "window")
    s = _per_dim(step, ndim, "step")
    lib = lib or _load()
    oshape = output_shape(x.shape, w, s, border, lib=lib)
    if indices is None:
        n = int(np.prod(oshape))
        idx_ptr = None
        shape_out = oshape
    else:
        idx = np.ascontiguousarray(indices, dtype=np.int64).ravel()
        n = idx.size
        idx_ptr = idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        shape_out = (n,)
    c64 = np.empty(n, np.float64)
    c32 = np.empty(n, np.float32)
    fl = np.empty(n, np.uint8)
    rc = lib.oracle_corr(ndim, _arr(ctypes.c_int64, x.shape), _arr(ctypes.c_int32, w),
                         _arr(ctypes.c_int32, s), BORDERS[border], DTYPES[x.dtype],
                         float(invalid), float(missing_le), x.ctypes.data, y.ctypes.data,
                         idx_ptr, n, c64.ctypes.data, c32.ctypes.data, fl.ctypes.data,
                         int(threads))
    if rc != 0:
        raise RuntimeError(f"oracle_corr failed ({rc})")
    return c32.reshape(shape_out), c64.reshape(shape_out), fl.reshape(shape_out)


def rn32_ratio(P: int, Q: int, R: int, lib=None) -> np.float32:
    """Exactly rounded float32 of P/sqrt(Q*R) (64-bit operands)."""
    return np.float32((lib or _load()).oracle_rn32_ratio(int(P), int(Q), int(R)))


def has_openmp() -> bool:
    return bool(_load().oracle_has_openmp())


def cloud_mask(c32, flags, tau):
    """The application's cloud test on a finished map (the paper's
    Introduction: under clouds the visible/infrared correlation is close to
    -1): 1 where the output is valid (flag 0) and c < -tau, compared in
    float32, else 0."""
    c32 = np.asarray(c32, dtype=np.float32)
    return ((np.asarray(flags) == 0) & (c32 < np.float32(-tau))).astype(np.uint8)
