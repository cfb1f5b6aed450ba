"""Build libswcorr.so (HIP, gfx950) in-tree.

    python -m paper_1807_06507_amd.build          # compile everything
    python -m paper_1807_06507_amd.build --check  # compile, then list symbols
    python -m paper_1807_06507_amd.build --out DIR/libswcorr.so -DNAME=VALUE ...
                                                  # a variant build elsewhere

Every translation unit under csrc/ is compiled by hipcc for gfx950 into
_build/, then linked into paper_1807_06507_amd/libswcorr.so next to this file.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libswcorr.so")
ARCH = os.environ.get("SWC_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                  if f.endswith(".hip") or f.endswith(".cpp"))


def _compile(src, build_dir=BUILD, defines=()):
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [_hipcc()] + HIP_FLAGS + list(defines) + lang + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every source and link `out` (default: the in-tree library).
    `defines` are extra -D options; a build with any goes to its own object
    directory next to `out`."""
    build_dir = BUILD if not defines and out == LIB else out + ".objs"
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda f: _compile(f, build_dir, defines), srcs))
    LIB_OUT = out
    tmp = LIB_OUT + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-ldl"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_OUT)
    if verbose:
        print(f"built {LIB_OUT}")
    return LIB_OUT


if __name__ == "__main__":
    _out = LIB
    if "--out" in sys.argv:
        _out = os.path.abspath(sys.argv[sys.argv.index("--out") + 1])
    build(verbose=True, out=_out, defines=[a for a in sys.argv[1:] if a.startswith("-D")])
    if "--check" in sys.argv:
        out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True)
        print("\n".join(l for l in out.stdout.splitlines() if " swc_" in l))
