"""Builds libtfstat.so (HIP kernels + C ABI runtime) for gfx950 with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
_CSRC = os.path.join(_HERE, "csrc")
LIB_NAME = "libtfstat.so"

SOURCES = ["kernels.hip", "kernels_mfma.hip", "kernels_recur.hip", "kernels_abc.hip", "noalloc.hip", "runtime.cpp"]

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # packed FP32 instructions are kept out of every build
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def library_path() -> str:
    return os.path.join(_HERE, LIB_NAME)


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("building %s failed" % LIB_NAME)


def build(verbose: bool = False) -> str:
    """Compiles every source to an object (in parallel), then links the
    shared library.  Always recompiles."""
    from concurrent.futures import ThreadPoolExecutor
    srcs = [os.path.join(_CSRC, s) for s in SOURCES if os.path.exists(os.path.join(_CSRC, s))]
    out = library_path()
    obj_dir = os.path.join(os.path.dirname(_HERE), "_build", "tfstat")
    os.makedirs(obj_dir, exist_ok=True)
    objs = [os.path.join(obj_dir, os.path.basename(s) + ".o") for s in srcs]
    cc = hipcc()
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        for f in [ex.submit(_run, [cc, *HIP_FLAGS, "-c", "-o", o, s], verbose) for s, o in zip(srcs, objs)]:
            f.result()
    tmp = out + ".tmp%d" % os.getpid()
    _run([cc, *HIP_FLAGS, "-shared", "-o", tmp, *objs, "-lpthread"], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
