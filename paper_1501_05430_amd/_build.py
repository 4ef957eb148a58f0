"""Compile liblbm.so for gfx950 with hipcc (in-tree, next to this file), plus the benchmark's probe library.

Each source is compiled to an object in parallel, then the objects are linked; the host functions that launch
kernels live in the same translation unit as their kernels, so no relocatable device code is needed.
"""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = [os.path.join(CSRC, "lbm_kernels.hip"), os.path.join(CSRC, "lbm_step2.hip"), os.path.join(CSRC, "lbm_adjoint.hip"),
           os.path.join(CSRC, "lbm_noalloc.hip"), os.path.join(CSRC, "lbm_api.cpp")]
HEADERS = [os.path.join(CSRC, "lbm_internal.h"), os.path.join(CSRC, "lbm_device.h"),
           os.path.join(os.path.dirname(HERE), "include", "lbm.h")]
# bandwidth probes used by bench.py for the copy ceiling (not part of the method's library)
PROBE_LIB = os.path.join(HERE, "libbwprobe.so")
PROBE_SOURCES = [os.path.join(CSRC, "bw_probe.hip")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in SOURCES + HEADERS if os.path.exists(s))


OBJ_DIR = os.path.join(HERE, "_build")  # object cache (git-ignored)


def _link(sources, out, verbose, force):
    os.makedirs(OBJ_DIR, exist_ok=True)
    jobs = max(1, min(len(sources), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    objs = [os.path.join(OBJ_DIR, os.path.basename(s) + ".o") for s in sources]
    newest_header = max(os.path.getmtime(h) for h in HEADERS)

    def compile_one(pair):
        src, obj = pair
        if (not force and os.path.exists(obj) and os.path.getmtime(obj) >= os.path.getmtime(src)
                and os.path.getmtime(obj) >= newest_header):
            return
        tmp = obj + ".tmp.o"
        cmd = [HIPCC, *FLAGS, "-c", src, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, obj)

    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(compile_one, zip(sources, objs)))
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(verbose: bool = False, force: bool = True) -> str:
    """Compile and link both libraries; force=False reuses objects newer than their source and the headers."""
    _link(PROBE_SOURCES, PROBE_LIB, verbose, force)
    return _link(SOURCES, LIB, verbose, force)


if __name__ == "__main__":
    import sys
    print(build(verbose=True, force="--incremental" not in sys.argv))
