"""Build the fork-processing library's HIP sources for the host CPU, against
the CPU stand-in for the HIP runtime in this folder (test infrastructure):

    python tests/simt/build.py [--asan]

The result, tests/simt/libfork_simt.so, exports the same C ABI as the GPU
library plus simt_check_* (the pool ownership checker's results).  Only the
tests load it, by path; the product binding never does.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2103_14915_amd", "csrc")
OUT = os.path.join(HERE, "_build")


def lib_path(asan: bool = False) -> str:
    return os.path.join(HERE, "libfork_simt_asan.so" if asan else "libfork_simt.so")


def build(asan: bool = False, force: bool = False) -> str:
    lib = lib_path(asan)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip"))) + [os.path.join(HERE, "simt.cpp"),
                                                              os.path.join(HERE, "check.cpp")]
    deps = srcs + sorted(glob.glob(os.path.join(CSRC, "*.h"))) + sorted(glob.glob(os.path.join(HERE, "hip", "*.h")))
    deps += [os.path.join(ROOT, "include", "fork.h"), os.path.abspath(__file__)]
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= max(os.path.getmtime(d) for d in deps):
        return lib
    os.makedirs(OUT, exist_ok=True)
    tag = "asan" if asan else "plain"
    flags = ["-std=c++17", "-O1", "-g", "-fPIC", "-pthread", "-Wno-attributes", "-Wno-unused-result",
             "-Wno-unused-function", "-fno-extern-tls-init", "-DFORK_CERT_MAX_PART=65536u", "-I", HERE, "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    if asan:
        flags += ["-fsanitize=address", "-fno-omit-frame-pointer"]

    def comp(src):
        obj = os.path.join(OUT, f"{os.path.basename(src)}.{tag}.o")
        lang = ["-x", "c++"] if src.endswith(".hip") else []
        r = subprocess.run(["g++", *flags, *lang, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(f"g++ failed for {src}:\n{r.stderr[-6000:]}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(comp, srcs))
    tmp = lib + ".tmp%d" % os.getpid()
    r = subprocess.run(["g++", *flags, "-shared", "-o", tmp, *objs], capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(asan="--asan" in sys.argv, force=True))
