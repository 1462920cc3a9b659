"""Build the gfx950 HIP library libfgs.so in-tree with hipcc.

Every .hip kernel file and the runtime are compiled for gfx950 only.
k_project.hip (preprocessing and key emission) is compiled with
-ffp-contract=off so that its binary32 arithmetic is the canonical operation
sequence; the other kernels may contract multiply-adds.  Packed FP32
instructions are disabled for all device code.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfgs.so")

COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
PER_FILE = {
    "k_project.hip": ["-ffp-contract=off"],
}
SOURCES = ["runtime.cpp", "pipeline.cpp", "server.cpp", "noalloc.hip", "k_project.hip", "k_radix.hip", "k_sort.hip",
           "k_blend.hip", "k_backward.hip", "k_peaks.hip"]


def hipcc():
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c


def _compile(src, outdir, verbose):
    out = os.path.join(outdir, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [hipcc(), *COMMON, *PER_FILE.get(os.path.basename(src), []), *lang, "-c", os.path.join(CSRC, src),
           "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = ("packed-fp32-ops", "argument unused during compilation: '--hip-link'")
    msgs = "\n".join(l for l in (r.stderr or "").splitlines() if not any(n in l for n in noise))
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msgs}")
    if msgs.strip() and verbose:
        print(msgs)
    return out


def build(verbose=False):
    with tempfile.TemporaryDirectory() as td:
        with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
            objs = list(ex.map(lambda s: _compile(s, td, verbose), SOURCES))
        tmp = LIB + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr}")
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
