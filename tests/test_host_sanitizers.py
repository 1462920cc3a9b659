"""Host code under AddressSanitizer, LeakSanitizer and UBSan (CPU only).

* The runtime's host sources (runtime.cpp, pipeline.cpp, server.cpp) are
  compiled for the host alone with the sanitizers, the kernel launchers
  replaced by stand-ins that abort (tests/host/launch_stubs.cpp), and linked
  into tests/host/sanitize_driver.cpp, which runs the C ABI's argument
  validation and error paths (no GPU here, so no call reaches a launch) and a
  long random sequence of the admission arena against a granule map.
* The oracle (orc_core.c in both modes, orc_grad.c, orc_math.c) is compiled
  with the sanitizers into tests/host/oracle_driver.c, which renders a small
  scene with degenerate Gaussians through every binning mode and the adjoint.

Any sanitizer report ends the process with a non-zero status
(-fno-sanitize-recover=all); leaks inside the HIP runtime's own libraries are
not ours and are suppressed by library name.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2408_07967_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")
ORC = os.path.join(ROOT, "oracle")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _env(td):
    supp = os.path.join(td, "lsan.supp")
    with open(supp, "w") as f:
        f.write("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libhsakmt\nleak:libdrm\n")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["LSAN_OPTIONS"] = f"suppressions={supp}"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    return env


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang not installed")
def test_runtime_host_paths_under_sanitizers():
    td = tempfile.mkdtemp(prefix="fgs_san_")
    try:
        flags = ["-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
                 "-I", CSRC, *SAN]
        srcs = [os.path.join(CSRC, f) for f in ("runtime.cpp", "pipeline.cpp", "server.cpp")]
        srcs += [os.path.join(HOST, f) for f in ("launch_stubs.cpp", "sanitize_driver.cpp")]
        objs = []
        for s in srcs:
            o = os.path.join(td, os.path.basename(s) + ".o")
            _run([CLANG, *flags, "-c", s, "-o", o])
            objs.append(o)
        exe = os.path.join(td, "sanitize_driver")
        _run([CLANG, *SAN, *objs, "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lpthread",
              "-o", exe])
        r = _run([exe], env=_env(td), timeout=300)
        assert "sanitize ok" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    finally:
        shutil.rmtree(td, ignore_errors=True)


def test_oracle_under_sanitizers():
    td = tempfile.mkdtemp(prefix="orc_san_")
    try:
        cflags = ["gcc", "-std=c11", "-fopenmp", "-ffp-contract=off", "-I", ORC, *SAN]
        objs = []
        for src, defs, name in ((os.path.join(ORC, "orc_core.c"), ["-DORC_FP64"], "core64.o"),
                                (os.path.join(ORC, "orc_core.c"), ["-DORC_FP32"], "core32.o"),
                                (os.path.join(ORC, "orc_grad.c"), [], "grad.o"),
                                (os.path.join(ORC, "orc_math.c"), [], "math.o"),
                                (os.path.join(HOST, "oracle_driver.c"), [], "driver.o")):
            o = os.path.join(td, name)
            _run([*cflags, *defs, "-c", src, "-o", o])
            objs.append(o)
        exe = os.path.join(td, "oracle_driver")
        _run(["gcc", *SAN, "-fopenmp", *objs, "-lm", "-o", exe])
        r = _run([exe], env=_env(td), timeout=300)
        assert "oracle sanitize ok" in r.stdout
        assert "runtime error" not in r.stderr, r.stderr[-4000:]
    finally:
        shutil.rmtree(td, ignore_errors=True)
