"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code (CPU).

The C oracle (every public function, including the clustering of the mixture
approximations) and the library's host half (configuration checks, ordering,
partition, per-block CSR/CSC, workspace sizing and plan introspection through
bmf_init_host, over every order, several partitions and every approximation)
are compiled with both sanitizers on the host side only and run as child
processes; any invalid access or undefined operation aborts the child.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


def test_oracle_under_sanitizers():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=c99"] + SAN + [os.path.join(ROOT, "tests", "asan", "oracle_driver.c"),
                                                  "-o", exe, "-lm"])
    r = _run([exe], env=ENV, timeout=300)
    assert "oracle driver done" in r.stdout


def test_library_host_half_under_sanitizers():
    hipcc = "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    from paper_1703_00734_amd import build as B
    os.makedirs(OUT, exist_ok=True)
    dev_objs = []
    for src in ("kernels.hip", "planner_gpu.hip"):         # device code, no sanitizer
        obj = os.path.join(B.BUILD, os.path.splitext(src)[0] + ".o")
        if not os.path.exists(obj):
            os.makedirs(B.BUILD, exist_ok=True)
            obj = B._compile(src)
        dev_objs.append(obj)
    host = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-I" + os.path.join(ROOT, "include"),
            "-I" + B.CSRC, "-Wno-unused-value", "-Wno-unused-result"]
    for f in SAN:
        host += ["-Xarch_host", f]
    objs = []
    for src in (os.path.join(ROOT, "tests", "asan", "host_driver.cpp"), os.path.join(B.CSRC, "api.cpp"),
                os.path.join(B.CSRC, "planner.cpp")):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        _run([hipcc, "-c"] + host + [src, "-o", obj])
        objs.append(obj)
    exe = os.path.join(OUT, "host_driver")
    _run([hipcc, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address,undefined"] + objs + dev_objs + ["-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "host driver done, 0 failures" in r.stdout
