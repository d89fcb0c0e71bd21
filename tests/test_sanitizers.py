"""Host code under the address and undefined-behaviour sanitizers (CPU).

The oracle source is compiled with gcc into a driver that steps small
domains forward and backward through every branch (absorbing faces, a
two-pole box, Bloch-periodic axes with a box on the seam, tensor media);
the library's host code is compiled with hipcc, the sanitizers on the host
side only, and a driver calls fdtd_create and fdtd_stream_create through
the C-ABI on valid descriptors under a tiny budget and on invalid ones, so
that the descriptor checks, the node-by-node tensor admission, the memory
estimates and the streamed slab plan run without a GPU.  Each driver must
finish with status 0 and no sanitizer report.  Both builds go to a
temporary directory.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, **kw)


def _clean(out):
    return "runtime error" not in out and "AddressSanitizer" not in out and "Sanitizer" not in out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_driver")
        b = _run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                  "-fno-sanitize-recover=undefined", "-Wno-unknown-pragmas",
                  os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe, "-lm"])
        assert b.returncode == 0, b.stderr[-2000:]
        r = _run([exe], env=SAN_ENV, timeout=300)
        out = r.stdout + r.stderr
        assert r.returncode == 0 and _clean(out), out[-4000:]
        assert out.count(": ok") == 3, out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_runtime_host_code_under_asan_ubsan():
    csrc = os.path.join(ROOT, "paper_2609_30039_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Wno-unused-command-line-argument",
             "-Wno-unknown-warning-option"]
    from paper_2609_30039_amd.build import SOURCES
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        for src in SOURCES:
            o = os.path.join(tmp, src + ".o")
            b = _run([HIPCC, "-x", "hip", *flags, "-I", inc, "-I", csrc, "-c", os.path.join(csrc, src), "-o", o])
            assert b.returncode == 0, b.stderr[-2000:]
            objs.append(o)
        lib = os.path.join(tmp, "libfdtd_san.so")
        b = _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
                  "-Xarch_host", "-fsanitize=undefined", *objs, "-o", lib])
        assert b.returncode == 0, b.stderr[-2000:]
        exe = os.path.join(tmp, "runtime_driver")
        b = _run([HIPCC, "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                  "-fsanitize=undefined", "-I", inc, "-x", "c++",
                  os.path.join(ROOT, "tests", "sanitize", "runtime_driver.cpp"), "-x", "none", lib,
                  "-Wl,-rpath," + tmp, "-o", exe])
        assert b.returncode == 0, b.stderr[-2000:]
        r = _run([exe], env=SAN_ENV, timeout=300)
        out = r.stdout + r.stderr
        assert r.returncode == 0 and _clean(out), out[-4000:]
        assert out.rstrip().endswith("ok"), out[-2000:]
