"""Host sanitizer runs (CPU only): the FP64 oracle and the library's
host-side logic (workspace sizing and argument checks of every entry point)
built with AddressSanitizer and UndefinedBehaviorSanitizer and driven by the
small C programs under tests/sanitize/.  A run passes when the driver exits 0
and the sanitizers print nothing.  GPU code is not instrumented: the library
copy is built with the sanitizers on the host side only (-Xarch_host), and
the driver calls no entry point that reaches the GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(ROOT, "_build", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)
    return r.returncode, r.stdout + r.stderr


def _san_env():
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    return env


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc missing")
def test_oracle_under_asan_ubsan():
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_driver")
    rc, log = _run(["gcc", "-O1", "-g", "-std=c11", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-ffp-contract=off",
                    "-o", exe, os.path.join(ROOT, "oracle", "rcholqr_oracle.c"),
                    os.path.join(SAN, "oracle_driver.c"), "-lm"])
    assert rc == 0, log
    rc, log = _run([exe], env=_san_env())
    print(log)
    assert rc == 0, log
    assert "runtime error" not in log and "ERROR: AddressSanitizer" not in log
    assert "0 failures" in log


@pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(HIPCC)),
                    reason="ROCm clang / hipcc missing")
def test_library_host_logic_under_asan_ubsan():
    from paper_2210_09953_amd import build as hipbuild
    os.makedirs(OUT, exist_ok=True)
    flags = list(hipbuild.FLAGS)
    # Host-side sanitizers only (device code is not instrumented).
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xarch_host", "-g"]
    # api.hip holds every entry point's argument checks and workspace
    # layouts: it is the instrumented object; the kernels' objects come from
    # the regular build (built here if missing).
    objs = []
    for src in hipbuild.sources():
        if os.path.basename(src) == "api.hip":
            obj = os.path.join(OUT, "api.hip.o")
            rc, log = _run([HIPCC] + flags + san + ["-c", src, "-o", obj], timeout=900)
            assert rc == 0, log
        else:
            obj = os.path.join(hipbuild.BUILD, os.path.basename(src) + ".o")
            if not os.path.exists(obj):
                os.makedirs(hipbuild.BUILD, exist_ok=True)
                obj = hipbuild._compile(src)
        objs.append(obj)
    lib = os.path.join(OUT, "librcholqr_san.so")
    rc, log = _run([HIPCC, "-shared", f"--offload-arch={hipbuild.ARCH}", "-Xarch_host",
                    "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-o", lib] + objs)
    assert rc == 0, log
    exe = os.path.join(OUT, "api_driver")
    rc, log = _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", os.path.join(ROOT, "include"), "-o", exe,
                    os.path.join(SAN, "api_driver.c"), lib, "-Wl,-rpath," + OUT])
    assert rc == 0, log
    env = _san_env()
    # The HIP runtime the library loads is not instrumented and keeps its
    # allocations until exit: leak reports would be about it, not this code.
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    rc, log = _run([exe], env=env)
    print(log)
    assert rc == 0, log
    assert "runtime error" not in log and "ERROR: AddressSanitizer" not in log
    assert "0 failures" in log
