"""Host sanitizers (CPU only): the oracle built with gcc's address and
undefined-behaviour sanitizers and driven over degenerate inputs, and the
collapse library's host side (argument validation of the C ABI) built with
the same sanitizers on the host pass only and driven over invalid calls.
Any sanitizer report fails the run (halt_on_error / no recovery)."""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "oracle", "collapse_oracle.c"), os.path.join(HERE, "oracle_driver.c"),
           "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    _run(exe)


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not installed")
def test_abi_validation_under_host_asan_ubsan(tmp_path):
    exe = str(tmp_path / "abi_driver")
    lib = str(tmp_path / "libpino_san.so")
    hipcc = "/opt/rocm/bin/hipcc"
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.run([hipcc, *common, "-shared", os.path.join(ROOT, "paper_2510_02873_amd", "csrc",
                                                              "pino_collapse.hip"),
                    "-o", lib, "-L/opt/rocm/lib", "-lhipfft"], check=True, capture_output=True, timeout=900)
    # the C driver with the same (clang) sanitizer runtime as the library
    subprocess.run(["/opt/rocm/llvm/bin/clang", "-fsanitize=address,undefined", "-g",
                    os.path.join(HERE, "abi_driver.c"), "-o", exe, lib,
                    "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath,/opt/rocm/lib"],
                   check=True, capture_output=True, timeout=300)
    _run(exe)
