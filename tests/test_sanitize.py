"""The FP64 oracle and the host side of the C ABI built with
AddressSanitizer and UndefinedBehaviorSanitizer and run on the CPU: no
out-of-bounds access, use after free, leak or undefined behaviour.

- oracle: gcc -fsanitize=address,undefined of oracle/sc_oracle.c with a
  driver that calls every entry point (tests/sanitize/oracle_driver.c);
- library host side: hipcc with -Xarch_host -fsanitize=address,undefined
  (host code only; the GPU code is built as usual) of csrc/sc_lbm.cpp and
  the kernel units, linked with a driver that calls the entry points that
  validate their arguments before any device work
  (tests/sanitize/abi_driver.cpp); no GPU is needed.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="abort_on_error=1:detect_leaks=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-ffp-contract=off",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           os.path.join(ROOT, "oracle", "sc_oracle.c"), os.path.join(HERE, "oracle_driver.c"),
                           "-o", exe, "-lm"])
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr[-4000:]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc") or shutil.which("gcc") is None,
                    reason="needs hipcc")
def test_abi_host_side_under_asan_ubsan(tmp_path):
    from paper_1906_11027_amd import build as B
    objs = [os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o") for s in B.SOURCES if s != "sc_lbm.cpp"]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    lib_o, drv_o, exe = str(tmp_path / "sc_lbm_asan.o"), str(tmp_path / "drv.o"), str(tmp_path / "abi_asan")
    subprocess.check_call([_hipcc(), "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=" + B.ARCH,
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + san +
                          ["-x", "hip", "-c", os.path.join(B.CSRC, "sc_lbm.cpp"), "-o", lib_o])
    subprocess.check_call([_hipcc(), "-O1", "-g", "-std=c++17"] + san +
                          ["-c", os.path.join(HERE, "abi_driver.cpp"), "-o", drv_o])
    subprocess.check_call([_hipcc(), "--offload-arch=" + B.ARCH] + san + [drv_o, lib_o] + objs + ["-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr[-4000:]
