"""The host side of the C ABI and the CPU oracle under AddressSanitizer and
UBSan (no GPU).

* ``sanitize/host_check.cpp`` drives every validation, sizing and
  argument-rejection path of ``include/lbm.h`` that runs before any device
  work, against a build of the library whose host code carries the
  sanitizers and the C++ library's checked containers (_GLIBCXX_ASSERTIONS;
  its device code is compiled without optimisation, to keep the build
  short; it never runs here).
* ``sanitize/oracle_check.c`` runs every oracle entry point on small and
  ragged lattices (down to 1 x 1) with every option, built together with the
  oracle's source under the sanitizers.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s\n%s" % (" ".join(cmd), r.stdout[-3000:], r.stderr[-3000:])
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-ffp-contract=off", "-Wall", "-Wextra", "-Wno-unknown-pragmas", "-I" + os.path.join(ROOT, "oracle"),
          os.path.join(HERE, "sanitize", "oracle_check.c"), os.path.join(ROOT, "oracle", "lbm_oracle.c"),
          "-lm", "-o", exe])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "oracle checks passed" in r.stdout


@pytest.mark.timeout(600)
@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm compilers not found")
def test_host_abi_under_address_and_ub_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1802_01272_amd", "csrc")
    lib = str(tmp_path / "liblbm_san.so")
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-Xarch_device", "-O0", "-g0", "-std=c++17", "-fPIC",
          "-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-omit-frame-pointer",
          "-Xarch_host", "-g", "-Xarch_host", "-D_GLIBCXX_ASSERTIONS",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include"), "-I" + csrc, "-shared",
          os.path.join(csrc, "lbm_api.hip"), os.path.join(csrc, "lbm_kernels.hip"), "-o", lib])
    exe = str(tmp_path / "host_check")
    _run([CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-D_GLIBCXX_ASSERTIONS",
          "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "sanitize", "host_check.cpp"),
          "-L" + str(tmp_path), "-llbm_san", "-Wl,-rpath," + str(tmp_path), "-o", exe])
    r = _run([exe], env=SAN_ENV, timeout=300)
    assert "host checks passed" in r.stdout
