"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU (no GPU needed):

* the oracle (vfs_oracle.c, vfso.c) built with gcc's sanitizers and run
  through oracle/sanitize_driver.c: every entry point, the whole method in
  both regularisers and all three data terms, leak detection on;
* the library's host code (every .hip file, sanitizers on the host side
  only) driven by tests/abi_sanitize_driver.c through every entry point's
  argument validation, which returns before any device work.

Both executables must exit 0 with no sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, (cmd[0], r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    return r


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-o", exe, os.path.join(ROOT, "oracle", "vfs_oracle.c"),
          os.path.join(ROOT, "oracle", "vfso.c"), os.path.join(ROOT, "oracle", "sanitize_driver.c"), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="4")
    r = _run([exe], env=env)
    assert "ok" in r.stdout


def test_library_argument_validation_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    lib = str(tmp_path / "libvfs_san.so")
    srcs = sorted(os.path.join(ROOT, "paper_1909_07545_amd", "csrc", f)
                  for f in os.listdir(os.path.join(ROOT, "paper_1909_07545_amd", "csrc")) if f.endswith(".hip"))
    _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-I", os.path.join(ROOT, "include"), "-o", lib] + srcs)
    exe = str(tmp_path / "abi_san")
    _run([CLANG, "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"),
          "-o", exe, os.path.join(ROOT, "tests", "abi_sanitize_driver.c"), "-L", str(tmp_path), "-lvfs_san",
          "-Wl,-rpath," + str(tmp_path), "-lm"])
    # the HIP runtime's own start-up allocations are not ours to report
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = _run([exe], env=env, timeout=120)
    assert "ok" in r.stdout
