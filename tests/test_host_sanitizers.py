"""Host code of libads under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the library is built with both sanitizers on its host pass
(device code unchanged), and tests/host_sanitize_driver.c drives every host
path that runs without a GPU (argument validation, the clean-up of a setup
that fails at its first device call, the tuning-cache and weights-file
parsers, the network shape arithmetic).  Any sanitizer report fails the run.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = "/opt/rocm"


@pytest.mark.skipif(not os.path.exists(os.path.join(ROCM, "llvm", "bin", "clang")),
                    reason="ROCm LLVM toolchain not installed")
@pytest.mark.timeout(600)
def test_host_paths_clean_under_asan_and_ubsan(tmp_path):
    from paper_2201_02250_amd import build
    lib = build.build(sanitize=True, out=str(tmp_path / "libads_hostsan.so"))
    clang = os.path.join(ROCM, "llvm", "bin", "clang")
    exe = str(tmp_path / "host_sanitize_driver")
    cmd = [clang, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-shared-libsan", "-I", os.path.join(ROOT, "include"),
           os.path.join(HERE, "host_sanitize_driver.c"), lib,
           "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath," + os.path.dirname(
               subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                              capture_output=True, text=True).stdout.strip()),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    scratch = tmp_path / "scratch"
    scratch.mkdir()
    env = dict(os.environ)
    # leaks of our host code are reported; the HIP runtime's one-time
    # allocations at process exit are not ours
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1:protect_shadow_gap=0"
    env["LSAN_OPTIONS"] = "suppressions=" + str(tmp_path / "lsan.supp")
    (tmp_path / "lsan.supp").write_text("leak:libamdhip64\nleak:libhsa-runtime64\nleak:libdrm\n")
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe, str(scratch)], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    print(out)
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out
    assert "ERROR: LeakSanitizer" not in out, out
    assert r.returncode == 0, out
