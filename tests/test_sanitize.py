"""Sanitizer builds on the CPU: the C oracle under AddressSanitizer and
UndefinedBehaviorSanitizer, run on a small seeded problem by a driver that also
checks exact properties of the direct sums (weighted adjoint identity, PSF
symmetry and peak).  Any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_adjoint")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "sanitize", "oracle_adjoint.c"), os.path.join(ROOT, "oracle", "pfb_oracle.c"),
           "-lm", "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert r.stdout.strip().endswith("ok")


def _hipcc():
    p = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    return p if os.path.exists(p) else shutil.which("hipcc")


def test_host_code_under_asan_ubsan(tmp_path):
    """The library's host code (plan creation and argument validation) rebuilt with
    host-side AddressSanitizer and UndefinedBehaviorSanitizer, linked with the built
    kernel objects, running the validation paths that need no GPU."""
    hipcc = _hipcc()
    build = os.path.join(ROOT, "paper_2101_08072_amd", "_build")
    objs = [os.path.join(build, n) for n in ("pfb_kernels.o", "pfb_sort.o")]
    if hipcc is None or not all(os.path.exists(o) for o in objs):
        pytest.skip("hipcc or the built kernel objects are missing (run __graft_entry__.build())")
    csrc = os.path.join(ROOT, "paper_2101_08072_amd", "csrc")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["-std=c++17", "-O1", "-g", "--offload-arch=gfx950", "-I", os.path.join(ROOT, "include"), "-I", csrc,
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    host = str(tmp_path / "host.o")
    drv = str(tmp_path / "drv.o")
    exe = str(tmp_path / "host_validation")
    subprocess.check_call([hipcc, *common, *san, "-c", os.path.join(csrc, "pfb_host.cpp"), "-o", host],
                          stderr=subprocess.DEVNULL)
    subprocess.check_call([hipcc, *common, *san, "-c", os.path.join(HERE, "sanitize", "host_validation.cpp"),
                           "-o", drv], stderr=subprocess.DEVNULL)
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                           "-Xarch_host", "-fsanitize=undefined", drv, host, *objs, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert r.stdout.strip().endswith("ok")
