"""The host library (hk_api.cpp) built with AddressSanitizer and UndefinedBehaviorSanitizer
against host-only stand-ins for the kernel launches, driven through every entry point of the C
ABI with invalid arguments and without a device: each returns its documented status, and the
sanitizers report nothing."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc for the HIP host headers")
def test_validation_paths_under_sanitizers(tmp_path):
    exe = str(tmp_path / "hk_validate")
    src = [os.path.join(ROOT, "paper_2101_02005_amd", "csrc", "hk_api.cpp"),
           os.path.join(HERE, "sanitize", "launch_stubs.cpp"),
           os.path.join(HERE, "sanitize", "validation_driver.cpp")]
    # host code only: each -fsanitize applies to the host pass
    cmd = ["hipcc", "-O1", "-g", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_2101_02005_amd", "csrc"),
           "-o", exe] + src
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", HIP_VISIBLE_DEVICES="",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=120)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-4000:]
    assert "ok: 0 failures" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stdout and "runtime error" not in r.stdout
