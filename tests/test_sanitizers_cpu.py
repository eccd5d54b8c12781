"""Host code under the address and undefined-behaviour sanitizers (CPU).

The FP64 oracle (oracle/dp_oracle.c) is compiled together with a small driver
(tests/native/oracle_sanitize_main.c) with -fsanitize=address,undefined and run on small
random problems of every edge shape (S = 2, zero window, window >= S, K = 1); any
out-of-bounds access, leak or undefined operation aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           os.path.join(ROOT, "oracle", "dp_oracle.c"),
           os.path.join(ROOT, "tests", "native", "oracle_sanitize_main.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # verify_asan_link_order=0: the run tolerates a library preloaded ahead of the
    # sanitizer runtime by the environment
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok", r.stdout + r.stderr


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not found")
def test_library_host_code_under_address_and_ub_sanitizers(tmp_path):
    """The library's sources built with the sanitizers on the host side only (the device
    code is built as usual), linked with a driver that calls every host-only path: argument
    validation of each field, workspace and checkpoint sizes, error strings, the paper-mode
    grid sizes and the plan's rejections.  No call reaches the device."""
    exe = str(tmp_path / "abi_asan")
    csrc = os.path.join(ROOT, "paper_2511_15629_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in ("dp_kernels.hip", "dp_api.hip", "dp_batch.hip",
                                            "dp_iid.hip")]
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), "-I", csrc] + srcs + [
           os.path.join(ROOT, "tests", "native", "abi_host_sanitize_main.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok"), r.stdout + r.stderr
