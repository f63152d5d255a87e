"""The C ABI's host code under AddressSanitizer and UBSan, without a GPU:
sedimi_api.cpp and a driver (abi_sanitize_driver.cpp) are compiled with the
sanitizers on their host side only and linked with the library's kernel
objects; the driver runs every host-side path that needs no device
(parameter checks, workspace sizing, calls before a workspace, state-blob
guards, null handling)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1601_03801_amd")
KERNEL_OBJS = ["k_neighbors.o", "k_forces.o", "k_average.o", "k_nn.o", "k_spectral.o"]


def test_c_abi_host_paths_clean_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc is not available")
    objdir = os.path.join(PKG, "_build")
    if not all(os.path.exists(os.path.join(objdir, o)) for o in KERNEL_OBJS):
        from paper_1601_03801_amd import build
        build.build()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    common = ["-std=c++17", "-O1", "-g", "--offload-arch=gfx950", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")] + san
    objs = []
    for src in (os.path.join(PKG, "csrc", "sedimi_api.cpp"),
                os.path.join(ROOT, "tests", "abi_sanitize_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([hipcc, "-c", "-x", "hip", src, "-o", obj] + common,
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    exe = str(tmp_path / "abi_sanitized")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address",
                        "-Xarch_host", "-fsanitize=undefined"] + objs +
                       [os.path.join(objdir, o) for o in KERNEL_OBJS] + ["-o", exe],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    # leaks inside the HIP runtime are not this library's: leak checking off
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout, run.stderr[-2000:])
    assert run.returncode == 0, run.stderr[-3000:]
    assert run.stdout.strip().endswith("ok")
