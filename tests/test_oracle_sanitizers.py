"""The oracle's C code under the host AddressSanitizer and
UndefinedBehaviorSanitizer: a driver calls every oracle entry point on a
small seeded bed (pairs, forces with every component, a run with averaging,
deposition and flux, both pseudo-time schemes, the solid velocity, the
network routines) in a build with both sanitizers, halting on the first
report.  CPU only; the GPU library is not involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
SOURCES = ["orc_pairs.c", "orc_forces.c", "orc_average.c", "orc_cnn.c", "orc_mesh.c"]


def test_oracle_clean_under_address_and_undefined_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc is not available")
    exe = str(tmp_path / "oracle_sanitized")
    cmd = [gcc, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", ORACLE,
           *[os.path.join(ORACLE, s) for s in SOURCES],
           os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"), "-lm", "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if build.returncode != 0 and "sanitize" in build.stderr and "unrecognized" in build.stderr:
        pytest.skip("this gcc has no sanitizer support")
    assert build.returncode == 0, build.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(run.stdout)
    assert run.returncode == 0, run.stderr[-3000:]
    assert run.stdout.startswith("ok ")
