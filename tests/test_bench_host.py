"""bench.py's host-side contract, without a GPU: more than one GPU is
refused with a message, the averaging rooflines count what the docstring
states, and the stored force-kernel counters name their sources and
profile."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_averaging_roofline_bytes_and_flops():
    n, ncell, mesh = 1000, 64, (4, 4, 4)
    dep, sol = bench.averaging_rooflines(n, ncell, 1.0, 1.0, True, mesh)
    assert dep["bytes"] == 60 * n + 32 * ncell
    # the solve against its algorithmic minimum (read raw, write smooth)
    assert sol["bound"] == "hbm" and sol["bytes"] == 16 * ncell * 4
    assert sol["frac"] == round(16 * ncell * 4 / 1e-3 / 1e9 / bench.HBM_PEAK_GBS, 4)
    assert sol["transforms"]["gflop"] == round(4 * 12 * ncell * 4 / 1e9, 3)
    dep7, sol7 = bench.averaging_rooflines(n, ncell, 1.0, 1.0, True, mesh, nch=7)
    assert dep7["bytes"] == 84 * n + 56 * ncell
    assert sol7["transforms"]["gflop"] == round(4 * 12 * ncell * 7 / 1e9, 3)
    _, it = bench.averaging_rooflines(n, ncell, 1.0, 1.0, False, mesh)
    assert "transforms" not in it and it["bound"] == "hbm"
    big = 10 ** 8  # large enough for the rounded HBM minimum
    _, s4 = bench.averaging_rooflines(n, big, 1.0, 1.0, True, mesh)
    _, s7 = bench.averaging_rooflines(n, big, 1.0, 1.0, True, mesh, nch=7)
    assert s4["hbm_minimum_ms"] == round(16 * big * 4 / bench.HBM_PEAK_GBS / 1e6, 5)
    assert s7["hbm_minimum_ms"] == round(16 * big * 7 / bench.HBM_PEAK_GBS / 1e6, 5)


def test_stored_force_counters_name_their_sources_and_profile():
    """The HBM traffic in the bench line is reported only while the hash of
    the force kernel's sources equals the one the counters were taken on
    (otherwise it is null); the counters' profile summary is committed."""
    assert bench.FORCE_PMC
    assert len(bench.force_sources_sha()) == 64
    for (workload, precision), pmc in bench.FORCE_PMC.items():
        assert workload in ("bed1m", "bed10m") and precision in ("fp64", "mixed")
        assert len(pmc["sources_sha256"]) == 64
        assert os.path.exists(os.path.join(ROOT, pmc["profile"]))


def test_rebuild_bytes_count_what_the_docstring_states():
    b = bench.rebuild_bytes_per_particle(8.0, 4.0, False)
    assert b == 40 + 12 + 520 + 72 + 32 + 4 * (48 + 56)
    assert bench.rebuild_bytes_per_particle(8.0, 4.0, True) == b - 4 * 24
