"""Host code under the address and undefined-behaviour sanitizers (CPU only).

Two programs are built with the host compiler and run:
  * tests/sanitize/host_checks.cpp with the library's host planning code
    (csrc/qieo_host.cpp: arena layout and the segment sums' sizing, segment
    numbering, the device pool's offset allocator with exhaustion, the
    batch's shape classes and tile tables, snapshot header checks, argument
    validation), checked against models and invariants;
  * tests/sanitize/oracle_checks.c with the CPU oracle's sources, built with
    the oracle's own floating-point flags, driving every entry point.
Any sanitizer report aborts the program (-fno-sanitize-recover), so a pass
means no memory error, leak or undefined behaviour on these paths.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


def _build_and_run(tmp_path, compiler, std, sources, extra, name):
    if shutil.which(compiler) is None:
        pytest.skip("%s not available" % compiler)
    exe = str(tmp_path / name)
    cmd = [compiler, std, *SAN, *extra, "-o", exe, *[os.path.join(ROOT, s) for s in sources]]
    r = subprocess.run(cmd + (["-lm"] if compiler == "gcc" else []), capture_output=True,
                       text=True)
    assert r.returncode == 0, "build failed:\n" + r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="abort_on_error=0:detect_leaks=1",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="3")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, "%s failed (%d):\n%s%s" % (name, r.returncode, r.stdout, r.stderr)
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
    return r.stdout


def test_host_planning_code_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "g++", "-std=c++17",
                         ["tests/sanitize/host_checks.cpp",
                          "paper_2609_30862_amd/csrc/qieo_host.cpp"],
                         ["-Wall", "-Wextra", "-Werror"], "host_checks")
    assert "host checks passed" in out


def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc", "-std=c11",
                         ["tests/sanitize/oracle_checks.c", "oracle/qieo_oracle.c",
                          "oracle/knapsack_exact.c"],
                         ["-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-Wall"],
                         "oracle_checks")
    assert "oracle checks passed" in out
