"""Host sanitizer build: the renderer's host-side checks and mesh tables
(paper_2303_10440_amd/csrc/dm_topo.cpp: grid and covariance validation, face
validation, closure and orientation, triangle strips, vertex incidence and
adjacency, density-weight closure), its sweep launch planning
(paper_2303_10440_amd/csrc/dm_plan.h: coverage, bounds, the shared launch's
tile floor) and the FP64 oracle's C routines, each
compiled alone with -fsanitize=address,undefined and run on its harness
(tests/sanitize/), which checks table invariants and closed forms on
closed, open, non-manifold, degenerate, random and out-of-range inputs.
CPU only; no GPU code is built here."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_10440_amd", "csrc")
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def _build_and_run(tmp_path, compiler, flags, sources, name):
    exe = str(tmp_path / name)
    b = _run([compiler] + flags + SAN + sources + ["-o", exe] + (["-lm"] if compiler == "gcc" else []))
    if b.returncode != 0 and "sanitize" in b.stderr and ("cannot find" in b.stderr or "unrecognized" in b.stderr):
        pytest.skip("sanitizer runtime not available: " + b.stderr[-300:])
    assert b.returncode == 0, b.stderr[-3000:]
    r = _run([exe], env=ENV)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout
    return r.stdout


def test_host_topology_and_validation_under_asan_ubsan(tmp_path):
    _need("g++")
    out = _build_and_run(tmp_path, "g++", ["-std=c++17", "-Wall", "-I" + CSRC],
                         [os.path.join(ROOT, "tests", "sanitize", "topo_harness.cpp"), os.path.join(CSRC, "dm_topo.cpp")],
                         "topo_harness")
    assert "topo harness" in out


def test_oracle_under_asan_ubsan(tmp_path):
    _need("gcc")
    out = _build_and_run(tmp_path, "gcc", ["-std=c11", "-fopenmp", "-Wall"],
                         [os.path.join(ROOT, "tests", "sanitize", "oracle_harness.c"),
                          os.path.join(ROOT, "oracle", "meshft_oracle.c")],
                         "oracle_harness")
    assert "oracle harness" in out
