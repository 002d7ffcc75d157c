"""The host-only C++ of librte (validation, sphere pairing, P1 pattern, reverse Cuthill-McKee,
host band Cholesky, sliced-ELL layout, footprint prediction: csrc/host.cpp) built with g++ and
the address and undefined-behaviour sanitizers, and run on the realistic 2D mesh and a 3D mesh
(tests/sanitize/host_check.cpp states the checks).  Any sanitizer report or failed check fails
the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2102_09038_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2102_09038_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


def _write(dirname, name, inst):
    for key, arr, dt in (("vert", inst.vert, np.float64), ("cell", inst.cell, np.int32),
                         ("sigma_t", inst.sigma_t, np.float64), ("sigma_s", inst.sigma_s, np.float64),
                         ("svert", inst.svert, np.float64), ("stri", inst.stri, np.int32),
                         ("q", inst.q_nodal, np.float64)):
        np.ascontiguousarray(arr, dtype=dt).tofile(os.path.join(dirname, f"{name}.{key}"))


def test_host_code_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, "host.cpp"), os.path.join(ROOT, "tests", "sanitize", "host_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    _write(str(tmp_path), "grid2d", inputs.config_realistic())
    _write(str(tmp_path), "grid3d", inputs.make_instance("san-3d", 3, 8, 3, 0.8, 0.9, seed=5))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host_check ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
