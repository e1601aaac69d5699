"""Host tests of the kernels' integer index arithmetic, built with the address
and undefined-behaviour sanitizers:
- csrc/lbm_index.hpp (tests/index_check.cpp): the XCD-aware block order is a
  permutation of every launch size, and the magic-number division by a lattice
  extent is exact for every extent up to 1290 and every dividend below 2^31;
- csrc/lbm_tb2_plan.hpp (tests/tb2_plan_check.cpp): the two-step kernel's work
  plan covers every (tile, plane) unit exactly once for every shape tried."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_index_arithmetic_sanitized(tmp_path):
    exe = str(tmp_path / "index_check")
    # the sanitizers apply to the host code only (the file has no kernels)
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "paper_2512_23116_amd", "csrc"),
           os.path.join(ROOT, "tests", "index_check.cpp"), "-o", exe]
    subprocess.check_call(cmd)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("ok:")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_two_step_work_plan_sanitized(tmp_path):
    exe = str(tmp_path / "tb2_plan_check")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "paper_2512_23116_amd", "csrc"),
           os.path.join(ROOT, "tests", "tb2_plan_check.cpp"), "-o", exe]
    subprocess.check_call(cmd)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("ok:")
