"""Host sanitizer builds (CPU only): the oracle (serial and OpenMP timing
builds) under AddressSanitizer and UndefinedBehaviorSanitizer running a scene
with every wall kind, both contact models, both integrators and all rolling
options; the library's host code under the same sanitizers (device code built
normally) on the entry points' argument checks and error paths, the paths
that need no GPU.  A sanitizer report aborts the driver with a non-zero
exit status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")


def _run(exe, env_extra=None, timeout=300):
    env = dict(os.environ, **(env_extra or {}))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


@pytest.mark.parametrize("parallel", [False, True])
def test_oracle_under_address_and_ub_sanitizers(tmp_path, parallel):
    exe = str(tmp_path / "oracle_san")
    extra = ["-fopenmp", "-DORA_PARALLEL"] if parallel else []
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", *extra,
           "-I", os.path.join(ROOT, "oracle"), "-o", exe,
           os.path.join(SAN, "oracle_sanitize_main.c"), os.path.join(ROOT, "oracle", "oracle_dem.c"),
           "-lm"]
    subprocess.run(cmd, check=True, timeout=300)
    out = _run(exe, {"OMP_NUM_THREADS": "3"})
    assert "clean" in out


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_library_host_code_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "dem_san")
    C = os.path.join(ROOT, "paper_2106_09576_amd", "csrc")
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", C,
           "-o", exe, os.path.join(SAN, "dem_host_sanitize_main.cpp"),
           os.path.join(C, "dem_api.hip"), os.path.join(C, "dem_kernels.hip")]
    subprocess.run(cmd, check=True, timeout=600, capture_output=True)
    # the HIP runtime keeps allocations until exit: leaks are not checked
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=0"})
    assert "clean" in out
