"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): api.hip, which holds the argument validation, the workspace and
batch layouts and the host-side operand packing of the handles, is compiled
with the sanitizers on its host pass only and linked with the library's other
objects into tests/sanitize/abi_driver.cpp, which drives those paths."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2107_11627_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
OTHERS = ["fields", "anchors", "mlp", "blur", "warp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# host pass only: each sanitizer flag directly after -Xarch_host
SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host", "-fno-sanitize-recover=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]


def test_host_code_is_clean_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    objs = [os.path.join(BUILD, f + ".o") for f in OTHERS]
    for f, o in zip(OTHERS, objs):
        if not os.path.exists(o) or os.path.getmtime(o) < os.path.getmtime(os.path.join(SRC, f + ".hip")):
            pytest.skip("build the library first (paper_2107_11627_amd/build.py): its objects are linked here")
    common = ["--offload-arch=gfx950", "-O1", "-g", "-fPIC", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", SRC]
    api = str(tmp_path / "api.o")
    drv = str(tmp_path / "drv.o")
    exe = str(tmp_path / "abi_driver")
    for cmd in ([HIPCC] + common + SAN + ["-c", os.path.join(SRC, "api.hip"), "-o", api],
                [HIPCC, "-O1", "-g", "-std=c++17", "-I", os.path.join(ROOT, "include")] + SAN +
                ["-c", os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp"), "-o", drv],
                [HIPCC, "--offload-arch=gfx950"] + SAN[:2] + ["-o", exe, drv, api] + objs):
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    report = r.stdout + r.stderr
    assert "AddressSanitizer" not in report and "runtime error" not in report, report
    assert r.returncode == 0, report
    assert "all host-side checks passed" in r.stdout
