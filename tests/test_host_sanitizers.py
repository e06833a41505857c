"""The library's host setup (setup.cpp) built on its own with AddressSanitizer
and UndefinedBehaviorSanitizer (g++, host code only) and driven over meshes
with every option (orders, precisions, fluxes, mixed orders, SIP, PML,
dipoles, instances) and the mesh error paths: no sanitizer report, and the
decomposition invariants hold (tests/sanitize/host_driver.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_08733_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_setup_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(os.path.join(CSRC, "refops_gen.h")):
        from paper_2002_08733_amd import build
        build.generate()
    exe = str(tmp_path / "mdg_host_asan")
    subprocess.run(["g++", "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(CSRC, "setup.cpp"), os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
                    "-o", exe], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "cases clean" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
