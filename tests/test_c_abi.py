"""The boundary is plain C: a C99 program that includes only include/qgemm.h
compiles warning-free with gcc, links against libqgemm.so and gets the
documented status codes and argument indices (host validation, no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_1903_05575_amd")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_c_program_uses_the_abi(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "libqgemm.so")):
        pytest.skip("libqgemm.so not built")
    exe = str(tmp_path / "abi_check")
    rocm_lib = "/opt/rocm/lib"
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "c", "abi_check.c"), "-o", exe, f"-L{LIBDIR}", "-lqgemm",
           f"-Wl,-rpath,{LIBDIR}", f"-Wl,-rpath-link,{rocm_lib}", f"-Wl,-rpath,{rocm_lib}"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "FAIL" not in r.stdout
    assert r.stdout.count("ok ") == 14
