"""Host C++ of the library under AddressSanitizer (no GPU).

Compiles the library's host sources (set-up, C ABI, mesh, reference element,
operator packing) with -fsanitize=address, links them with the normally
built device objects into tests/asan_host_abi.cpp's driver, and runs it: the
host-side entry points and the validation paths of dg_create (all of its
host work, up to the workspace check) must pass with no memory error.
"""

import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1602_07997_amd")
CSRC = os.path.join(PKG, "csrc")


@pytest.mark.timeout(900)
def test_host_abi_under_asan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    from paper_1602_07997_amd import build_native as bn

    hip_objs = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        obj = os.path.join(bn.BUILD, os.path.basename(src) + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < os.path.getmtime(src):
            os.makedirs(bn.BUILD, exist_ok=True)
            obj = bn._compile(src)
        hip_objs.append(obj)
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address", "-D__HIP_PLATFORM_AMD__",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", "/opt/rocm/include"]
    objs = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))) + [os.path.join(ROOT, "tests", "asan_host_abi.cpp")]:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(["g++", *flags, "-c", src, "-o", obj], check=True)
        objs.append(obj)
    exe = str(tmp_path / "asan_host_abi")
    subprocess.run(["g++", "-fsanitize=address", *objs, *hip_objs, "-o", exe, "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "checks passed" in r.stdout
