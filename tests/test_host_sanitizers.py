"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): runtime.cpp and the checks in tests/sanitize/abi_host_check.cpp are
compiled with g++ -fsanitize=address,undefined and linked with the device
objects of the normal build; the checks exercise argument and material
validation, the options defaults, the footprint, the allocation-free
product's limits and, without a GPU, the clean-up of a plan whose first HIP
call fails.  Any sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1601_05970_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_1601_05970_amd", "_build")
ROCM = "/opt/rocm"


def _need(path):
    if not os.path.exists(path):
        pytest.skip(f"{path} missing (run the library build first)")


def test_host_runtime_under_asan_and_ubsan(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    objs = [os.path.join(BUILD, "kernels.o"), os.path.join(BUILD, "noalloc.o")]
    for o in objs:
        _need(o)
    _need(os.path.join(ROCM, "lib", "libamdhip64.so"))
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
    inc = ["-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", f"-I{ROOT}/include", f"-I{CSRC}"]
    run = lambda cmd: subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=600)
    rt = str(tmp_path / "runtime_san.o")
    ck = str(tmp_path / "check.o")
    exe = str(tmp_path / "abi_host_check")
    r = run(["g++", "-std=c++17", "-O1", "-g", "-w"] + san + inc + ["-c", os.path.join(CSRC, "runtime.cpp"), "-o", rt])
    assert r.returncode == 0, r.stdout[-3000:]
    r = run(["g++", "-std=c++17", "-O1", "-g"] + san + inc +
            ["-c", os.path.join(ROOT, "tests", "sanitize", "abi_host_check.cpp"), "-o", ck])
    assert r.returncode == 0, r.stdout[-3000:]
    r = run(["g++"] + san + [ck, rt] + objs + [f"-L{ROCM}/lib", f"-Wl,-rpath,{ROCM}/lib", "-lamdhip64", "-o", exe])
    assert r.returncode == 0, r.stdout[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-5000:]
    assert "0 failed" in r.stdout
    assert "runtime error" not in r.stdout and "AddressSanitizer" not in r.stdout, r.stdout[-5000:]
