"""The library's host code under AddressSanitizer and UndefinedBehavior-
Sanitizer (CPU only): libx2c is rebuilt with the sanitizers on its host
side (device code unchanged) and a C++ driver runs the ABI's host paths:
argument checks, the workspace layouts of uneven batches for every method,
the DKHn plans of every order and the status strings."""
import os
import subprocess

import pytest

from paper_1303_4446_amd import builder

HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.slow
def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(builder.hipcc()):
        pytest.skip("no hipcc")
    lib = builder.build(out=str(tmp_path / "libx2c_san.so"), build_dir=str(tmp_path / "obj"), extra=SAN)
    exe = str(tmp_path / "abi_driver")
    # the driver is plain host C++: the ROCm clang that hipcc drives, with
    # the same sanitizer runtime as the library's host code
    clang = os.path.join(os.path.dirname(os.path.realpath(builder.hipcc())), "..", "llvm", "bin", "clang++")
    cmd = [clang, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-I", os.path.join(builder.ROOT, "include"),
           os.path.join(HERE, "asan", "abi_driver.cpp"), lib, f"-Wl,-rpath,{tmp_path}", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "0 failure(s)" in r.stdout
