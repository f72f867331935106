"""The C ABI's host code (validation, work plans, workspace sizing, the server's
argument checks: csrc/api.hip and csrc/server.hip) built with AddressSanitizer and
UBSan on the host side and run on the CPU (tests/native/api_host_test.cpp).  Every
call there returns before any device work, so no GPU is needed; the device code is
compiled for gfx950 as usual and never launched."""
import concurrent.futures
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2312_12285_amd", "csrc")
INC = os.path.join(ROOT, "include")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def test_api_host_code_under_sanitizers(tmp_path):
    if shutil.which("hipcc") is None or shutil.which("g++") is None:
        pytest.skip("needs hipcc and g++")

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(["hipcc", "-c", "-std=c++17", "-O1", "-fPIC", "--offload-arch=gfx950", "-Xclang",
                        "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN, "-I", INC, "-I", CSRC, src,
                        "-o", obj], check=True, capture_output=True, text=True)
        return obj

    with concurrent.futures.ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(compile_one, sorted(glob.glob(os.path.join(CSRC, "*.hip")))))
    test_obj = str(tmp_path / "api_host_test.o")
    subprocess.run(["g++", "-std=c++17", "-O1", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-fno-sanitize-recover=all", "-I", INC, "-c",
                    os.path.join(ROOT, "tests", "native", "api_host_test.cpp"), "-o", test_obj], check=True)
    exe = str(tmp_path / "api_host_test")
    subprocess.run(["hipcc", "--offload-arch=gfx950", *HOST_SAN, test_obj, *objs, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout
