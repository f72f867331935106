"""Host-side checks of the request server: its arena, memory admission (arrival
order, passing until aged) and work-item schedule (chunks of point slices,
shortest remaining work first, aged requests first; paper_2312_12285_amd/csrc/
server_core.h) under a simulated executor, compiled with g++ under AddressSanitizer
and UBSan and run on the CPU."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_server_core_simulation(tmp_path):
    exe = tmp_path / "server_core_test"
    src = os.path.join(ROOT, "tests", "native", "server_core_test.cpp")
    inc = os.path.join(ROOT, "paper_2312_12285_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror", "-fsanitize=address,undefined",
                    "-I", inc, src, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "OK" in r.stdout
    print(r.stdout)
