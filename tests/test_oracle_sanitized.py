"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code only):
every entry point on small, edge and extreme inputs (empty and one-point catalogs, exact
poles, lmax 0 and 16383, near-pole points at the top degree, the coupling matrix and its
rows), in a child process with the sanitizer runtimes preloaded.  Any out-of-bounds
access, use after free or undefined operation ends the child with an error."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = textwrap.dedent('''
    import sys, math
    sys.path.insert(0, ROOT)
    import numpy as np
    from oracle import ref
    from paper_2312_12285_amd.synth import uniform_sphere, shear_components, window_spectrum
    with ref.use_library(SO):
        for n, lmax in [(0, 5), (1, 0), (1, 1), (37, 17), (200, 64)]:
            t, p = uniform_sphere(n, 3)
            t[:min(n, 2)] = [0.0, math.pi][:min(n, 2)]
            w = np.ones(n)
            a = ref.alm_from_points(t, p, w, lmax, nthreads=2)
            b = ref.alm_from_points(t, p, w, lmax, nthreads=1, long_double=True)
            ref.alm_from_points(t, p, w, lmax, long_double=True, fp64_trig=True)
            ref.alm_entries(t, p, w, [0, lmax, lmax], [0, 0, lmax])
            ref.cl_from_alm(a, lmax)
            ref.cross_cl(a, b, lmax)
            g1, g2 = shear_components(n, 4)
            ref.spin_alm(t, p, w, g1, g2, lmax)
            ref.spin_entries(t, p, w, g1, g2, [max(2, lmax)], [0])
        t = np.array([1e-6, 3.0e-3, math.pi - 2e-5, 1.2])
        p = np.array([0.1, 2.0, 4.0, 5.5])
        w = np.array([1.0, 2.0, 0.5, 1.5])
        ref.alm_entries(t, p, w, [16383, 9000, 16383], [16383, 4000, 0])
        ref.spin_entries(t, p, w, w, w, [16383, 600], [16000, 2])
        W = window_spectrum(300, seed=5)
        ref.coupling_matrix(W, 120)
        ref.coupling_rows(W, 120, [0, 60, 120])
        for l in (0, 5, 100):
            ref.threej000(l, l + 2, 2)
    print("SANITIZED OK")
''')


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    libs = []
    for name in ("libasan.so", "libubsan.so"):
        path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
        if not os.path.isabs(path) or not os.path.exists(path):
            pytest.skip(f"{name} not available")
        libs.append(path)
    so = tmp_path / "libptalm_ref_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", "-o", str(so), os.path.join(ROOT, "oracle", "ptalm_ref.c"), "-lm"],
                   check=True)
    script = tmp_path / "run.py"
    script.write_text(f"ROOT = {ROOT!r}\nSO = {str(so)!r}\n" + SCRIPT)
    env = dict(os.environ, LD_PRELOAD=" ".join(libs), ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "SANITIZED OK" in r.stdout
