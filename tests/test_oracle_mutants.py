"""Plants one plausible mistake at a time in a copy of the oracle source, builds
that copy, and requires at least one pin to catch it.  This shows the pins are
strong enough to guard the oracle: a dropped term, a wrong sign, a wrong
coefficient, index or normalisation each fail a check.  Everything runs on the
CPU; the real oracle is never modified.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import pins
from oracle import ref

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")

MUTANTS = {
    "drop_condon_shortley_sign": ("    if (m & 1) f = -f;\n    if (e > -900)", "    if (e > -900)"),
    "recurrence_A_wrong": ("A[l - m] = outer * ((2.0 * l - 1.0) / lm);", "A[l - m] = outer * ((2.0 * l + 1.0) / lm);"),
    "recurrence_B_sign": ("else v = A[j] * x * prev1 - B[j] * prev2;", "else v = A[j] * x * prev1 + B[j] * prev2;"),
    "recurrence_B_dropped": ("else v = A[j] * x * prev1 - B[j] * prev2;", "else v = A[j] * x * prev1;"),
    "second_step_wrong": ("const double a1 = sqrt(2.0 * m + 1.0);", "const double a1 = sqrt(2.0 * m);"),
    "sectoral_constant_wrong": ("c[m] = c[m - 1] * sqrt(1.0 - 1.0 / (2.0 * m));", "c[m] = c[m - 1] * sqrt(1.0 - 1.0 / (2.0 * m + 1.0));"),
    "phase_not_conjugated": ("long double wi = -(long double)w[i] * sinl(ang);\n            pbar_column(",
                             "long double wi = (long double)w[i] * sinl(ang);\n            pbar_column("),
    "normalisation_2pi": ("""            long double norm = sqrtl((2.0L * l + 1.0L) / (4.0L * PI_L));
            int64_t k = hp_index(lmax, l, m);
            alm[2 * k] = (double)(norm * acc[2 * j]);
            alm[2 * k + 1] = (m == 0) ? 0.0 : (double)(norm * acc[2 * j + 1]);
        }
        free(A); free(B); free(p); free(acc);
    }
    free(c); free(xs); free(ss);""", """            long double norm = sqrtl((2.0L * l + 1.0L) / (2.0L * PI_L));
            int64_t k = hp_index(lmax, l, m);
            alm[2 * k] = (double)(norm * acc[2 * j]);
            alm[2 * k + 1] = (m == 0) ? 0.0 : (double)(norm * acc[2 * j + 1]);
        }
        free(A); free(B); free(p); free(acc);
    }
    free(c); free(xs); free(ss);"""),
    "healpy_index_off": ("return (int64_t)m * (2 * lmax + 1 - m) / 2 + l;", "return (int64_t)m * (2 * lmax - m) / 2 + l;"),
    "cl_missing_negative_m": ("            s += (m == 0) ? sq : 2.0L * sq;", "            s += sq;"),
    "cross_imag_sign": ("long double re = (long double)alm1[2 * k] * alm2[2 * k] + (long double)alm1[2 * k + 1] * alm2[2 * k + 1];",
                        "long double re = (long double)alm1[2 * k] * alm2[2 * k] - (long double)alm1[2 * k + 1] * alm2[2 * k + 1];"),
    "rescale_forgets_previous": ("                v *= 0x1p-600;\n                prev1 *= 0x1p-600;", "                v *= 0x1p-600;"),
    "exponent_conversion_forgets_previous": ("                prev1 = ldexp(prev1, (int)e);\n                e = 0;", "                e = 0;"),
    "cos_for_sin": ("xs[i] = cos(theta[i]); ss[i] = sin(theta[i]);", "xs[i] = cos(theta[i]); ss[i] = cos(theta[i]);"),
}


def run_pins():
    """The pin battery, with the tolerances of test_oracle_pins; True if all pass."""
    fn = lambda th, ph, w, lmax: ref.alm_from_points(th, ph, w, lmax)
    eps = 2.0 ** -53
    checks = [
        pins.pin_closed_forms(fn) < 1e-15,
        pins.pin_scipy(fn, lmax=40) < 1e-13,
        pins.pin_special_values(fn, lmax=64) < 1e-13,
        pins.pin_addition_theorem(fn, 1024, [0.4, 1.0, 2.2]) < 1e-12,
        pins.pin_pair_sum(fn, ref.cl_from_alm, ref.cross_cl, lmax=32, nA=60, nB=50) < 1e-11,
        pins.pin_monopole_dipole(fn) < 1e-12,
    ]
    # near-pole exponent path: FP64 variant against the long-double variant
    lmax = 2048
    th = np.array([2e-4, 3e-3, math.pi - 1e-3])
    ph = np.array([0.3, 2.0, 4.0])
    w = np.ones(3)
    a = ref.alm_from_points(th, ph, w, lmax)
    b = ref.alm_from_points(th, ph, w, lmax, long_double=True, fp64_trig=True)
    from conftest import per_l_rel_err
    checks.append(per_l_rel_err(a, b, lmax).max() < 200 * lmax * eps)
    return all(checks)


def test_real_oracle_passes_battery():
    assert run_pins()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(os.path.join(ORACLE_DIR, "ptalm_ref.c")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique in the oracle source"
    shutil.copy(os.path.join(ORACLE_DIR, "ptalm_ref.h"), tmp_path / "ptalm_ref.h")
    (tmp_path / "ptalm_ref.c").write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(so),
                    str(tmp_path / "ptalm_ref.c"), "-lm"], check=True)
    with ref.use_library(str(so)):
        assert not run_pins(), f"planted mistake {name!r} passed every pin"


COUPLING_MUTANTS = {
    "threej_sign_lost": ("return (double)((h & 1) ? -v : v);", "return (double)v;"),
    "threej_factorial_wrong": ("- lfact(L + 1))", "- lfact(L))"),
    "coupling_lambda_weight_dropped": ("sum += (2.0L * lam + 1.0L) * t * t * (long double)Wl[lam];",
                                       "sum += t * t * (long double)Wl[lam];"),
    "coupling_wrong_degree_factor": ("(double)((2.0L * lp + 1.0L) * inv4pi * sum)", "(double)((2.0L * l + 1.0L) * inv4pi * sum)"),
    "coupling_lambda_range_short": ("const int hi = l + lp < lmax_w ? l + lp : lmax_w;",
                                    "const int hi = l + lp < lmax_w ? l + lp : lmax_w - 1;"),
    "coupling_first_lambda_dropped": ("for (int lam = lo; lam <= hi; lam += 2) {",
                                      "for (int lam = lo + 2; lam <= hi; lam += 2) {"),
    "coupling_window_index_shifted": ("sum += (2.0L * lam + 1.0L) * t * t * (long double)Wl[lam];",
                                      "sum += (2.0L * lam + 1.0L) * t * t * (long double)Wl[lam > 0 ? lam - 1 : 0];"),
    "coupling_two_pi": ("const long double inv4pi = 1.0L / (4.0L * 3.14159265358979323846264338327950288L);",
                        "const long double inv4pi = 1.0L / (2.0L * 3.14159265358979323846264338327950288L);"),
    "threej_factorial_index": ("lfact(h) - lfact(h - l1) - lfact(h - l2) - lfact(h - l3);",
                               "lfact(h) - lfact(h - l1) - lfact(h - l1) - lfact(h - l3);"),
}


def run_coupling_pins():
    """The coupling pin battery of test_oracle_coupling; True if all pass."""
    import test_oracle_coupling as t
    checks = [t.test_threej_textbook_values, t.test_threej_paper_terminal_and_recurrence,
              t.test_threej_gaunt_integral_quadrature, t.test_threej_orthogonality,
              t.test_coupling_full_sky_is_identity, t.test_coupling_row_sums_shot_noise_bracket,
              t.test_coupling_equals_its_definition_by_quadrature]
    for c in checks:
        try:
            c(ref)
        except AssertionError:
            return False
    return True


def test_real_oracle_passes_coupling_battery():
    assert run_coupling_pins()


@pytest.mark.parametrize("name", sorted(COUPLING_MUTANTS))
def test_planted_coupling_mistake_is_caught(name, tmp_path):
    old, new = COUPLING_MUTANTS[name]
    src = open(os.path.join(ORACLE_DIR, "ptalm_ref.c")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique in the oracle source"
    shutil.copy(os.path.join(ORACLE_DIR, "ptalm_ref.h"), tmp_path / "ptalm_ref.h")
    (tmp_path / "ptalm_ref.c").write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(so),
                    str(tmp_path / "ptalm_ref.c"), "-lm"], check=True)
    with ref.use_library(str(so)):
        assert not run_coupling_pins(), f"planted mistake {name!r} passed every coupling pin"


# Planted mistakes in the oracle's bandpower algebra (plain numpy): each replaces one
# statement of a function of oracle/ref.py for the duration of the test.
BANDPOWER_MUTANTS = {
    "coupled_bins_averaged_twice": ("decoupled_bandpowers", "Mbb = theta @ M @ chi", "Mbb = theta @ M @ theta.T"),
    "bandpowers_not_decoupled": ("decoupled_bandpowers", "cb = np.linalg.solve(Mbb, theta @ np.asarray(cl_hat))",
                                 "cb = theta @ np.asarray(cl_hat)"),
    "window_not_decoupled": ("decoupled_bandpowers", "window = np.linalg.solve(Mbb, theta @ M)", "window = theta @ M"),
    "normalisation_two_pi": ("normalized_bandpowers", "(2 * lam + 1) / (4 * np.pi) * Wl", "(2 * lam + 1) / (2 * np.pi) * Wl"),
    "normalisation_weight": ("normalized_bandpowers", "(2 * lam + 1) / (4 * np.pi) * Wl", "(2 * lam) / (4 * np.pi) * Wl"),
    "bin_weight_not_averaged": ("bin_matrix", "theta[b, lo:lo + delta_l] = 1.0 / delta_l", "theta[b, lo:lo + delta_l] = 1.0"),
    "bin_one_short": ("bin_matrix", "theta[b, lo:lo + delta_l] = 1.0 / delta_l",
                      "theta[b, lo:lo + delta_l - 1] = 1.0 / delta_l"),
}


@pytest.mark.parametrize("name", sorted(BANDPOWER_MUTANTS))
def test_planted_bandpower_mistake_is_caught(name, monkeypatch):
    import inspect
    import test_oracle_coupling as t
    fn, old, new = BANDPOWER_MUTANTS[name]
    src = inspect.getsource(getattr(ref, fn))
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    ns = dict(ref.__dict__)
    exec(src.replace(old, new), ns)
    monkeypatch.setattr(ref, fn, ns[fn])
    with pytest.raises(AssertionError):
        t.test_bandpowers_recover_piecewise_constant_and_shot_noise(ref)


def test_real_oracle_passes_bandpower_pin():
    import test_oracle_coupling as t
    t.test_bandpowers_recover_piecewise_constant_and_shot_noise(ref)
