"""Pins of the interpolated-transform oracle (App. A.2) and its derivative table (App. A.1).

* exactness where the spline is exact: y_lm with m even and l <= 3 is a
  polynomial of degree <= 3 in x, which a cubic Hermite spline reproduces, so
  those a_lm equal the direct sum on any node set;
* the derivative relation against central differences of the oracle's y_lm;
* the Hermite basis: values and slopes at both ends of an interval;
* convergence: the error falls like h^4 (x16 per halving) on a smooth band-limited case;
* the polar split: a cut that leaves every point polar reduces to the direct sum.
Planted mistakes in a copy of the module must fail at least one pin.
"""
import importlib.util
import math
import os

import numpy as np
import pytest

from paper_2312_12285_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "spline.py")


def _catalog(n=4000, seed=8):
    t, p = synth.uniform_sphere(n, seed)
    w = synth.lognormal_weights(n, 0.3, seed + 1)
    return t, p, w


def pin_polynomial_exactness(sp, ref):
    t, p, w = _catalog()
    lmax = 5
    a = sp.alm_spline(t, p, w, lmax, 6, math.radians(10))
    d = ref.alm_from_points(t, p, w, lmax)
    idx = lambda l, m: m * (2 * lmax + 1 - m) // 2 + l
    for l, m in ((0, 0), (1, 0), (2, 0), (3, 0), (2, 2), (3, 2)):
        if abs(a[idx(l, m)] - d[idx(l, m)]) > 1e-11 * max(1.0, abs(d[idx(l, m)])):
            return False
    # and not exact where it cannot be (l = 5): the check has teeth
    return abs(a[idx(5, 0)] - d[idx(5, 0)]) > 1e-8


def pin_derivative(sp, ref):
    lmax = 40
    th = np.array([0.3, 1.0, 1.9, 2.6])
    x = np.cos(th)
    y = sp.ylm_table(lmax, th)
    dy = sp.dylm_table(lmax, x, y)
    dx = 1e-6
    yp = sp.ylm_table(lmax, np.arccos(x + dx))
    ym = sp.ylm_table(lmax, np.arccos(x - dx))
    fd = (yp - ym) / (2 * dx)
    return np.abs(dy - fd).max() <= 1e-5 * np.abs(dy).max()


def pin_basis(sp, ref):
    c0, c1 = sp.hermite_basis(np.array([0.0, 1.0])).T
    e = 1e-7
    s0 = (sp.hermite_basis(np.array([e])) - sp.hermite_basis(np.array([0.0]))).ravel() / e
    s1 = (sp.hermite_basis(np.array([1.0])) - sp.hermite_basis(np.array([1.0 - e]))).ravel() / e
    ok = np.allclose(c0, [1, 0, 0, 0]) and np.allclose(c1, [0, 0, 1, 0])
    ok &= np.allclose(s0, [0, 1, 0, 0], atol=1e-6) and np.allclose(s1, [0, 0, 0, 1], atol=1e-6)
    return bool(ok)


def pin_convergence(sp, ref):
    t, p, w = _catalog(3000, 12)
    lmax = 16
    d = ref.alm_from_points(t, p, w, lmax)
    errs = [np.abs(sp.alm_spline(t, p, w, lmax, n, math.radians(8)) - d).max() for n in (48, 96)]
    return errs[0] / errs[1] > 11.0 and errs[1] < 1e-4 * np.abs(d).max()


def pin_polar_split(sp, ref):
    t, p, w = _catalog(2000, 14)
    lmax = 12
    a = sp.alm_spline(t, p, w, lmax, 4, math.pi / 2 - 1e-9)   # the spline band is empty
    d = ref.alm_from_points(t, p, w, lmax)
    return np.abs(a - d).max() <= 1e-13 * np.abs(d).max()


PINS = [pin_polynomial_exactness, pin_derivative, pin_basis, pin_convergence, pin_polar_split]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_spline_oracle_pin(oracle, pin):
    from oracle import spline
    assert pin(spline, oracle)


def _load_copy(tmp_path, old, new):
    text = open(SRC).read()
    assert old in text, old
    path = tmp_path / "spline_mutant.py"
    path.write_text(text.replace(old, new).replace("from . import ref", "from oracle import ref"))
    spec = importlib.util.spec_from_file_location("spline_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


MUTANTS = {
    "dx_dropped_on_derivatives": ("(vm[:, 1] * dx) @ dy[:-1, sl]", "vm[:, 1] @ dy[:-1, sl]"),
    "basis_c1_sign": ("t * (1 - t) ** 2,", "-t * (1 - t) ** 2,"),
    "basis_c2_wrong": ("t * t * (3 - 2 * t)", "t * t * (3 - t)"),
    "derivative_sign": ("(-l * x * yl + c * prev)", "(l * x * yl + c * prev)"),
    "derivative_norm_ratio": ("math.sqrt((2 * l + 1) / (2 * l - 1) * (l - m) * (l + m))",
                              "math.sqrt((l - m) * (l + m))"),
    "interval_off_by_one": ("j = np.floor(u).astype(np.int64)", "j = np.ceil(u).astype(np.int64)"),
    "phase_sign": ("e = ww * np.exp(-1j * m * ph)", "e = ww * np.exp(1j * m * ph)"),
    "polar_points_dropped": ("        out += ref.alm_from_points(th, ph, ww, lmax)", "        pass"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_spline_mistake_is_caught(oracle, tmp_path, name):
    sp = _load_copy(tmp_path, *MUTANTS[name])
    results = []
    for pin in PINS:
        try:
            results.append(bool(pin(sp, oracle)))
        except Exception:
            results.append(False)
    assert not all(results), f"planted mistake {name!r} passed every spline pin"


def test_entries_match_the_full_oracle(oracle):
    """The single-coefficient form used for full-size sampled checks equals the full form."""
    from oracle import spline
    t, p, w = _catalog(5000, 21)
    lmax, nn, cut = 20, 40, math.radians(7)
    full = spline.alm_spline(t, p, w, lmax, nn, cut)
    pairs = [(0, 0), (5, 0), (20, 3), (20, 20), (7, 6)]
    got = spline.alm_spline_entries(t, p, w, lmax, nn, cut, pairs)
    idx = [m * (2 * lmax + 1 - m) // 2 + l for l, m in pairs]
    assert np.abs(got - full[idx]).max() <= 1e-14 * np.abs(full[idx]).max()
