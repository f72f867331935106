"""Pins of the spin-weighted oracle (spin +-2 harmonics for shear, end of Sec. 4).

Each pin ties the oracle to something outside itself:
* Goldberg et al.'s explicit sum for sY_lm (a different formula from the Wigner-d
  recurrence the oracle's transform runs);
* the definition through the spin-raising operator: _1Y_lm and _2Y_lm from
  finite differences of scipy's scalar Y_lm (fixes the sign convention);
* the spin addition theorem sum_m |sY_lm|^2 = (2l+1)/4pi at every point and every
  l up to 600, near the poles included (m < 0 through _{-s}Y_lm);
* orthonormality under Gauss-Legendre x uniform-phi quadrature;
* the parity relation _{-s}lambda_lm(pi - theta) = (-1)^(l+m) _s lambda_lm(theta);
* E/B: a shear field built as the second spin-raising derivative of a real
  potential psi (finite differences again) has a^B = 0 and
  a^E = -sqrt((l+2)!/(l-2)!) psi_lm; its rotation by 45 degrees swaps E and B;
* spin 0 reduces to the scalar oracle.
Planted mistakes in a copy of the module must fail at least one pin.
"""
import importlib.util
import math
import os

import numpy as np
import pytest
from scipy.special import sph_harm_y

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "spin.py")


def _points(n, seed):
    rng = np.random.default_rng(seed)
    th = np.arccos(rng.uniform(-1, 1, n))
    th[:4] = [1e-3, 2e-6, math.pi - 1e-4, math.pi / 2]   # near the poles and on the equator
    return th, rng.uniform(0, 2 * math.pi, n)


def _quadrature(lmax):
    """Gauss-Legendre in cos(theta) x uniform phi, exact for band limit 2 lmax."""
    nx, nphi = lmax + 2, 2 * lmax + 3
    x, wx = np.polynomial.legendre.leggauss(nx)
    ph = 2 * math.pi * np.arange(nphi) / nphi
    T, P = np.meshgrid(np.arccos(x), ph, indexing="ij")
    W = np.repeat(wx[:, None] * (2 * math.pi / nphi), nphi, axis=1)
    return T.ravel(), P.ravel(), W.ravel()


def _ylm(l, m, th, ph):
    """scipy's scalar Y_lm (Condon-Shortley phase), any sign of m."""
    return sph_harm_y(l, m, th, ph)


def _eth_fd(l, m, th, ph, spin_to):
    """_1Y_lm or _2Y_lm from the spin-raising operator applied to scipy's Y_lm by
    central differences in theta (phi derivatives are exact: i m)."""
    h = 1e-4
    f = lambda t: _ylm(l, m, t, ph)
    d1 = (f(th - 2 * h) - 8 * f(th - h) + 8 * f(th + h) - f(th + 2 * h)) / (12 * h)
    s, c = np.sin(th), np.cos(th)
    y = f(th)
    if spin_to == 1:
        return -(d1 - m / s * y) / math.sqrt(l * (l + 1))
    d2 = (-f(th - 2 * h) + 16 * f(th - h) - 30 * y + 16 * f(th + h) - f(th + 2 * h)) / (12 * h * h)
    eth2 = d2 - c / s * d1 + (m * m / s ** 2) * y - 2 * m / s * (d1 - c / s * y)
    return eth2 / math.sqrt((l - 1) * l * (l + 1) * (l + 2))


def _lam_all(sp, s, lmax, th):
    """lambda[m][l, point] for m = 0..lmax."""
    return [sp.spin_lambda(s, m, lmax, th) for m in range(lmax + 1)]


def pin_goldberg(sp, ref):
    th, ph = _points(40, 1)
    th = th[4:]
    err = 0.0
    for s in (-2, -1, 1, 2):
        for m in range(0, 9):
            lam = sp.spin_lambda(s, m, 10, th)
            for l in range(0, 11):
                g = sp.goldberg(s, l, m, th, 0 * th).real
                err = max(err, np.abs(lam[l] - g).max())
    return err < 1e-12


def pin_eth_definition(sp, ref):
    th = np.array([0.4, 1.1, 1.7, 2.5])
    ph = np.array([0.3, 2.0, 4.1, 5.5])
    err = 0.0
    for s in (1, 2):
        for l in range(s, 7):
            for m in range(0, l + 1):
                lam = sp.spin_lambda(s, m, l, th)[l]
                got = lam * np.exp(1j * m * ph)
                err = max(err, np.abs(got - _eth_fd(l, m, th, ph, s)).max())
    return err < 1e-6


def pin_addition_theorem(sp, ref):
    lmax = 600
    th, _ = _points(6, 2)
    tot = np.zeros((lmax + 1, th.size))
    for m in range(lmax + 1):
        a = sp.spin_lambda(2, m, lmax, th)
        b = sp.spin_lambda(-2, m, lmax, th)
        tot += a * a + (b * b if m > 0 else 0.0)
    l = np.arange(lmax + 1)
    want = np.where(l >= 2, (2 * l + 1) / (4 * math.pi), 0.0)
    return np.abs(tot - want[:, None]).max() < 1e-10 * want.max()


def pin_orthonormality(sp, ref):
    lmax = 10
    T, P, W = _quadrature(lmax)
    for s in (2, -2):
        for (lp, mp) in ((2, 0), (5, 3), (10, 10), (7, 1)):
            f = sp.goldberg(s, lp, mp, T, P)
            a = sp.spin_alm(s, T, P, W, f, lmax)
            want = np.zeros_like(a)
            want[mp * (2 * lmax + 1 - mp) // 2 + lp] = 1.0
            if np.abs(a - want).max() > 1e-11:
                return False
    return True


def pin_parity(sp, ref):
    th, _ = _points(30, 3)
    lmax = 40
    for m in (0, 1, 2, 7, 33):
        a = sp.spin_lambda(-2, m, lmax, math.pi - th)
        b = sp.spin_lambda(2, m, lmax, th)
        sign = (-1.0) ** (np.arange(lmax + 1) + m)
        if np.abs(a - sign[:, None] * b).max() > 1e-11 * max(1.0, np.abs(b).max()):
            return False
    return True


def _psi_field(lmax, T, P, seed):
    """A real band-limited potential psi = sum psi_lm Y_lm (m < 0 by reality) and its
    coefficients (healpy order, m >= 0); zero for l < 2."""
    rng = np.random.default_rng(seed)
    nT = (lmax + 1) * (lmax + 2) // 2
    psi = np.zeros(nT, complex)
    for m in range(lmax + 1):
        for l in range(max(m, 2), lmax + 1):
            v = rng.normal() + (1j * rng.normal() if m else 0.0)
            psi[m * (2 * lmax + 1 - m) // 2 + l] = v
    return psi


def _eth2_of(psi, lmax, T, P):
    """eth^2 psi at the points by finite differences of the scalar field."""
    out = np.zeros(T.size, complex)
    for m in range(lmax + 1):
        for l in range(max(m, 2), lmax + 1):
            c = psi[m * (2 * lmax + 1 - m) // 2 + l]
            N = math.sqrt((l - 1) * l * (l + 1) * (l + 2))
            out += c * N * _eth_fd(l, m, T, P, 2)
            if m > 0:   # psi_{l,-m} = (-1)^m conj(psi_lm)
                out += (-1) ** m * np.conj(c) * N * _eth_fd(l, -m, T, P, 2)
    return out


def pin_eb(sp, ref):
    lmax = 6
    T, P, W = _quadrature(lmax)
    psi = _psi_field(lmax, T, P, 4)
    g = _eth2_of(psi, lmax, T, P)                 # pure-E shear field gamma = eth^2 psi
    E, B = sp.shear_eb(T, P, W, g.real, g.imag, lmax)
    l = np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])
    N = np.sqrt(np.where(l >= 2, (l - 1.0) * l * (l + 1) * (l + 2), 0.0))
    ok = np.abs(E + N * psi).max() < 1e-5 * np.abs(N * psi).max() and np.abs(B).max() < 1e-5 * np.abs(N * psi).max()
    E2, B2 = sp.shear_eb(T, P, W, -g.imag, g.real, lmax)    # gamma -> i gamma: E -> B
    ok &= np.abs(B2 + N * psi).max() < 1e-5 * np.abs(N * psi).max() and np.abs(E2).max() < 1e-5 * np.abs(N * psi).max()
    return bool(ok)


def pin_spin0_is_scalar(sp, ref):
    th, ph = _points(300, 5)
    w = np.random.default_rng(6).lognormal(0, 0.3, th.size)
    a = sp.spin_alm(0, th, ph, w, np.ones(th.size), 30)
    d = ref.alm_from_points(th, ph, w, 30)
    return np.abs(a - d).max() < 1e-12 * np.abs(d).max()


PINS = [pin_goldberg, pin_eth_definition, pin_addition_theorem, pin_orthonormality, pin_parity, pin_eb,
        pin_spin0_is_scalar]


@pytest.mark.parametrize("pin", PINS, ids=lambda f: f.__name__)
def test_spin_oracle_pin(oracle, pin):
    from oracle import spin
    assert pin(spin, oracle)


def _load_copy(tmp_path, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, old
    path = tmp_path / "spin_mutant.py"
    path.write_text(text.replace(old, new))
    spec = importlib.util.spec_from_file_location("spin_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


MUTANTS = {
    "recurrence_mmp_sign": ("(l * (l + 1) * x - m * mp)", "(l * (l + 1) * x + m * mp)"),
    "recurrence_lag_dropped": ("* d - c * d_prev) / a", "* d) / a"),
    "recurrence_lag_factor": ("c = (l + 1) * math.sqrt", "c = l * math.sqrt"),
    "spin_sign_convention": ("    mp = -s\n    l0", "    mp = s\n    l0"),
    "normalisation_2pi": ("norm = (-1.0) ** m * np.sqrt((2 * ls + 1) / (4 * math.pi))",
                          "norm = (-1.0) ** m * np.sqrt((2 * ls + 1) / (2 * math.pi))"),
    "condon_shortley_dropped": ("norm = (-1.0) ** m * np.sqrt", "norm = np.sqrt"),
    "phase_not_conjugated": ("z = q * np.exp(-1j * m * phi)", "z = q * np.exp(1j * m * phi)"),
    "seed_half_angle_swap": ("c, s = np.cos(beta / 2), np.sin(beta / 2)", "s, c = np.cos(beta / 2), np.sin(beta / 2)"),
    "eb_sign": ("return -(a2 + am2) / 2, 1j * (a2 - am2) / 2", "return (a2 + am2) / 2, 1j * (a2 - am2) / 2"),
    "shear_not_conjugated_for_minus2": ("am2 = spin_alm(-2, theta, phi, w, np.conj(gp), lmax)",
                                        "am2 = spin_alm(-2, theta, phi, w, gp, lmax)"),
    "seed_l0_wrong": ("l0 = max(abs(m), abs(mp))", "l0 = max(abs(m), abs(mp), 1)"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_spin_mistake_is_caught(oracle, tmp_path, name):
    sp = _load_copy(tmp_path, *MUTANTS[name])
    for pin in PINS:
        try:
            if not pin(sp, oracle):
                return
        except Exception:
            return
    pytest.fail(f"planted mistake {name!r} passed every spin pin")


# ---------------------------------------------------------------------------
# The C form of the spin oracle (selected coefficients over every point, used for
# sampled checks at full size), pinned against the Python oracle above and against
# the spin addition theorem at l = 3072.
# ---------------------------------------------------------------------------
def c_pin_matches_python(ref):
    from oracle import spin
    rng = np.random.default_rng(5)
    n, lmax = 2000, 48
    t = np.arccos(rng.uniform(-1, 1, n))
    t[:4] = [0.0, math.pi, 1e-5, math.pi - 1e-6]
    p = rng.uniform(0, 2 * math.pi, n)
    w = rng.lognormal(0, 0.3, n)
    g1, g2 = rng.normal(0, 0.26, n), rng.normal(0, 0.26, n)
    G = g1 + 1j * g2
    a2 = spin.spin_alm(2, t, p, w, G, lmax)
    am2 = spin.spin_alm(-2, t, p, w, np.conj(G), lmax)
    pairs = [(l, m) for m in range(lmax + 1) for l in range(max(m, 2), lmax + 1)]
    idx = [m * (2 * lmax + 1 - m) // 2 + l for l, m in pairs]
    e2, em2 = ref.spin_entries(t, p, w, g1, g2, [l for l, _ in pairs], [m for _, m in pairs])
    return (np.abs(e2 - a2[idx]).max() <= 1e-12 * np.abs(a2).max()
            and np.abs(em2 - am2[idx]).max() <= 1e-12 * np.abs(am2).max())


def c_pin_addition_theorem(ref):
    """sum_{m>=0} |_2Y_lm|^2 + sum_{m>0} |_-2Y_lm|^2 = (2l+1)/4pi at l = 3072 (one point,
    unit weight, g = 1).  Near the poles the FP64 value of cos(theta) fixes theta only to
    ~eps/theta, which moves the sum by up to ~(l theta)^2 eps / theta^2: 2e-9 there, 1e-11
    elsewhere."""
    L = 3072
    for th, tol in ((0.3, 1e-11), (1.7, 1e-11), (2.9, 1e-11), (1e-4, 2e-9), (math.pi - 1e-3, 2e-9)):
        one = np.ones(1)
        e2, em2 = ref.spin_entries(np.array([th]), np.array([0.7]), one, one, 0 * one,
                                   np.full(L + 1, L), np.arange(L + 1))
        tot = np.sum(np.abs(e2) ** 2) + np.sum(np.abs(em2[1:]) ** 2)
        if abs(tot / ((2 * L + 1) / (4 * math.pi)) - 1) > tol:
            return False
    return True


def c_pin_full_matches_python(ref):
    from oracle import spin
    rng = np.random.default_rng(9)
    n, lmax = 1500, 40
    t = np.arccos(rng.uniform(-1, 1, n))
    t[:2] = [2e-6, math.pi - 3e-5]
    p = rng.uniform(0, 2 * math.pi, n)
    w = rng.lognormal(0, 0.3, n)
    g1, g2 = rng.normal(0, 0.26, n), rng.normal(0, 0.26, n)
    E, B = spin.shear_eb(t, p, w, g1, g2, lmax)
    Ec, Bc = ref.shear_eb(t, p, w, g1, g2, lmax)
    return np.abs(Ec - E).max() <= 1e-12 * np.abs(E).max() and np.abs(Bc - B).max() <= 1e-12 * np.abs(B).max()


C_PINS = [c_pin_matches_python, c_pin_addition_theorem, c_pin_full_matches_python]


@pytest.mark.parametrize("pin", C_PINS, ids=lambda f: f.__name__)
def test_spin_c_oracle_pin(oracle, pin):
    assert pin(oracle)


C_MUTANTS = {
    "c_recurrence_mmp_sign": ("B[l] = (2.0 * l + 1.0) * dm * dp / D;", "B[l] = -(2.0 * l + 1.0) * dm * dp / D;"),
    "c_lag_factor": ("C[l] = l1 * sqrt((dl * dl - dm * dm) * (dl * dl - dp * dp)) / D;",
                     "C[l] = dl * sqrt((dl * dl - dm * dm) * (dl * dl - dp * dp)) / D;"),
    "c_condon_shortley_dropped": ("        if (m & 1) norm = -norm;\n        for (int q", "        for (int q"),
    "c_seed_constant_off": ("for (int k = 1; k <= m + 2; ++k) {", "for (int k = 1; k <= m + 1; ++k) {"),
    "c_shear_sign": ("pr += ww * dp * (a * er - b * ei);", "pr += ww * dp * (a * er + b * ei);"),
    "c_full_accumulates_wrong_part": ("acc[4 * l + 1] += qpi * dp[l];", "acc[4 * l + 1] += qpr * dp[l];"),
    "c_full_sign_dropped": ("            if (m & 1) norm = -norm;\n            const int64_t k", "            const int64_t k"),
    "c_m1_seed_sign": ("f = (mp < 0) ? 2.0 * c * s * s * s : -2.0 * c * c * c * s;",
                       "f = (mp < 0) ? 2.0 * c * s * s * s : 2.0 * c * c * c * s;"),
}


@pytest.mark.parametrize("name", sorted(C_MUTANTS))
def test_planted_spin_c_mistake_is_caught(oracle, tmp_path, name):
    import shutil
    import subprocess
    from oracle import ref
    old, new = C_MUTANTS[name]
    odir = os.path.join(os.path.dirname(HERE), "oracle")
    src = open(os.path.join(odir, "ptalm_ref.c")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    shutil.copy(os.path.join(odir, "ptalm_ref.h"), tmp_path / "ptalm_ref.h")
    (tmp_path / "ptalm_ref.c").write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", str(so),
                    str(tmp_path / "ptalm_ref.c"), "-lm"], check=True)
    with ref.use_library(str(so)):
        assert not all(pin(ref) for pin in C_PINS), f"planted mistake {name!r} passed every C spin pin"
