"""Checks that pin an implementation of a_lm = sum_i w_i Y*_lm(theta_i, phi_i) to
facts fixed by the paper and by mathematics, independently of any other
implementation.  Each check takes the transform as a callable
``alm_fn(theta, phi, w, lmax) -> complex128[T]`` (healpy order) and returns the
largest error it saw, so the same checks pin the CPU oracle, a copy of the
oracle with a planted mistake, and the GPU library.
"""
import math
import os

import numpy as np
from scipy.special import sph_harm_y

from conftest import alm_index, ell_of_index, m_of_index

FOUR_PI = 4.0 * math.pi
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# Standard table of spherical harmonics up to l = 3 with the Condon-Shortley
# phase (the minus sign in the sectoral recurrence of App. A.1), orthonormal on
# the unit sphere (the normalisation N_lm of Sec. 2.2).
def ylm_closed_form(l, m, th, ph):
    c, s = np.cos(th), np.sin(th)
    e = np.exp(1j * m * ph)
    pi = math.pi
    table = {
        (0, 0): 0.5 * math.sqrt(1 / pi) * np.ones_like(c),
        (1, 0): 0.5 * math.sqrt(3 / pi) * c,
        (1, 1): -0.5 * math.sqrt(3 / (2 * pi)) * s,
        (2, 0): 0.25 * math.sqrt(5 / pi) * (3 * c * c - 1),
        (2, 1): -0.5 * math.sqrt(15 / (2 * pi)) * s * c,
        (2, 2): 0.25 * math.sqrt(15 / (2 * pi)) * s * s,
        (3, 0): 0.25 * math.sqrt(7 / pi) * (5 * c ** 3 - 3 * c),
        (3, 1): -0.125 * math.sqrt(21 / pi) * s * (5 * c * c - 1),
        (3, 2): 0.25 * math.sqrt(105 / (2 * pi)) * s * s * c,
        (3, 3): -0.125 * math.sqrt(35 / pi) * s ** 3,
    }
    return table[(l, m)] * e


def special_points():
    th = np.array([0.0, math.pi, math.pi / 2, 1e-3, 0.3, 1.1, 2.0, math.pi - 1e-3, 2.9])
    ph = np.array([0.0, 1.0, 2.5, 0.7, 4.0, 6.2, 3.3, 5.1, 0.1])
    return th, ph


def pin_closed_forms(alm_fn):
    """P1a: single-point a_lm = conj(Y_lm) for l <= 3 against the textbook table."""
    th, ph = special_points()
    lmax = 3
    worst = 0.0
    for i in range(th.size):
        a = alm_fn(th[i:i + 1], ph[i:i + 1], np.ones(1), lmax)
        for l in range(lmax + 1):
            for m in range(l + 1):
                y = ylm_closed_form(l, m, th[i], ph[i])
                worst = max(worst, abs(a[alm_index(lmax, l, m)] - np.conj(y)))
    return worst


def pin_scipy(alm_fn, lmax=60, n=40, seed=7):
    """P1b: weighted multi-point a_lm against scipy.special.sph_harm_y (library routine)."""
    rng = np.random.default_rng(seed)
    th = np.arccos(rng.uniform(-1, 1, n))
    ph = rng.uniform(0, 2 * math.pi, n)
    w = rng.normal(size=n)
    a = alm_fn(th, ph, w, lmax)
    L, M = ell_of_index(lmax), m_of_index(lmax)
    ref = np.array([np.sum(w * np.conj(sph_harm_y(l, m, th, ph))) for l, m in zip(L, M)])
    return float(np.max(np.abs(a - ref)) / max(1.0, np.max(np.abs(ref))))


def single_point_cl(alm, lmax):
    L, M = ell_of_index(lmax), m_of_index(lmax)
    p = np.abs(alm) ** 2 * np.where(M == 0, 1.0, 2.0)
    return np.bincount(L, weights=p, minlength=lmax + 1) / (2 * np.arange(lmax + 1) + 1)


def pin_addition_theorem(alm_fn, lmax, thetas, weight=1.7):
    """P2: sum_{m=-l..l} |Y_lm(n)|^2 = (2l+1)/4pi at every point, i.e. the
    single-point pseudo-spectrum is w^2/4pi for every l.  Returns the largest
    relative deviation over l and points."""
    worst = 0.0
    for t in thetas:
        a = alm_fn(np.array([t]), np.array([1.234]), np.array([weight]), lmax)
        cl = single_point_cl(a, lmax)
        worst = max(worst, float(np.max(np.abs(cl * FOUR_PI / weight ** 2 - 1.0))))
    return worst


def pin_gl_orthonormality(alm_fn, lmax):
    """P3: Gauss-Legendre x uniform-phi quadrature makes the transform of a
    sampled band-limited function exact.  Returns the largest absolute error of
    a_lm against its exact value for f = 1, f = Y_l'0, f = Re Y_l'm', f = Im Y_l'm'."""
    from paper_2312_12285_amd.synth import gauss_legendre_grid

    th, ph, g = gauss_legendre_grid(lmax)
    worst = 0.0
    cases = [(None, None), (min(5, lmax), 0), (lmax, 0), (min(7, lmax), min(3, lmax)), (lmax, lmax // 2)]
    for (lp, mp) in cases:
        if lp is None:
            f = np.ones_like(th)
            want = {(0, 0): math.sqrt(FOUR_PI)}
            parts = [(f, want)]
        elif mp == 0:
            f = np.real(sph_harm_y(lp, 0, th, ph))
            parts = [(f, {(lp, 0): 1.0})]
        else:
            y = sph_harm_y(lp, mp, th, ph)
            parts = [(np.real(y), {(lp, mp): 0.5}), (np.imag(y), {(lp, mp): -0.5j})]
        for f, want in parts:
            a = alm_fn(th, ph, g * f, lmax)
            exp = np.zeros_like(a)
            for (l, m), v in want.items():
                exp[alm_index(lmax, l, m)] = v
            worst = max(worst, float(np.max(np.abs(a - exp))))
    return worst


def load_special_values():
    vals = {}
    with open(os.path.join(GOLDEN, "special_values.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            l, lab, v = line.split()
            vals[(int(l), lab)] = float(v)
    return vals


def pin_special_values(alm_fn, lmax=64):
    """P4: poles and equator from closed forms (tests/golden/special_values.txt):
    a_l0 exact, a_lm = 0 for m > 0 at the poles; single-point C_l = w^2/4pi."""
    vals = load_special_values()
    worst = 0.0
    pts = {"north": 0.0, "south": math.pi, "equator": math.pi / 2}
    M = m_of_index(lmax)
    for lab, t in pts.items():
        a = alm_fn(np.array([t]), np.array([0.9]), np.array([1.0]), lmax)
        for l in range(lmax + 1):
            worst = max(worst, abs(a[alm_index(lmax, l, 0)] - vals[(l, lab)]))
        if lab != "equator":
            worst = max(worst, float(np.max(np.abs(a[M > 0]))))
    return worst


def legendre_bonnet(lmax, mu):
    """P_l(mu) for l = 0..lmax by Bonnet's recurrence (l+1)P_{l+1} = (2l+1) mu P_l - l P_{l-1}."""
    out = np.empty((lmax + 1,) + mu.shape)
    out[0] = 1.0
    if lmax >= 1:
        out[1] = mu
    for l in range(1, lmax):
        out[l + 1] = ((2 * l + 1) * mu * out[l] - l * out[l - 1]) / (l + 1)
    return out


def unit_vectors(th, ph):
    return np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=-1)


def pair_sum_cross(thA, phA, wA, thB, phB, wB, lmax):
    """C^AB_l = (1/4pi) sum_{i in A} sum_{j in B} w_i w_j P_l(n_i . n_j) (addition theorem)."""
    mu = np.clip(unit_vectors(thA, phA) @ unit_vectors(thB, phB).T, -1.0, 1.0)
    P = legendre_bonnet(lmax, mu)
    return np.einsum("i,lij,j->l", wA, P, wB) / FOUR_PI


def pin_pair_sum(alm_fn, cl_fn, cross_fn, lmax=48, nA=150, nB=120, seed=11):
    """P5: auto and cross pseudo-spectra against the brute-force pair sum (no Y_lm
    involved).  Returns the largest relative error over l."""
    rng = np.random.default_rng(seed)
    thA = np.arccos(rng.uniform(-1, 1, nA)); phA = rng.uniform(0, 2 * math.pi, nA); wA = rng.lognormal(0, 0.3, nA)
    thB = np.arccos(rng.uniform(-1, 1, nB)); phB = rng.uniform(0, 2 * math.pi, nB); wB = rng.normal(size=nB)
    a = alm_fn(thA, phA, wA, lmax)
    b = alm_fn(thB, phB, wB, lmax)
    auto = cl_fn(a, lmax)
    cross = cross_fn(a, b, lmax)
    ref_auto = pair_sum_cross(thA, phA, wA, thA, phA, wA, lmax)
    ref_cross = pair_sum_cross(thA, phA, wA, thB, phB, wB, lmax)
    scale = np.sqrt(np.abs(ref_auto) * np.abs(pair_sum_cross(thB, phB, wB, thB, phB, wB, lmax)))
    e1 = np.max(np.abs(auto - ref_auto) / np.abs(ref_auto))
    e2 = np.max(np.abs(cross - ref_cross) / scale)
    return float(max(e1, e2))


def pin_monopole_dipole(alm_fn, n=500, seed=3):
    """P7: a_00 = sum w / sqrt(4pi); a_10 = sqrt(3/4pi) sum w cos(theta);
    a_11 = -sqrt(3/8pi) sum w sin(theta) e^{-i phi}."""
    rng = np.random.default_rng(seed)
    th = np.arccos(rng.uniform(-1, 1, n)); ph = rng.uniform(0, 2 * math.pi, n); w = rng.normal(size=n)
    a = alm_fn(th, ph, w, 1)
    e00 = np.sum(w) / math.sqrt(FOUR_PI)
    e10 = math.sqrt(3 / FOUR_PI) * np.sum(w * np.cos(th))
    e11 = -math.sqrt(3 / (2 * FOUR_PI)) * np.sum(w * np.sin(th) * np.exp(-1j * ph))
    return float(max(abs(a[0] - e00), abs(a[1] - e10), abs(a[2] - e11)))


def random_rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def pin_symmetries(alm_fn, lmax=40, n=300, seed=5):
    """P6: phi shift, reflection theta -> pi - theta, phi -> -phi, linearity,
    concatenation, permutation, and rotation invariance of C_l.  Returns the
    largest relative deviation."""
    rng = np.random.default_rng(seed)
    th = np.arccos(rng.uniform(-1, 1, n)); ph = rng.uniform(0, 2 * math.pi, n)
    w1 = rng.normal(size=n); w2 = rng.lognormal(0, 0.3, n)
    L, M = ell_of_index(lmax), m_of_index(lmax)
    a = alm_fn(th, ph, w1, lmax)
    nrm = np.max(np.abs(a))
    errs = []
    beta = 0.8123
    errs.append(np.max(np.abs(alm_fn(th, np.mod(ph + beta, 2 * math.pi), w1, lmax) - np.exp(-1j * M * beta) * a)))
    errs.append(np.max(np.abs(alm_fn(math.pi - th, ph, w1, lmax) - (-1.0) ** (L + M) * a)))
    errs.append(np.max(np.abs(alm_fn(th, np.mod(-ph, 2 * math.pi), w1, lmax) - np.conj(a))))
    b = alm_fn(th, ph, w2, lmax)
    errs.append(np.max(np.abs(alm_fn(th, ph, 2.5 * w1 - 0.75 * w2, lmax) - (2.5 * a - 0.75 * b))))
    half = n // 3
    errs.append(np.max(np.abs(alm_fn(th[:half], ph[:half], w1[:half], lmax)
                              + alm_fn(th[half:], ph[half:], w1[half:], lmax) - a)))
    perm = rng.permutation(n)
    errs.append(np.max(np.abs(alm_fn(th[perm], ph[perm], w1[perm], lmax) - a)))
    R = random_rotation(rng)
    v = unit_vectors(th, ph) @ R.T
    th_r = np.arccos(np.clip(v[:, 2], -1, 1)); ph_r = np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * math.pi)
    cl = single_point_cl(a, lmax)
    cl_r = single_point_cl(alm_fn(th_r, ph_r, w1, lmax), lmax)
    rel = max(float(np.max(errs)) / nrm, float(np.max(np.abs(cl_r - cl) / cl)))
    return rel
