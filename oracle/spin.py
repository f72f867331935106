"""Oracle of the spin-weighted transform for shear (test infrastructure only).

The paper notes that fields of non-zero spin (cosmic shear) take spin-weighted
harmonics +-2 Y_lm in place of Y_lm, computed by recurrences (end of Sec. 4).
This module writes that generalisation out in plain numpy:

* sY_lm by the explicit finite sum of Goldberg et al. (J. Math. Phys. 8, 2155,
  1967) for small l (the pins' reference), with sY_lm(theta, phi) =
  (-1)^m sqrt((2l+1)/(4 pi)) d^l_{m,-s}(theta) e^{i m phi} and the Wigner d of
  the Wigner sum formula;
* for the transform, the same functions by the three-term recurrence of the
  Wigner d in l at fixed (m, m'), seeded at l = max(|m|, |m'|) by the one-term
  case of the sum formula (fp64, vectorised over points);
* _s a_lm = sum_i w_i f_i sY*_lm(theta_i, phi_i), m >= 0, for a spin-s field
  f (f = gamma_1 + i gamma_2 for s = 2 and its conjugate for s = -2), and the
  E/B combinations a^E = -(_2a + _-2a)/2, a^B = i (_2a - _-2a)/2.
"""
import math

import numpy as np


def wigner_d_explicit(l: int, m: int, mp: int, beta):
    """d^l_{m mp}(beta) by the Wigner sum formula (any l; exact for small l)."""
    beta = np.asarray(beta, dtype=np.float64)
    c, s = np.cos(beta / 2), np.sin(beta / 2)
    f = math.factorial
    pref = math.sqrt(f(l + m) * f(l - m) * f(l + mp) * f(l - mp))
    out = np.zeros_like(beta)
    for k in range(max(0, m - mp), min(l + m, l - mp) + 1):
        den = f(l + m - k) * f(k) * f(l - k - mp) * f(k - m + mp)
        sign = -1.0 if (k - m + mp) % 2 else 1.0
        out += sign * pref / den * c ** (2 * l - 2 * k + m - mp) * s ** (2 * k - m + mp)
    return out


def sylm_explicit(s: int, l: int, m: int, theta, phi):
    """sY_lm(theta, phi) = (-1)^m sqrt((2l+1)/(4 pi)) d^l_{m,-s}(theta) e^{i m phi}."""
    if l < max(abs(m), abs(s)):
        return np.zeros(np.shape(theta), dtype=np.complex128)
    d = wigner_d_explicit(l, m, -s, theta)
    return (-1.0) ** m * math.sqrt((2 * l + 1) / (4 * math.pi)) * d * np.exp(1j * m * np.asarray(phi))


def goldberg(s: int, l: int, m: int, theta, phi):
    """Goldberg et al.'s explicit sum for sY_lm (independent form for the pins)."""
    theta = np.asarray(theta, dtype=np.float64)
    f = math.factorial
    if l < max(abs(m), abs(s)):
        return np.zeros(theta.shape, dtype=np.complex128)
    pref = (-1.0) ** m * math.sqrt(f(l + m) * f(l - m) * (2 * l + 1) / (4 * math.pi * f(l + s) * f(l - s)))
    sh2 = np.sin(theta / 2) ** (2 * l)
    cot = 1.0 / np.tan(theta / 2)
    tot = np.zeros(theta.shape)
    for r in range(0, l - s + 1):
        k = r + s - m
        if k < 0 or k > l + s:
            continue
        tot += math.comb(l - s, r) * math.comb(l + s, k) * (-1.0) ** (l - r - s) * cot ** (2 * r + s - m)
    return pref * sh2 * tot * np.exp(1j * m * np.asarray(phi))


def _pow_scaled(b, p: int):
    """b**p as (mantissa, exponent) arrays, mantissa in [0.5, 1) (or 0), by binary
    powering with renormalisation after every product."""
    mant = np.ones_like(b)
    ex = np.zeros(b.shape, dtype=np.int64)
    bm, be = np.frexp(b)
    be = be.astype(np.int64)
    while p:
        if p & 1:
            mant, e = np.frexp(mant * bm)
            ex += be + e
        p >>= 1
        if p:
            bm, e = np.frexp(bm * bm)
            be = 2 * be + e
    return mant, ex


def _seed(l0: int, m: int, mp: int, beta):
    """d^{l0}_{m mp}(beta) at l0 = max(|m|, |mp|), where the sum formula has a single
    term, as (mantissa, exponent): for l0 = m it is sqrt(C(2m, m+mp)) c^(m+mp) s^(m-mp)
    with c, s = cos, sin(beta/2); the binomial is an exact integer."""
    if l0 != m:
        v = wigner_d_explicit(l0, m, mp, beta)   # small l0 (= |mp|)
        mant, ex = np.frexp(v)
        return mant, ex.astype(np.int64)
    C = math.comb(2 * m, m + mp)
    sh = max(C.bit_length() - 100, 0)
    sh += sh & 1
    k = math.sqrt(float(C >> sh))                # sqrt(C) = k 2^(sh/2), relative error < 2^-53
    cm, ce = _pow_scaled(np.cos(beta / 2), m + mp)
    sm, se = _pow_scaled(np.sin(beta / 2), m - mp)
    mant, e = np.frexp(k * cm * sm)
    return mant, ce + se + e + sh // 2


def spin_lambda(s: int, m: int, lmax: int, theta):
    """sY_lm(theta, 0) for l = max(|m|,|s|)..lmax (rows) at each theta (columns), m >= 0,
    by the Wigner-d recurrence in l:
      l sqrt(((l+1)^2-m^2)((l+1)^2-mp^2)) d^{l+1}
        = (2l+1) (l(l+1) cos b - m mp) d^l - (l+1) sqrt((l^2-m^2)(l^2-mp^2)) d^{l-1},
    with mp = -s.  The chain runs on mantissas with a per-point binary exponent
    (rescaled by 2^-300 when it passes 2^300), so seeds far below the FP64 range
    near the poles still give every value that is representable."""
    theta = np.asarray(theta, dtype=np.float64)
    mp = -s
    l0 = max(abs(m), abs(mp))
    out = np.zeros((lmax + 1, theta.size))
    if l0 > lmax:
        return out
    x = np.cos(theta)
    d_prev = np.zeros(theta.size)
    d, ex = _seed(l0, m, mp, theta)
    out[l0] = np.ldexp(d, ex)
    for l in range(l0, lmax):
        a = l * math.sqrt(((l + 1) ** 2 - m * m) * ((l + 1) ** 2 - mp * mp))
        b = (2 * l + 1)
        c = (l + 1) * math.sqrt((l * l - m * m) * (l * l - mp * mp)) if l > 0 else 0.0
        if a == 0.0:          # only at l = 0 with l0 = 0
            d_next = x * d    # d^1_{00} = cos b
        else:
            d_next = (b * (l * (l + 1) * x - m * mp) * d - c * d_prev) / a
        big = np.abs(d_next) > 2.0 ** 300
        if big.any():
            d_next = np.where(big, np.ldexp(d_next, -300), d_next)
            d = np.where(big, np.ldexp(d, -300), d)
            ex = ex + 300 * big
        d_prev, d = d, d_next
        out[l + 1] = np.ldexp(d, np.minimum(np.maximum(ex, -2000), 2000))
    ls = np.arange(lmax + 1)
    norm = (-1.0) ** m * np.sqrt((2 * ls + 1) / (4 * math.pi))
    return out * norm[:, None]


def spin_alm(s: int, theta, phi, w, f, lmax: int):
    """_s a_lm = sum_i w_i f_i sY*_lm(theta_i, phi_i), m >= 0, healpy order (complex)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    q = np.asarray(w, dtype=np.float64) * np.asarray(f, dtype=np.complex128)
    T = (lmax + 1) * (lmax + 2) // 2
    out = np.zeros(T, dtype=np.complex128)
    for m in range(lmax + 1):
        lam = spin_lambda(s, m, lmax, theta)        # [l, point], real
        z = q * np.exp(-1j * m * phi)
        base = m * (2 * lmax + 1 - m) // 2
        out[base + m: base + lmax + 1] = lam[m:] @ z
    return out


def shear_eb(theta, phi, w, g1, g2, lmax: int):
    """(a^E, a^B) of a weighted shear catalog: a^E = -(_2a + _-2a)/2, a^B = i (_2a - _-2a)/2."""
    gp = np.asarray(g1) + 1j * np.asarray(g2)
    a2 = spin_alm(2, theta, phi, w, gp, lmax)
    am2 = spin_alm(-2, theta, phi, w, np.conj(gp), lmax)
    return -(a2 + am2) / 2, 1j * (a2 - am2) / 2
