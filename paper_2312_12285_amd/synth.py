"""Seeded synthetic point catalogs (numpy PCG64), shared by tests, bench and smoke.

Nothing here evaluates the transform: this module only draws positions and
weights.  Workload recipes:

* full sky: cos(theta) ~ U[-1, 1], phi ~ U[0, 2pi), unit weights;
* survey mask: positions read as equatorial (dec = 90deg - theta, RA = phi),
  kept where dec > -10deg and |galactic latitude| > 20deg (J2000 north
  galactic pole RA 192.85948deg, Dec 27.12825deg); uniform-in-mask positions by
  rejection sampling in chunks;
* lognormal weights w = exp(sigma z - sigma^2/2), z ~ N(0, 1) (mean one);
* clustering stand-in: a fraction of the catalog is copies of random parents
  displaced by an isotropic tangent-plane Gaussian (redrawn until inside the
  mask);
* Gauss-Legendre x uniform-phi quadrature grid (exact orthonormality check);
* shear components for the spin-2 transform: g1, g2 ~ N(0, 0.26^2) each
  (intrinsic-ellipticity scatter per component, no coherent signal);
* golden-spiral point set of Sec. 3.1 (cos theta_k = (1 - (2k+1)/N)/2,
  phi_k = 2 pi k / golden ratio, k < N), optionally perturbed.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

NGP_RA_DEG = 192.85948
NGP_DEC_DEG = 27.12825
TWO_PI = 2.0 * math.pi


def uniform_sphere(n: int, seed: int):
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, TWO_PI, n)
    return np.arccos(u), phi


def in_mask(theta, phi, dec_min_deg: float = -10.0, b_min_deg: float = 20.0):
    """Boolean mask: dec > dec_min and |galactic b| > b_min."""
    dec = 0.5 * math.pi - np.asarray(theta)
    ra = np.asarray(phi)
    dg = math.radians(NGP_DEC_DEG)
    ag = math.radians(NGP_RA_DEG)
    sinb = np.sin(dec) * math.sin(dg) + np.cos(dec) * math.cos(dg) * np.cos(ra - ag)
    return (dec > math.radians(dec_min_deg)) & (np.abs(sinb) > math.sin(math.radians(b_min_deg)))


MASK_CHUNK = 1 << 20


def uniform_in_mask(n: int, seed: int):
    """n positions uniform on the sphere restricted to the survey mask.

    Candidates are drawn in fixed chunks of 2^20, so the first k points of a
    catalog do not depend on its size: uniform_in_mask(k, s) equals
    uniform_in_mask(N, s)[:k] for k <= N (subsamples are prefixes)."""
    rng = np.random.default_rng(seed)
    theta = np.empty(n)
    phi = np.empty(n)
    filled = 0
    while filled < n:
        m = MASK_CHUNK
        u = rng.uniform(-1.0, 1.0, m)
        p = rng.uniform(0.0, TWO_PI, m)
        t = np.arccos(u)
        keep = in_mask(t, p)
        t, p = t[keep], p[keep]
        take = min(t.size, n - filled)
        theta[filled:filled + take] = t[:take]
        phi[filled:filled + take] = p[:take]
        filled += take
    return theta, phi


def lognormal_weights(n: int, sigma: float, seed: int):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(n)
    return np.exp(sigma * z - 0.5 * sigma * sigma)


def _jitter(theta, phi, sigma_rad, rng):
    """Displace each point by an isotropic tangent-plane Gaussian of width sigma_rad."""
    st, ct = np.sin(theta), np.cos(theta)
    sp, cp = np.sin(phi), np.cos(phi)
    n = np.stack([st * cp, st * sp, ct], axis=-1)
    e_t = np.stack([ct * cp, ct * sp, -st], axis=-1)
    e_p = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
    dx = rng.standard_normal(theta.size) * sigma_rad
    dy = rng.standard_normal(theta.size) * sigma_rad
    d = dx[:, None] * e_t + dy[:, None] * e_p
    r = np.sqrt(dx * dx + dy * dy)
    safe = np.where(r > 0, r, 1.0)
    v = n * np.cos(r)[:, None] + d * (np.sin(r) / safe)[:, None]
    v /= np.linalg.norm(v, axis=-1)[:, None]
    t2 = np.arccos(np.clip(v[:, 2], -1.0, 1.0))
    p2 = np.mod(np.arctan2(v[:, 1], v[:, 0]), TWO_PI)
    return t2, p2


def clustered_in_mask(n: int, seed: int, child_fraction: float = 0.02, jitter_deg: float = 0.1):
    """Uniform-in-mask parents plus jittered copies of randomly chosen parents."""
    rng = np.random.default_rng(seed)
    n_child = int(round(child_fraction * n))
    n_par = n - n_child
    theta, phi = uniform_in_mask(n_par, int(rng.integers(1 << 62)))
    src = rng.integers(0, n_par, n_child)
    ct, cp = theta[src].copy(), phi[src].copy()
    todo = np.arange(n_child)
    out_t, out_p = np.empty(n_child), np.empty(n_child)
    sig = math.radians(jitter_deg)
    while todo.size:
        t2, p2 = _jitter(ct[todo], cp[todo], sig, rng)
        ok = in_mask(t2, p2)
        out_t[todo[ok]] = t2[ok]
        out_p[todo[ok]] = p2[ok]
        todo = todo[~ok]
    return np.concatenate([theta, out_t]), np.concatenate([phi, out_p])


def gauss_legendre_grid(lmax: int):
    """Nodes (theta, phi) and quadrature weights g_k * 2pi/N_phi of a grid that
    integrates every product Y*_lm Y_l'm' with l, l' <= lmax exactly:
    N_theta = lmax+1 Gauss-Legendre nodes in cos(theta), N_phi = 2 lmax + 2."""
    from scipy.special import roots_legendre

    ntheta, nphi = lmax + 1, 2 * lmax + 2
    x, g = roots_legendre(ntheta)
    th = np.arccos(x)
    ph = TWO_PI * np.arange(nphi) / nphi
    theta = np.repeat(th, nphi)
    phi = np.tile(ph, ntheta)
    w = np.repeat(g, nphi) * (TWO_PI / nphi)
    return theta, phi, w


def golden_spiral(n: int, perturb: float = 0.0, seed: int = 0):
    """Golden-spiral points between cos(theta) = -1/2 and +1/2 (Sec. 3.1)."""
    k = np.arange(n, dtype=np.float64)
    golden = (1.0 + math.sqrt(5.0)) / 2.0
    cth = 0.5 * (1.0 - (2.0 * k + 1.0) / n)
    phi = np.mod(TWO_PI * k / golden, TWO_PI)
    theta = np.arccos(cth)
    if perturb > 0:
        rng = np.random.default_rng(seed)
        theta = np.clip(theta + perturb * rng.standard_normal(n), 0.0, math.pi)
        phi = np.mod(phi + perturb * rng.standard_normal(n), TWO_PI)
    return theta, phi


# ----------------------------------------------------------------------------------------
# The five benchmark workloads and their sizes
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class Catalog:
    theta: np.ndarray
    phi: np.ndarray
    w: np.ndarray

    @property
    def n(self) -> int:
        return int(self.theta.size)

    def head(self, k: int) -> "Catalog":
        return Catalog(self.theta[:k], self.phi[:k], self.w[:k])


def fullsky_uniform(n: int = 10_000, seed: int = 1) -> Catalog:
    """Full sky, unit weights (lmax 64 workload)."""
    t, p = uniform_sphere(n, seed)
    return Catalog(t, p, np.ones(n))


def masked_galaxies(n: int = 2_000_000, seed_pos: int = 21, seed_w: int = 22, sigma: float = 0.3) -> Catalog:
    """Galaxies in the survey mask with 2% jittered duplicates, lognormal weights."""
    t, p = clustered_in_mask(n, seed_pos)
    return Catalog(t, p, lognormal_weights(n, sigma, seed_w))


def shear_components(n: int, seed: int, sigma_e: float = 0.26):
    """Shear (g1, g2) per galaxy: independent Gaussian components of rms sigma_e."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, sigma_e, n), rng.normal(0.0, sigma_e, n)


def masked_randoms(n: int, seed: int) -> Catalog:
    """Randoms uniform in the survey mask, unit weights."""
    t, p = uniform_in_mask(n, seed)
    return Catalog(t, p, np.ones(n))


def multi_weight_positions(n: int = 10_000_000, n_weights: int = 32, seed_pos: int = 41,
                           seed_w0: int = 4100, sigma: float = 0.2):
    """One position set in the mask and n_weights lognormal weight vectors ([n_weights, n])."""
    t, p = uniform_in_mask(n, seed_pos)
    w = np.stack([lognormal_weights(n, sigma, seed_w0 + v) for v in range(n_weights)])
    return t, p, w


@dataclasses.dataclass
class Request:
    arrival_s: float
    n: int
    lmax: int
    seed: int


def served_trace(k: int = 500, rate_hz: float = 50.0, seed: int = 51,
                 lmaxes=(128, 256, 512, 1024, 2048), log10_n=(4.0, 7.0)):
    """Poisson arrivals; n log-uniform; lmax uniform over the set.  Catalog k is
    drawn with seed 5100 + k by ``served_catalog``."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, k)
    t = np.cumsum(gaps) - gaps[0]
    ns = np.round(10.0 ** rng.uniform(log10_n[0], log10_n[1], k)).astype(np.int64)
    ls = np.asarray(lmaxes)[rng.integers(0, len(lmaxes), k)]
    return [Request(float(t[i]), int(ns[i]), int(ls[i]), 5100 + i) for i in range(k)]


def served_catalog(req: Request, sigma: float = 0.3) -> Catalog:
    t, p = uniform_in_mask(req.n, req.seed)
    return Catalog(t, p, lognormal_weights(req.n, sigma, req.seed + 1_000_000))


def window_spectrum(lmax_w: int, seed: int, f_sky: float = 0.344, slope: float = 2.5):
    """Stand-in for the angular power spectrum of a survey window (mode-coupling workload):
    4 pi f_sky^2 at l = 0, then 0.3 * 4 pi f_sky^2 (1 + l)^-slope, each l scaled by an
    independent chi-square draw with 2(2l+1) degrees of freedom over its mean (the scatter of
    a power estimated from 2l+1 complex modes), plus a floor of 1e-9 of W_0.  All positive."""
    rng = np.random.default_rng(seed)
    l = np.arange(lmax_w + 1, dtype=np.float64)
    w0 = 4.0 * math.pi * f_sky * f_sky
    dof = 2.0 * (2.0 * l + 1.0)
    W = 0.3 * w0 * (1.0 + l) ** -slope * rng.chisquare(dof) / dof + 1e-9 * w0
    W[0] = w0
    return W


def pseudo_spectrum(lmax: int, seed: int, amp: float = 1e-4, slope: float = 1.2, shot: float = 2e-6):
    """Stand-in for a measured pseudo-spectrum of galaxy counts (bandpower workload):
    amp (1 + l/10)^-slope scaled per l by a chi-square draw with 2l+1 degrees of freedom over
    its mean, plus a constant shot-noise level."""
    rng = np.random.default_rng(seed)
    l = np.arange(lmax + 1, dtype=np.float64)
    dof = 2.0 * l + 1.0
    return amp * (1.0 + l / 10.0) ** -slope * rng.chisquare(dof) / dof + shot
