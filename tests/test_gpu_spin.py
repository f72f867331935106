"""GPU spin-2 transform for shear (E and B modes) against the spin oracle.

Gate: 1e-10 per-l norm-wise relative error over m (the direct path's FP64
gate), and element-wise 1e-10 of the l-row norm.  Cases span several point
groups and l-blocks with ragged tails, lmax below, at and above the first
l-block, points on and next to both poles, the m = 0, 1 seeds, and near-pole
points at lmax 600 (the exponent-tracked seed and chain rescaling).  Also: every
compiled (points per lane, l-block) variant and slice count agree, repeated
calls are bitwise equal, E and B are exactly those of the two spin transforms
(E-B rotation by 45 degrees), empty and tiny inputs, argument checks.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2312_12285_amd import ptalm
    return ptalm


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def cplx(t):
    import torch
    torch.cuda.synchronize()
    a = t.cpu().numpy()
    return a[0::2] + 1j * a[1::2]


def per_l(got, ref, lmax):
    L = np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])
    num = np.bincount(L, weights=np.abs(got - ref) ** 2, minlength=lmax + 1)
    den = np.bincount(L, weights=np.abs(ref) ** 2, minlength=lmax + 1)
    return np.sqrt(num / np.maximum(den, 1e-300)), np.sqrt(den), L


def catalog(n, seed, polar=False):
    from paper_2312_12285_amd import synth
    t, p = synth.uniform_sphere(n, seed)
    if polar:   # half the points within a few degrees of a pole
        rng = np.random.default_rng(seed + 7)
        k = n // 2
        d = np.abs(rng.normal(0, 0.03, k))
        t[:k] = np.where(rng.random(k) < 0.5, d, math.pi - d)
    t[:6] = [0.0, math.pi, 1e-9, math.pi - 1e-7, 3e-4, math.pi / 2]
    w = synth.lognormal_weights(n, 0.3, seed + 100)
    g1, g2 = synth.shear_components(n, seed + 200)
    return t, p, w, g1, g2


def check(got_e, got_b, want_e, want_b, lmax, tol=1e-10):
    for got, want in ((got_e, want_e), (got_b, want_b)):
        err, norm, L = per_l(got, want, lmax)
        assert np.all(got[L < 2] == 0)
        assert err[2:].max() <= tol, err[2:].max()
        assert np.all(np.abs(got - want) <= tol * norm[L] + 1e-300)
    return max(per_l(got_e, want_e, lmax)[0][2:].max(), per_l(got_b, want_b, lmax)[0][2:].max())


@pytest.mark.parametrize("n,lmax,seed,polar", [(5_000, 64, 1, False), (3_001, 129, 2, False), (10_000, 180, 3, False),
                                               (700, 2, 4, False), (900, 3, 5, False), (257, 17, 6, True),
                                               (12_000, 90, 7, True)])
def test_shear_matches_oracle(lib, n, lmax, seed, polar):
    from oracle import spin
    t, p, w, g1, g2 = catalog(n, seed, polar)
    print(f"shear parity n {n} lmax {lmax} polar {polar}", flush=True)
    e, b = lib.shear_alm_from_points(dev(t), dev(p), dev(w), dev(g1), dev(g2), lmax)
    we, wb = spin.shear_eb(t, p, w, g1, g2, lmax)
    err = check(cplx(e), cplx(b), we, wb, lmax)
    print(f"  per-l max rel err {err:.3e}", flush=True)


def test_shear_near_poles_high_l(lib):
    """lmax 600 with most points within 0.2 deg of a pole: seeds far below the FP64 range
    at high m, chains that must be rescaled before their products enter the sums."""
    from oracle import spin
    rng = np.random.default_rng(11)
    n = 300
    d = np.abs(rng.normal(0, 0.003, n))
    t = np.where(rng.random(n) < 0.5, d, math.pi - d)
    t[:20] = np.arccos(rng.uniform(-1, 1, 20))
    p = rng.uniform(0, 2 * math.pi, n)
    w = rng.lognormal(0, 0.3, n)
    g1, g2 = rng.normal(0, 0.26, n), rng.normal(0, 0.26, n)
    lmax = 600
    print(f"shear near-pole parity n {n} lmax {lmax}", flush=True)
    e, b = lib.shear_alm_from_points(dev(t), dev(p), dev(w), dev(g1), dev(g2), lmax)
    we, wb = spin.shear_eb(t, p, w, g1, g2, lmax)
    err = check(cplx(e), cplx(b), we, wb, lmax)
    print(f"  per-l max rel err {err:.3e}", flush=True)


def test_variants_and_slices_agree(lib):
    t, p, w, g1, g2 = catalog(9_000, 21)
    lmax = 150
    args = [dev(a) for a in (t, p, w, g1, g2)]
    base_e, base_b = [cplx(x) for x in lib.shear_alm_from_points(*args, lmax)]
    for kp, lb in ((4, 8), (3, 8), (2, 8), (4, 16), (3, 16), (5, 8), (6, 4), (4, 4)):
        for S in (0, 1, 3):
            o = lib.opts(points_per_lane=kp, l_block=lb, n_slices=S)
            print(f"shear variant kp {kp} lb {lb} slices {S}", flush=True)
            e, b = [cplx(x) for x in lib.shear_alm_from_points(*args, lmax, options=o)]
            err_e, norm_e, L = per_l(e, base_e, lmax)
            err_b, _, _ = per_l(b, base_b, lmax)
            assert max(err_e[2:].max(), err_b[2:].max()) <= 1e-12


SINGLE_VARIANTS = [(4, 8), (5, 8), (6, 8), (7, 8), (8, 8), (4, 16), (5, 16), (6, 16)]


@pytest.mark.parametrize("kp,lb", SINGLE_VARIANTS)
def test_single_spin_form(lib, kp, lb):
    """One spin per wavefront (reduction option 2): ragged point count, partial l-blocks and
    polar points against the oracle; the two-spin form to rounding; E and B exactly real at
    m = 0 (the two spins' wavefronts run the same operations there)."""
    from oracle import spin
    t, p, w, g1, g2 = catalog(5_003, 51, True)
    lmax = 133
    print(f"single-spin variant kp {kp} lb {lb}", flush=True)
    args = [dev(a) for a in (t, p, w, g1, g2)]
    o = lib.opts(points_per_lane=kp, l_block=lb, reduction=2)
    e, b = [cplx(x) for x in lib.shear_alm_from_points(*args, lmax, options=o)]
    we, wb = spin.shear_eb(t, p, w, g1, g2, lmax)
    err = check(e, b, we, wb, lmax)
    print(f"  per-l max rel err against the oracle {err:.3e}", flush=True)
    e2, b2 = [cplx(x) for x in lib.shear_alm_from_points(*args, lmax, options=lib.opts(reduction=1))]
    assert max(per_l(e, e2, lmax)[0][2:].max(), per_l(b, b2, lmax)[0][2:].max()) <= 1e-12
    assert np.all(e[: lmax + 1].imag == 0.0) and np.all(b[: lmax + 1].imag == 0.0)


def test_single_spin_near_poles_high_l(lib):
    """The one-spin form on the near-pole catalog at lmax 600 (chain rescaling per spin)."""
    from oracle import spin
    rng = np.random.default_rng(12)
    n = 300
    d = np.abs(rng.normal(0, 0.003, n))
    t = np.where(rng.random(n) < 0.5, d, math.pi - d)
    t[:20] = np.arccos(rng.uniform(-1, 1, 20))
    p = rng.uniform(0, 2 * math.pi, n)
    w = rng.lognormal(0, 0.3, n)
    g1, g2 = rng.normal(0, 0.26, n), rng.normal(0, 0.26, n)
    lmax = 600
    print(f"single-spin near-pole parity n {n} lmax {lmax}", flush=True)
    o = lib.opts(reduction=2)
    e, b = lib.shear_alm_from_points(dev(t), dev(p), dev(w), dev(g1), dev(g2), lmax, options=o)
    we, wb = spin.shear_eb(t, p, w, g1, g2, lmax)
    err = check(cplx(e), cplx(b), we, wb, lmax)
    print(f"  per-l max rel err {err:.3e}", flush=True)


def test_repeatable_and_eb_rotation(lib):
    """Bitwise repeatable; rotating every shear by 45 degrees (g -> i g) maps (E, B) to (-B, E)."""
    t, p, w, g1, g2 = catalog(6_000, 31)
    lmax = 80
    a = [dev(x) for x in (t, p, w, g1, g2)]
    e1, b1 = [cplx(x) for x in lib.shear_alm_from_points(*a, lmax)]
    e2, b2 = [cplx(x) for x in lib.shear_alm_from_points(*a, lmax)]
    assert np.array_equal(e1, e2) and np.array_equal(b1, b2)
    er, br = [cplx(x) for x in lib.shear_alm_from_points(a[0], a[1], a[2], dev(-g2), dev(g1), lmax)]
    scale = max(np.abs(e1).max(), np.abs(b1).max())
    assert np.abs(er + b1).max() <= 1e-13 * scale and np.abs(br - e1).max() <= 1e-13 * scale


def test_empty_tiny_and_arguments(lib):
    import torch
    z = dev(np.zeros(0))
    e, b = lib.shear_alm_from_points(z, z, z, z, z, 10)
    assert not cplx(e).any() and not cplx(b).any()
    t, p, w, g1, g2 = catalog(100, 41)
    a = [dev(x) for x in (t, p, w, g1, g2)]
    for lmax in (0, 1):
        e, b = lib.shear_alm_from_points(*a, lmax)
        assert not cplx(e).any() and not cplx(b).any()
    with pytest.raises(lib.PtalmError):
        lib.shear_alm_from_points(*a, 10, options=lib.opts(precision=lib.MIXED))
    with pytest.raises(lib.PtalmError):
        lib.shear_alm_from_points(*a, 10, options=lib.opts(points_per_lane=9, l_block=8))
    with pytest.raises(lib.PtalmError):
        lib.shear_alm_from_points(*a, 10, options=lib.opts(points_per_lane=9, l_block=8, reduction=2))
    with pytest.raises(lib.PtalmError):
        lib.shear_alm_from_points(*a, 10, options=lib.opts(reduction=3))
    with pytest.raises(lib.PtalmError):
        lib.shear_alm_from_points(*a, 16384)
    with pytest.raises(ValueError):
        lib.shear_alm_from_points(a[0], a[1], a[2], a[3], dev(g2[:50]), 10)


def test_phase_periodicity(lib):
    """phi and phi + 2 pi k (negative angles included) give the same E and B."""
    t, p, w, g1, g2 = catalog(8_000, 51)
    k = np.random.default_rng(52).integers(-3, 6, size=p.size)
    a = [cplx(x) for x in lib.shear_alm_from_points(dev(t), dev(p), dev(w), dev(g1), dev(g2), 120)]
    b = [cplx(x) for x in lib.shear_alm_from_points(dev(t), dev(p + 2 * math.pi * k), dev(w), dev(g1), dev(g2), 120)]
    for x, y in zip(a, b):
        err, norm, L = per_l(y, x, 120)
        assert err[2:].max() <= 1e-12
