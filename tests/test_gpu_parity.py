"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Gate (reading of the 1e-10 target as a norm over m at each l):
    err_l = ||a_gpu[l, :] - a_ref[l, :]||_2 / ||a_ref[l, :]||_2 <= 1e-10 for every l,
plus element-wise |a_gpu - a_ref| <= 1e-10 * ||a_ref[l, :]|| / sqrt(l+1).
Near the poles at large l the rounding of x = cos(theta) alone moves P_l by up
to l(l+1)/2 ulp(x); single-point checks there use that bound instead.
"""
import math
import sys

import numpy as np
import pytest

import pins
from conftest import alm_index, ell_of_index, m_of_index, per_l_rel_err

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53
GATE = 1e-10


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2312_12285_amd import ptalm   # raises if the HIP library is missing
    return ptalm


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(*arrs):
    import torch
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def gpu_alm(lib, th, ph, w, lmax, **opt):
    import torch
    t, p, ww = to_dev(th, ph, w)
    o = lib.opts(**opt) if opt else None
    out = lib.alm_from_points(t, p, ww, lmax, options=o)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.complex128).copy()


def gpu_fn(lib, **opt):
    return lambda th, ph, w, lmax: gpu_alm(lib, th, ph, w, lmax, **opt)


def assert_gate(a, ref, lmax, gate=GATE, what=""):
    err = per_l_rel_err(a, ref, lmax)
    L = ell_of_index(lmax)
    nrm = np.sqrt(np.bincount(L, weights=np.abs(ref) ** 2, minlength=lmax + 1))
    elem = np.abs(a - ref) / np.maximum(nrm[L] / np.sqrt(L + 1.0), 1e-300)
    say(f"{what}: max per-l err {err.max():.3e} (l={err.argmax()}), max element err {elem.max():.3e}")
    assert err.max() <= gate
    assert elem.max() <= gate


def test_fullsky_lmax64_n1e4(lib, oracle):
    """The small workload in full: 1e4 uniform points, unit weights, lmax 64."""
    from paper_2312_12285_amd.synth import fullsky_uniform
    say("case: full sky n=1e4 lmax=64")
    cat = fullsky_uniform(10_000, seed=1)
    a = gpu_alm(lib, cat.theta, cat.phi, cat.w, 64)
    ref = oracle.alm_from_points(cat.theta, cat.phi, cat.w, 64)
    assert_gate(a, ref, 64, what="fullsky 1e4")


FP64_VARIANTS = [(6, 8, 0, 0), (7, 8, 0, 0), (6, 16, 0, 0), (6, 16, 1, 0), (6, 16, 1, 1), (6, 16, 0, 1),
                 (5, 16, 1, 1), (8, 16, 1, 1), (10, 16, 1, 1), (12, 16, 1, 1), (12, 16, 0, 1), (14, 8, 0, 1),
                 (14, 8, 1, 1), (12, 8, 1, 1), (4, 8, 0, 0), (8, 32, 0, 0), (16, 8, 0, 0), (7, 8, 1, 1), (8, 8, 1, 1),
                 (6, 8, 1, 1), (7, 16, 1, 1)]


@pytest.mark.parametrize("kp,lb,swap,pipe", FP64_VARIANTS)
def test_every_kernel_variant(lib, oracle, kp, lb, swap, pipe):
    """Ragged point count (not a multiple of 64*KP) and odd lmax (partial l-blocks)."""
    from paper_2312_12285_amd.synth import masked_galaxies
    say(f"case: variant kp={kp} lb={lb} swap={swap} pipe={pipe} n=5003 lmax=257")
    cat = masked_galaxies(5003, seed_pos=5, seed_w=6)
    lmax = 257
    ref = oracle.alm_from_points(cat.theta, cat.phi, cat.w, lmax)
    a = gpu_alm(lib, cat.theta, cat.phi, cat.w, lmax, points_per_lane=kp, l_block=lb,
                reduction=1 + swap + 2 * pipe)
    assert_gate(a, ref, lmax, what=f"kp={kp} lb={lb} swap={swap} pipe={pipe}")


@pytest.mark.parametrize("S,R", [(1, 1), (1, 258), (3, 7), (7, 100), (2, 0), (0, 1)])
def test_work_decompositions(lib, oracle, S, R):
    from paper_2312_12285_amd.synth import masked_randoms
    say(f"case: slices={S} ranges={R}")
    cat = masked_randoms(4000, seed=17)
    lmax = 257
    ref = oracle.alm_from_points(cat.theta, cat.phi, cat.w, lmax)
    a = gpu_alm(lib, cat.theta, cat.phi, cat.w, lmax, n_slices=S, m_ranges=R)
    assert_gate(a, ref, lmax, what=f"S={S} R={R}")


def test_edge_sizes(lib, oracle):
    from paper_2312_12285_amd.synth import fullsky_uniform
    say("case: n = 0")
    a = gpu_alm(lib, np.zeros(0), np.zeros(0), np.zeros(0), 20)
    assert a.shape == ((21 * 22) // 2,) and np.all(a == 0)
    for n in (1, 63, 64, 65, 383, 384, 385, 64 * 6 * 3 + 1):
        cat = fullsky_uniform(n, seed=100 + n)
        for lmax in (0, 1, 2, 9, 40):
            say(f"case: n={n} lmax={lmax}")
            ref = oracle.alm_from_points(cat.theta, cat.phi, cat.w, lmax)
            a = gpu_alm(lib, cat.theta, cat.phi, cat.w, lmax)
            assert_gate(a, ref, lmax, what=f"n={n} lmax={lmax}")


def test_special_points_single(lib, oracle):
    """Poles, equator, near-pole points one at a time against the long-double oracle."""
    lmax = 1024
    for t in (0.0, math.pi, math.pi / 2, 1e-6, 1e-3, 0.04, 1.0, math.pi - 3e-4):
        say(f"case: single point theta={t} lmax={lmax}")
        ref = oracle.alm_from_points(np.array([t]), np.array([0.7]), np.array([1.3]), lmax, long_double=True)
        a = gpu_alm(lib, np.array([t]), np.array([0.7]), np.array([1.3]), lmax)
        err = per_l_rel_err(a, ref, lmax)
        bound = max(GATE, 4 * lmax * (lmax + 1) / 2 * EPS)
        say(f"  max per-l err {err.max():.3e}")
        assert err.max() <= bound


def test_pins_closed_forms_special_values(lib):
    say("case: pins closed forms / special values / monopole-dipole")
    fn = gpu_fn(lib)
    assert pins.pin_closed_forms(fn) < 1e-15
    assert pins.pin_special_values(fn, lmax=64) < 1e-13
    assert pins.pin_monopole_dipole(fn) < 1e-12


def test_pins_scipy_pairsum_symmetries(lib):
    import torch
    say("case: pins scipy / pair sum / symmetries")
    fn = gpu_fn(lib)
    assert pins.pin_scipy(fn, lmax=60) < 1e-13

    def cl(a, lmax):
        t = torch.as_tensor(np.ascontiguousarray(a).view(np.float64)).cuda()
        return lib.cl_from_alm(t, lmax).cpu().numpy()

    def cross(a, b, lmax):
        ta = torch.as_tensor(np.ascontiguousarray(a).view(np.float64)).cuda()
        tb = torch.as_tensor(np.ascontiguousarray(b).view(np.float64)).cuda()
        return lib.cross_cl(ta, tb, lmax).cpu().numpy()

    assert pins.pin_pair_sum(fn, cl, cross, lmax=48) < 1e-11
    assert pins.pin_symmetries(fn) < 1e-12


def test_addition_theorem_lmax3072(lib):
    say("case: addition theorem lmax=3072")
    fn = gpu_fn(lib)
    assert pins.pin_addition_theorem(fn, 3072, [0.4, 1.0, 1.5707963, 2.2]) < 1e-12
    lmax = 3072
    got = pins.pin_addition_theorem(fn, lmax, [0.0, 1e-4, 1e-3, 0.05, math.pi - 1e-3])
    assert got < 4 * lmax * (lmax + 1) / 2 * EPS


@pytest.mark.parametrize("lmax", [64, 256, 1024])
def test_gauss_legendre_orthonormality(lib, lmax):
    """Exact expected values, no oracle: quadrature grid nodes reach close to the poles."""
    say(f"case: GL orthonormality lmax={lmax}")
    tol = 10 * 4 * math.pi * math.sqrt((2 * lmax + 1) / (4 * math.pi)) * lmax * EPS
    got = pins.pin_gl_orthonormality(gpu_fn(lib), lmax)
    say(f"  worst abs err {got:.3e} (tol {tol:.3e})")
    assert got < tol


def test_deterministic(lib):
    from paper_2312_12285_amd.synth import masked_galaxies
    say("case: determinism")
    cat = masked_galaxies(20000, seed_pos=8, seed_w=9)
    a = gpu_alm(lib, cat.theta, cat.phi, cat.w, 300)
    b = gpu_alm(lib, cat.theta, cat.phi, cat.w, 300)
    assert np.array_equal(a.view(np.float64), b.view(np.float64))


def test_spectra_and_fkp_on_identical_input(lib, oracle):
    import torch
    from paper_2312_12285_amd.synth import masked_galaxies, masked_randoms
    say("case: cl / cross_cl / fkp on oracle a_lm")
    lmax = 200
    g = masked_galaxies(3000, seed_pos=30, seed_w=31)
    r = masked_randoms(9000, seed=32)
    ad = oracle.alm_from_points(g.theta, g.phi, g.w, lmax)
    ar = oracle.alm_from_points(r.theta, r.phi, r.w, lmax)
    td = torch.as_tensor(ad.view(np.float64)).cuda()
    tr = torch.as_tensor(ar.view(np.float64)).cuda()
    cl = lib.cl_from_alm(td, lmax).cpu().numpy()
    assert np.max(np.abs(cl - oracle.cl_from_alm(ad, lmax)) / oracle.cl_from_alm(ad, lmax)) < 1e-13
    xc = lib.cross_cl(td, tr, lmax).cpu().numpy()
    ref = oracle.cross_cl(ad, ar, lmax)
    scale = np.sqrt(oracle.cl_from_alm(ad, lmax) * oracle.cl_from_alm(ar, lmax))
    assert np.max(np.abs(xc - ref) / scale) < 1e-13
    delta, window, alpha = lib.fkp_fields(td, tr, lmax)
    a_host = ad[0].real / ar[0].real
    assert abs(alpha.item() - a_host) <= 1e-15 * abs(a_host)
    assert abs(alpha.item() - g.w.sum() / r.w.sum()) < 1e-12 * abs(a_host)   # a_00 = sum w / sqrt(4pi)
    dn = delta.cpu().numpy().view(np.complex128)
    wn = window.cpu().numpy().view(np.complex128)
    assert np.max(np.abs(dn - (ad - a_host * ar))) < 1e-13 * np.max(np.abs(ad))
    assert np.max(np.abs(wn - a_host * ar)) < 1e-13 * np.max(np.abs(ad))
    y = td.clone()
    lib.alm_axpy(-0.5, tr, y, lmax)
    assert np.max(np.abs(y.cpu().numpy().view(np.complex128) - (ad - 0.5 * ar))) < 1e-13 * np.max(np.abs(ad))


def test_masked_galaxies_subsample_lmax1024(lib, oracle):
    """Subsample of the masked galaxy + random workload at its lmax."""
    from paper_2312_12285_amd.synth import masked_galaxies, masked_randoms
    lmax = 1024
    say("case: masked galaxies 8000 + randoms 8000, lmax=1024")
    g = masked_galaxies(2_000_000, seed_pos=21, seed_w=22).head(8000)
    r = masked_randoms(8000, seed=23)          # prefix of the 2e7-random catalog
    for cat, name in ((g, "galaxies"), (r, "randoms")):
        ref = oracle.alm_from_points(cat.theta, cat.phi, cat.w, lmax)
        a = gpu_alm(lib, cat.theta, cat.phi, cat.w, lmax)
        assert_gate(a, ref, lmax, what=name)


def test_masked_randoms_subsample_lmax3072(lib, oracle):
    """First points of the 1e8-random workload at lmax 3072 (the mask reaches the north pole)."""
    from paper_2312_12285_amd.synth import uniform_in_mask
    lmax = 3072
    say("case: masked randoms n=1500 lmax=3072")
    th, ph = uniform_in_mask(1500, 31)
    w = np.ones(th.size)
    ref = oracle.alm_from_points(th, ph, w, lmax)
    a = gpu_alm(lib, th, ph, w, lmax)
    assert_gate(a, ref, lmax, what="randoms lmax3072")
