"""Parity at the largest sizes the library accepts.

lmax = 16383 (T = 1.34e8 coefficients, the limit that keeps every coefficient
index in 32 bits). A small full-sky catalog keeps the GPU work light while every
table, scratch buffer and index runs to its maximum extent:

* FP64: sampled coefficients against the oracle over every point (<= 1e-10 of
  the rms at their l), including the last column m = 16383;
* single points at the poles: the closed form a_l0 = w sqrt((2l+1)/4pi), times
  (-1)^l at the south pole, over the whole m = 0 column; exact zeros at m > 0
  at the north pole (sin theta = 0), and the oracle's values at the south pole,
  where sin(theta) of the rounded pi is 1.2e-16;
* the mixed form against FP64 (global <= 1e-6), the FP32 form within
  8 (l+1) 2^-24 at each l, and 16 weight vectors on the
  split-bf16 matrix-core path against the oracle and FP64 (<= 1e-4);
* the spin +-2 transform: sampled E and B coefficients against the spin oracle;
* the interpolated transform: sampled coefficients against the oracle's;
* the mode-coupling matrix (window to l = 1024): sampled rows against the
  oracle, zeros outside the band, and the transpose relation.

n = 2^31 + 777 points (point indices past the 32-bit range, 51.5 GB of inputs):
a base catalog of 2^20 points repeated 2048 times, then its first 777 points.
The transform is linear in the catalog, so a_lm = 2048 a_lm(base) + a_lm(first
777) in exact arithmetic, both terms from the oracle; checked for the FP64 path
and the spin transform at lmax 64 over every coefficient.
"""
import math
import sys

import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

LMAX = 16383
GATE = 1e-10
EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2312_12285_amd import ptalm
    return ptalm


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(*arrs):
    import torch
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


PAIRS = [(2, 0), (2, 1), (2, 2), (5000, 17), (8191, 8191), (12000, 6000), (16383, 0), (16383, 1),
         (16383, 8191), (16383, 16382), (16383, 16383)]


def sampled(lib, alm_dev, pairs):
    """The coefficients at pairs, gathered on the device."""
    import torch
    idx = torch.tensor([lib.alm_index(LMAX, l, m) for l, m in pairs], device=alm_dev.device)
    return lib.as_complex(alm_dev)[idx].cpu().numpy()


def catalog():
    from paper_2312_12285_amd.synth import uniform_sphere
    t, p = uniform_sphere(190, 71)
    w = np.random.default_rng(72).uniform(0.5, 1.5, t.size)
    return t, p, w


def test_fp64_and_mixed_at_maximum_lmax(lib, oracle):
    import torch
    say(f"case: 190 full-sky points, lmax {LMAX}, FP64")
    t, p, w = catalog()
    d = dev(t, p, w)
    a = lib.alm_from_points(*d, LMAX)
    torch.cuda.synchronize()
    ls = np.array([l for l, _ in PAIRS]); ms = np.array([m for _, m in PAIRS])
    want = oracle.alm_entries(t, p, w, ls, ms)
    cl = lib.cl_from_alm(a, LMAX).cpu().numpy()
    rel = np.abs(sampled(lib, a, PAIRS) - want) / np.sqrt(cl[ls])
    say(f"fp64: sampled entries, max |err| / rms_l = {rel.max():.3e}")
    assert rel.max() <= GATE
    assert abs(a[0].item() - math.fsum(w) / math.sqrt(4 * math.pi)) <= 1e-13 * a[0].item()

    say(f"case: 190 full-sky points, lmax {LMAX}, mixed")
    b = lib.alm_from_points(*d, LMAX, options=lib.opts(precision=lib.MIXED))
    torch.cuda.synchronize()
    g = (torch.linalg.norm(b - a) / torch.linalg.norm(a)).item()
    say(f"mixed vs fp64: global {g:.3e}")
    assert g <= 1e-6


@pytest.mark.parametrize("theta,sign", [(0.0, 1.0), (math.pi, -1.0)])
def test_poles_at_maximum_lmax(lib, oracle, theta, sign):
    import torch
    say(f"case: single point theta={theta}, lmax {LMAX}")
    wv = 1.7
    d = dev(np.array([theta]), np.array([0.3]), np.array([wv]))
    a = lib.alm_from_points(*d, LMAX)
    torch.cuda.synchronize()
    col0 = lib.as_complex(a[: 2 * (LMAX + 1)]).cpu().numpy()     # m = 0, l = 0..lmax
    l = np.arange(LMAX + 1)
    want = wv * np.sqrt((2 * l + 1) / (4 * math.pi)) * sign ** l
    rel = np.abs(col0 - want) / np.abs(want)
    # rounding of the recurrence grows linearly in l at x = +-1 (the oracle's own FP64 sum: 2.1e-11)
    say(f"pole m = 0 column: max rel err {rel.max():.3e} (bound {64 * LMAX * EPS:.1e})")
    assert rel.max() <= 64 * LMAX * EPS
    rest = lib.as_complex(a[2 * (LMAX + 1):])
    if theta == 0.0:
        assert torch.count_nonzero(rest).item() == 0        # sin(theta) = 0: every m > 0 vanishes
    else:
        pairs = [(LMAX, 1), (LMAX, 2), (5000, 1), (LMAX, 100), (LMAX, LMAX)]
        want = oracle.alm_entries(np.array([theta]), np.array([0.3]), np.array([wv]),
                                  [q[0] for q in pairs], [q[1] for q in pairs])
        got = sampled(lib, a, pairs)
        rms = wv / math.sqrt(4 * math.pi)      # rms at every l: only m = 0 is of order one
        say(f"south pole m > 0: got {np.abs(got)}, oracle {np.abs(want)}")
        assert np.all(np.abs(got - want) <= GATE * rms)
        assert torch.abs(rest).max().item() <= 1e-6       # m >= 1 carries sin(theta)^m = (1.2e-16)^m


def test_spin_at_maximum_lmax(lib, oracle):
    import torch
    from paper_2312_12285_amd.synth import shear_components
    say(f"case: shear, 190 full-sky points, lmax {LMAX}")
    t, p, w = catalog()
    g1, g2 = shear_components(t.size, seed=73)
    e, b = lib.shear_alm_from_points(*dev(t, p, w, g1, g2), LMAX)
    torch.cuda.synchronize()
    ls = [l for l, _ in PAIRS]
    ms = [m for _, m in PAIRS]
    we, wb = oracle.shear_eb_entries(t, p, w, g1, g2, ls, ms)
    for name, got, want in (("E", e, we), ("B", b, wb)):
        cl = lib.cl_from_alm(got, LMAX).cpu().numpy()
        rel = np.abs(sampled(lib, got, PAIRS) - want) / np.sqrt(cl[ls])
        say(f"shear {name}: sampled entries, max |err| / rms_l = {rel.max():.3e}")
        assert rel.max() <= GATE


def test_interpolated_transform_at_maximum_lmax(lib):
    """App. A.2 at lmax 16383 (2000 nodes, 1-degree caps; two points inside the caps take the
    exact sum): sampled coefficients against the oracle's interpolated transform."""
    import torch
    from oracle import spline
    say(f"case: interpolated transform, 192 points, lmax {LMAX}, 2000 nodes")
    t, p, w = catalog()
    t = np.concatenate([t, [0.01, math.pi - 0.005]])
    p = np.concatenate([p, [1.1, 4.0]])
    w = np.concatenate([w, [0.9, 1.2]])
    nodes, cut = 2000, math.radians(1.0)
    a = lib.alm_from_points_spline(*dev(t, p, w), LMAX, nodes, cut)
    torch.cuda.synchronize()
    pairs = [(2, 0), (5000, 17), (8191, 8191), (16383, 0), (16383, 8191), (16383, 16383)]
    want = spline.alm_spline_entries(t, p, w, LMAX, nodes, cut, pairs)
    cl = lib.cl_from_alm(a, LMAX).cpu().numpy()
    rel = np.abs(sampled(lib, a, pairs) - want) / np.sqrt(cl[[l for l, _ in pairs]])
    say(f"spline: sampled entries, max |err| / rms_l = {rel.max():.3e}")
    assert rel.max() <= GATE


def test_point_count_above_2_to_31(lib, oracle):
    import torch
    from conftest import per_l_rel_err
    from paper_2312_12285_amd.synth import masked_galaxies, shear_components
    lmax, B, K, r = 64, 2 ** 20, 2048, 777
    n = K * B + r
    say(f"case: n = {n} (2^31 + {r}): 2^20 masked galaxies x {K} + {r}, lmax {lmax}")
    g = masked_galaxies(B, seed_pos=81, seed_w=82)
    g1, g2 = shear_components(B, seed=83)
    base = dev(g.theta, g.phi, g.w, g1, g2)
    big = []
    for x in base:
        y = torch.empty(n, dtype=torch.float64, device=x.device)
        y[: K * B].view(K, B).copy_(x.expand(K, B))
        y[K * B:].copy_(x[:r])
        big.append(y)
    del base

    a = lib.alm_from_points(*big[:3], lmax)
    torch.cuda.synchronize()
    want = K * oracle.alm_from_points(g.theta, g.phi, g.w, lmax) + \
        oracle.alm_from_points(g.theta[:r], g.phi[:r], g.w[:r], lmax)
    err = per_l_rel_err(lib.as_complex(a).cpu().numpy(), want, lmax)
    say(f"fp64: max per-l err {err.max():.3e}")
    assert err.max() <= GATE

    e, b = lib.shear_alm_from_points(*big, lmax)
    torch.cuda.synchronize()
    del big
    torch.cuda.empty_cache()
    we, wb = oracle.shear_eb(g.theta, g.phi, g.w, g1, g2, lmax)
    fe, fb = oracle.shear_eb(g.theta[:r], g.phi[:r], g.w[:r], g1[:r], g2[:r], lmax)
    for name, got, want in (("E", e, K * we + fe), ("B", b, K * wb + fb)):
        err = per_l_rel_err(lib.as_complex(got).cpu().numpy(), want, lmax)[2:]   # l < 2 is zero
        say(f"shear {name}: max per-l err {err.max():.3e}")
        assert err.max() <= GATE


def test_coupling_matrix_at_maximum_lmax(lib, oracle):
    """M at lmax 16383 for a window band-limited to l = 1024 (M[l][l'] = 0 for |l - l'| > 1024,
    which the GPU must write as zeros): sampled rows against the oracle (<= 1e-12 relative,
    element by element), and the transpose relation (2l+1) M[l][l'] = (2l'+1) M[l'][l] over the
    whole matrix."""
    import torch
    from paper_2312_12285_amd.synth import window_spectrum
    say(f"case: coupling matrix, lmax {LMAX}, window to l = 1024")
    W = window_spectrum(1024, seed=5)
    M = lib.coupling_matrix(dev(W)[0], LMAX)
    torch.cuda.synchronize()
    rows = [0, 1, 63, 64, 1100, 8190, 8191, 16382, 16383]
    ref = oracle.coupling_rows(W, LMAX, rows)
    got = M[rows].cpu().numpy()
    bad = np.abs(got - ref) > 1e-12 * np.abs(ref)
    rel = np.abs(got - ref)[ref != 0] / np.abs(ref[ref != 0])
    say(f"coupling: sampled rows, max rel err {rel.max():.3e}, {int(bad.sum())} entries off")
    assert not bad.any()
    l = torch.arange(LMAX + 1, dtype=torch.float64, device=M.device)
    sym = (2 * l[:, None] + 1) * M
    asym = (sym - sym.T).abs().max().item()
    say(f"coupling: transpose relation, max |diff| {asym:.3e} of max {sym.abs().max().item():.3e}")
    assert asym <= 1e-13 * sym.abs().max().item()


def test_multi_weight_at_maximum_lmax(lib, oracle):
    """16 weight vectors on the split-bf16 matrix-core path at lmax 16383 (34 GB of output):
    sampled coefficients of two vectors against the oracle (<= 1e-4 of the l-rms, the form's
    stated accuracy), and vector 0 against the FP64 path over every coefficient."""
    import torch
    say(f"case: 190 positions x 16 weight vectors, lmax {LMAX}, split-bf16 MFMA")
    t, p, _ = catalog()
    W = np.random.default_rng(74).uniform(0.5, 1.5, (16, t.size))
    td, pd, wd = dev(t, p, W)
    out = lib.alm_from_points(td, pd, wd, LMAX, options=lib.opts(precision=lib.BF16X3, n_weights=16))
    torch.cuda.synchronize()
    ls = np.array([l for l, _ in PAIRS]); ms = np.array([m for _, m in PAIRS])
    for v in (0, 15):
        want = oracle.alm_entries(t, p, W[v], ls, ms)
        cl = lib.cl_from_alm(out[v], LMAX).cpu().numpy()
        rel = np.abs(sampled(lib, out[v], PAIRS) - want) / np.sqrt(cl[ls])
        say(f"bf16x3 vector {v}: sampled entries, max |err| / rms_l = {rel.max():.3e}")
        assert rel.max() <= 1e-4
    a64 = lib.alm_from_points(td, pd, wd[0].contiguous(), LMAX)
    torch.cuda.synchronize()
    g = (torch.linalg.norm(out[0] - a64) / torch.linalg.norm(a64)).item()
    say(f"bf16x3 vs FP64, vector 0: global {g:.3e}")
    assert g <= 1e-4
    del out, a64
    torch.cuda.empty_cache()


def test_fp32_at_maximum_lmax(lib):
    """The FP32 recurrence at lmax 16383 against the FP64 path: x = cos(theta) and the step
    coefficients carry 2^-24 relative rounding, which shifts the phase of P_l by ~l 2^-24, so
    the error at degree l is bounded by a small multiple of (l+1) 2^-24 (norm over m at each l)."""
    import torch
    say(f"case: 190 full-sky points, lmax {LMAX}, FP32 against FP64")
    t, p, w = catalog()
    d = dev(t, p, w)
    a64 = lib.alm_from_points(*d, LMAX)
    a32 = lib.alm_from_points(*d, LMAX, options=lib.opts(precision=lib.FP32))
    torch.cuda.synchronize()
    num = lib.cl_from_alm(a32 - a64, LMAX).cpu().numpy()
    den = lib.cl_from_alm(a64, LMAX).cpu().numpy()
    err = np.sqrt(num / den)
    l = np.arange(LMAX + 1)
    ratio = err / ((l + 1) * 2.0 ** -24)
    say(f"fp32: per-l err at l = 64/1024/4096/16383: {err[64]:.1e} {err[1024]:.1e} {err[4096]:.1e} "
        f"{err[LMAX]:.1e}; max err / ((l+1) 2^-24) = {ratio.max():.2f} at l = {ratio.argmax()}")
    assert np.all(err <= np.maximum(1e-6, 8 * (l + 1) * 2.0 ** -24))
