"""GPU interpolated transform (App. A.2) against the oracle's interpolated transform.

The node counts cover both paths of the stable sort into intervals (one LDS
window of bucket counters up to 16384 nodes, several windows above).  Both
evaluate the same approximation (same nodes, same Hermite basis, same polar
split), so they agree to rounding: gate 1e-10 per-l norm-wise relative
(the direct path's gate), element-wise 1e-10 of the l-row norm.  Also: the
spline path converges to the exact GPU direct sum like h^4, a cut that makes
every point polar reduces it to the direct sum, empty input, argument checks,
repeated calls are bitwise equal, and a call captured into a HIP graph (with a
caller workspace) replays bitwise equal to eager calls.
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
    return np.sqrt(num / np.maximum(den, 1e-300)), np.sqrt(den)


@pytest.mark.parametrize("n,lmax,n_nodes,cut_deg,seed", [(20_000, 64, 200, 5.0, 1), (7_001, 100, 37, 20.0, 2),
                                                          (30_000, 40, 513, 0.5, 3), (5_000, 3, 2, 30.0, 4),
                                                          (40_000, 12, 20_000, 2.0, 5)])
def test_spline_matches_oracle(lib, oracle, n, lmax, n_nodes, cut_deg, seed):
    from oracle import spline
    from paper_2312_12285_amd import synth
    t, p = synth.uniform_sphere(n, seed)
    w = synth.lognormal_weights(n, 0.3, seed + 100)
    cut = math.radians(cut_deg)
    print(f"spline parity n {n} lmax {lmax} nodes {n_nodes} cut {cut_deg} deg", flush=True)
    got = cplx(lib.alm_from_points_spline(dev(t), dev(p), dev(w), lmax, n_nodes, cut))
    want = spline.alm_spline(t, p, w, lmax, n_nodes, cut)
    err, norm = per_l(got, want, lmax)
    print(f"  per-l max rel err {err.max():.3e}", flush=True)
    assert err.max() <= 1e-10
    L = np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])
    assert np.all(np.abs(got - want) <= 1e-10 * norm[L] + 1e-300)


def test_spline_converges_to_the_direct_sum(lib):
    from paper_2312_12285_amd import synth
    t, p = synth.uniform_in_mask(40_000, 5)
    w = np.ones(t.size)
    lmax = 48
    d = cplx(lib.alm_from_points(dev(t), dev(p), dev(w), lmax))
    errs = []
    for nodes in (96, 192, 384):
        a = cplx(lib.alm_from_points_spline(dev(t), dev(p), dev(w), lmax, nodes, math.radians(2.0)))
        errs.append(np.abs(a - d).max() / np.abs(d).max())
    print("spline vs direct:", errs, flush=True)
    assert errs[0] / errs[1] > 11 and errs[1] / errs[2] > 11


def test_all_polar_is_the_direct_sum(lib):
    from paper_2312_12285_amd import synth
    t, p = synth.uniform_sphere(10_000, 6)
    w = synth.lognormal_weights(t.size, 0.3, 7)
    lmax = 30
    d = cplx(lib.alm_from_points(dev(t), dev(p), dev(w), lmax))
    a = cplx(lib.alm_from_points_spline(dev(t), dev(p), dev(w), lmax, 8, math.pi / 2 - 1e-12))
    assert np.abs(a - d).max() <= 1e-12 * np.abs(d).max()


def test_empty_and_argument_checks(lib):
    import torch
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    out = lib.alm_from_points_spline(e, e, e, 10, 16, 0.1)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    x = dev(np.array([1.0]))
    for nodes, cut in ((1, 0.1), (16, 0.0), (16, math.pi / 2), (70000, 0.1)):
        with pytest.raises(lib.PtalmError):
            lib.alm_from_points_spline(x, x, x, 10, nodes, cut)


def test_timing_option_times_the_binning_kernel(lib):
    """opts.timing records events around the binning kernel; the result is unchanged."""
    from paper_2312_12285_amd import synth
    t, p = synth.uniform_sphere(20_000, 31)
    w = synth.lognormal_weights(20_000, 0.3, 32)
    a = cplx(lib.alm_from_points_spline(dev(t), dev(p), dev(w), 48, 120, 0.05))
    b = cplx(lib.alm_from_points_spline(dev(t), dev(p), dev(w), 48, 120, 0.05, options=lib.opts(timing=1)))
    ms = lib.last_timing_ms()
    print(f"binning kernel {ms:.3f} ms", flush=True)
    assert ms > 0.0
    assert np.array_equal(a, b)


def test_spline_is_deterministic_and_capturable(lib):
    """The stable sort keeps the input order inside each interval, so repeated calls give the
    same bits (polar caps included); with a caller workspace and prepared tables the call
    allocates and synchronizes nothing, and a captured graph replays bitwise equal to eager
    calls, with eager calls on the same workspace between the replays."""
    import torch
    from paper_2312_12285_amd import synth
    n, lmax, nodes, cut = 60_000, 96, 300, math.radians(3.0)
    t, p = synth.uniform_in_mask(n, 51)          # the mask reaches the north cap: polar points too
    w = synth.lognormal_weights(n, 0.3, 52)
    T, P, W = dev(t), dev(p), dev(w)
    first = lib.alm_from_points_spline(T, P, W, lmax, nodes, cut).clone()
    for _ in range(3):
        again = lib.alm_from_points_spline(T, P, W, lmax, nodes, cut)
        torch.cuda.synchronize()
        assert torch.equal(first, again)
    lib.prepare_spline_call(n, lmax, nodes)
    ws = torch.empty(lib.spline_workspace_bytes(n, lmax, nodes), dtype=torch.uint8, device="cuda")
    eager = lib.alm_from_points_spline(T, P, W, lmax, nodes, cut, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(eager, first)
    out = torch.empty_like(first)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        lib.alm_from_points_spline(T, P, W, lmax, nodes, cut, out=out, workspace=ws)
    for k in range(4):
        out.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, first), f"replay {k}"
        lib.alm_from_points_spline(T, P, W, lmax, nodes, cut, workspace=ws)    # eager work in between
        torch.cuda.synchronize()


def test_phase_periodicity(lib):
    """phi and phi + 2 pi k (k = -3 .. 5, negative angles included) give the same a_lm: the
    binning reduces m0 phi / (2 pi) modulo 1 itself."""
    from paper_2312_12285_amd import synth
    t, p = synth.uniform_sphere(30_000, 41)
    w = synth.lognormal_weights(30_000, 0.3, 42)
    k = np.random.default_rng(43).integers(-3, 6, size=p.size)
    a = cplx(lib.alm_from_points_spline(dev(t), dev(p), dev(w), 200, 400, 0.05))
    b = cplx(lib.alm_from_points_spline(dev(t), dev(p + 2 * math.pi * k), dev(w), 200, 400, 0.05))
    err, norm = per_l(b, a, 200)
    print(f"phase periodicity: per-l max rel diff {err.max():.3e}", flush=True)
    assert err.max() <= 1e-12
