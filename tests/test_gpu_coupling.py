"""GPU mode coupling and bandpowers (Sec. 2.1 eq. chat, eq. mode_coupling) against the oracle.

Gates: coupling matrix element-wise <= 1e-12 relative (all entries are sums of
positive terms; the kernel's 3j squares come from products of rational
factors, ~1e-16 each); window shot noise 1e-13; bandpowers 1e-9 relative to
the largest bandpower (the decoupling solve amplifies rounding by the
condition number of Mbb).  Includes the full path from two catalogs: a_lm of
data and randoms, FKP field, C^_l, W_l with shot noise removed, M, and both
bandpower conventions, against the same path in the oracle.
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


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("lmax,lmax_w", [(0, 0), (1, 3), (64, 128), (200, 400), (150, 60)])
def test_coupling_matrix_matches_oracle(lib, oracle, lmax, lmax_w):
    rng = np.random.default_rng(lmax + 17)
    W = np.abs(rng.normal(size=lmax_w + 1)) * np.exp(-np.arange(lmax_w + 1) / 20.0)
    W[0] = 4 * math.pi * 0.4
    M = host(lib.coupling_matrix(dev(W), lmax))
    ref = oracle.coupling_matrix(W, lmax)
    nz = ref != 0
    assert np.array_equal(M == 0, ~nz)
    rel = np.abs(M[nz] - ref[nz]) / ref[nz]
    print(f"coupling lmax {lmax} lmax_w {lmax_w}: max rel err {rel.max() if rel.size else 0:.3e}", flush=True)
    assert rel.size == 0 or rel.max() <= 1e-12


def test_coupling_capture_and_table_cache(lib, oracle):
    """The lmax-only tables are kept per (device, lmax) after the first call outside
    capture; a call captured for an lmax not seen before computes them into its own
    scratch.  Graph replays of both forms equal the eager call bit for bit, with
    eager work between the replays, and match the oracle."""
    import torch
    lmax, lmax_w = 333, 700      # an lmax no other test uses, so the first call below is captured
    rng = np.random.default_rng(333)
    W = np.abs(rng.normal(size=lmax_w + 1)) * np.exp(-np.arange(lmax_w + 1) / 30.0)
    W[0] = 4 * math.pi * 0.3
    Wd = dev(W)
    out = torch.empty((lmax + 1, lmax + 1), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    graphs = []
    for form in ("tables in the call's scratch", "kept tables"):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            lib.coupling_matrix(Wd, lmax, out=out)
        graphs.append((form, g))
        if form.startswith("tables"):
            eager = lib.coupling_matrix(Wd, lmax)     # first call outside capture: keeps the tables
            torch.cuda.synchronize()
    for form, g in graphs:
        for rep in range(3):
            out.fill_(-1.0)                           # eager work between replays
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(out, eager), f"{form}: replay {rep} differs from the eager call"
    ref = oracle.coupling_matrix(W, lmax)
    M = host(eager)
    nz = ref != 0
    assert np.array_equal(M == 0, ~nz)
    assert (np.abs(M[nz] - ref[nz]) / ref[nz]).max() <= 1e-12


def test_release_cache_frees_and_rebuilds_coupling_tables(lib):
    """ptalm_release_cache frees the kept lmax-only coupling tables (and reports success);
    the next call for that lmax builds them again and gives the same matrix bit for bit."""
    import torch
    lmax, lmax_w = 257, 514
    W = np.exp(-np.arange(lmax_w + 1) / 40.0)
    W[0] = 4 * math.pi * 0.5
    Wd = dev(W)
    first = lib.coupling_matrix(Wd, lmax)
    torch.cuda.synchronize()
    lib.release_cache()
    again = lib.coupling_matrix(Wd, lmax)
    torch.cuda.synchronize()
    assert torch.equal(first, again)
    lib.release_cache()                      # twice in a row: nothing left to free, still OK
    lib.release_cache()


def test_full_sky_identity(lib):
    W = np.zeros(600)
    W[0] = 4 * math.pi
    M = host(lib.coupling_matrix(dev(W), 300))
    assert np.abs(M - np.eye(301)).max() < 1e-14


def test_shot_noise_and_subtraction(lib, oracle):
    import torch
    rng = np.random.default_rng(4)
    w = rng.lognormal(0.0, 0.3, 100_003)
    alpha = dev(np.array([0.37]))
    s = host(lib.window_shot_noise(dev(w), alpha))[0]
    want = 0.37 ** 2 * math.fsum(w * w) / (4 * math.pi)
    assert abs(s - want) <= 1e-13 * want
    W = np.abs(rng.normal(size=81)) + 1.0
    M = host(lib.coupling_matrix(dev(W), 40, shot=dev(np.array([s]))))
    ref = oracle.coupling_matrix(W - s, 40)
    assert np.abs(M - ref).max() <= 1e-12 * np.abs(ref).max()


def test_bandpowers_match_oracle(lib, oracle):
    rng = np.random.default_rng(9)
    lmax, lw, dl, lmin = 200, 400, 10, 2
    W = np.abs(rng.normal(size=lw + 1)) * np.exp(-np.arange(lw + 1) / 15.0)
    W[0] = 4 * math.pi * 0.35
    Mh = oracle.coupling_matrix(W, lmax)
    cl_hat = Mh @ (1.0 + 50.0 / (np.arange(lmax + 1) + 5.0))
    Md = dev(Mh)
    theta, chi = oracle.bin_matrix(lmax, dl, lmin)
    cb, window = lib.bandpowers(dev(cl_hat), Md, lmax, dl, lmin=lmin, mode=0)
    cb_ref, win_ref, _ = oracle.decoupled_bandpowers(cl_hat, Mh, theta, chi)
    assert lib.bandpower_count(lmax, lmin, dl) == theta.shape[0]
    assert np.abs(host(cb) - cb_ref).max() <= 1e-9 * np.abs(cb_ref).max()
    assert np.abs(host(window) - win_ref).max() <= 1e-9 * np.abs(win_ref).max()
    cbn, winn = lib.bandpowers(dev(cl_hat), Md, lmax, dl, lmin=lmin, mode=1, Wl=dev(W))
    cbn_ref, winn_ref, _ = oracle.normalized_bandpowers(cl_hat, Mh, theta, W)
    assert np.abs(host(cbn) - cbn_ref).max() <= 1e-12 * np.abs(cbn_ref).max()
    assert np.abs(host(winn) - winn_ref).max() <= 1e-12 * np.abs(winn_ref).max()


def test_bandpower_argument_checks(lib):
    M = dev(np.eye(11))
    c = dev(np.ones(11))
    for kw in (dict(delta_l=20), dict(delta_l=0), dict(delta_l=2, lmin=11)):
        with pytest.raises(lib.PtalmError):
            lib.bandpowers(c, M, 10, **kw)
    with pytest.raises(lib.PtalmError):
        lib.bandpowers(c, M, 10, 2, mode=1)           # normalised without W


def test_two_catalog_path_to_bandpowers(lib, oracle):
    """Data and randoms -> FKP field -> C^_l, W_l (shot noise removed) -> M -> bandpowers."""
    import torch
    from paper_2312_12285_amd.synth import masked_galaxies, masked_randoms
    lmax, lw, dl, lmin = 96, 192, 8, 2
    g = masked_galaxies(20_000, seed_pos=71, seed_w=72)
    r = masked_randoms(100_000, seed=73)
    ad = lib.alm_from_points(dev(g.theta), dev(g.phi), dev(g.w), lw)
    ar = lib.alm_from_points(dev(r.theta), dev(r.phi), dev(r.w), lw)
    delta, window, alpha = lib.fkp_fields(ad, ar, lw)
    cl_all = lib.cl_from_alm(delta, lw)
    Wl = lib.cl_from_alm(window, lw)
    shot = lib.window_shot_noise(dev(r.w), alpha)
    M = lib.coupling_matrix(Wl, lmax, shot=shot)
    cl_hat = cl_all[:lmax + 1].contiguous()
    Wsub = (Wl - shot).contiguous()
    cb, win = lib.bandpowers(cl_hat, M, lmax, dl, lmin=lmin, mode=0)
    cbn, winn = lib.bandpowers(cl_hat, M, lmax, dl, lmin=lmin, mode=1, Wl=Wsub)
    torch.cuda.synchronize()
    # the same path in the oracle
    add = oracle.alm_from_points(g.theta, g.phi, g.w, lw)
    arr = oracle.alm_from_points(r.theta, r.phi, r.w, lw)
    a = add[0].real / arr[0].real
    cl_ref = oracle.cl_from_alm(add - a * arr, lw)[:lmax + 1]
    W_ref = oracle.cl_from_alm(a * arr, lw) - a * a * math.fsum(r.w * r.w) / (4 * math.pi)
    M_ref = oracle.coupling_matrix(W_ref, lmax)
    theta, chi = oracle.bin_matrix(lmax, dl, lmin)
    cb_ref, _, _ = oracle.decoupled_bandpowers(cl_ref, M_ref, theta, chi)
    cbn_ref, _, _ = oracle.normalized_bandpowers(cl_ref, M_ref, theta, W_ref)
    errd = np.abs(host(cb) - cb_ref).max() / np.abs(cb_ref).max()
    errn = np.abs(host(cbn) - cbn_ref).max() / np.abs(cbn_ref).max()
    print(f"two-catalog bandpowers: decoupled {errd:.2e}, normalised {errn:.2e}", flush=True)
    assert errd <= 1e-8 and errn <= 1e-9


@pytest.mark.parametrize("lmax,dl,lmin", [(0, 1, 0), (126, 1, 0), (127, 1, 0), (128, 1, 0), (150, 1, 11), (139, 1, 0), (140, 1, 0), (299, 1, 0),
                                          (1023, 1, 0), (700, 3, 5)])
def test_bandpower_solve_sizes(lib, oracle, lmax, dl, lmin):
    """The decoupling solve at bin counts on both sides of the in-register (128) and in-LDS (140)
    factorisation limits and
    at the 1024-bin maximum, on a well-conditioned synthetic coupling matrix."""
    rng = np.random.default_rng(lmax + dl)
    n1 = lmax + 1
    Mh = np.eye(n1) * (1.0 + rng.random(n1)) + rng.random((n1, n1)) * (0.5 / n1)
    cl_hat = 1.0 + rng.random(n1)
    theta, chi = oracle.bin_matrix(lmax, dl, lmin)
    print(f"bandpower solve lmax {lmax} delta_l {dl} lmin {lmin}: nb {theta.shape[0]}", flush=True)
    cb, window = lib.bandpowers(dev(cl_hat), dev(Mh), lmax, dl, lmin=lmin, mode=0)
    cb_ref, win_ref, _ = oracle.decoupled_bandpowers(cl_hat, Mh, theta, chi)
    assert np.abs(host(cb) - cb_ref).max() <= 1e-12 * np.abs(cb_ref).max()
    assert np.abs(host(window) - win_ref).max() <= 1e-12 * np.abs(win_ref).max()


def test_coupling_and_bandpowers_full_size(lib, oracle):
    """Full size of the coupling workload (lmax 3072 from W_l to 6144): sampled rows of M
    against the oracle row by row (every tile column, the diagonal block, both parities,
    the last rows), and both bandpower conventions against the oracle's bandpower algebra
    applied to the same M."""
    import torch
    from paper_2312_12285_amd.synth import window_spectrum
    lmax, lw, dl = 3072, 6144, 25
    W = window_spectrum(lw, seed=5)
    Wd = dev(W)
    M = lib.coupling_matrix(Wd, lmax)
    rows = [0, 1, 2, 63, 64, 65, 1000, 2047, 3071, 3072]
    Mh = host(M)
    ref = oracle.coupling_rows(W, lmax, rows)
    rel = np.abs(Mh[rows] - ref) / np.abs(ref)
    print(f"coupling lmax {lmax}: sampled-row max rel err {rel.max():.3e}", flush=True)
    assert rel.max() <= 1e-12
    # the transpose relation of the definition: (2l+1) M[l][l'] = (2l'+1) M[l'][l]
    l = np.arange(lmax + 1.0)
    sym = (2 * l[:, None] + 1) * Mh
    assert np.abs(sym - sym.T).max() <= 1e-13 * np.abs(sym).max()
    rng = np.random.default_rng(6)
    cl_hat = Mh @ (1.0 + 30.0 / (l + 10.0)) + 1e-3 * rng.random(lmax + 1)
    theta, chi = oracle.bin_matrix(lmax, dl, 2)
    cb, win = lib.bandpowers(dev(cl_hat), M, lmax, dl, lmin=2, mode=0)
    cbn, winn = lib.bandpowers(dev(cl_hat), M, lmax, dl, lmin=2, mode=1, Wl=Wd)
    torch.cuda.synchronize()
    cb_ref, win_ref, _ = oracle.decoupled_bandpowers(cl_hat, Mh, theta, chi)
    cbn_ref, winn_ref, _ = oracle.normalized_bandpowers(cl_hat, Mh, theta, W)
    assert np.abs(host(cb) - cb_ref).max() <= 1e-9 * np.abs(cb_ref).max()
    assert np.abs(host(win) - win_ref).max() <= 1e-9 * np.abs(win_ref).max()
    assert np.abs(host(cbn) - cbn_ref).max() <= 1e-12 * np.abs(cbn_ref).max()
    assert np.abs(host(winn) - winn_ref).max() <= 1e-12 * np.abs(winn_ref).max()
