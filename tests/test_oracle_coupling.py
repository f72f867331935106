"""Pins of the mode-coupling oracle (Sec. 2.1 eq. chat, eq. mode_coupling; App. B).

The oracle's 3j symbols come from the closed form; they are pinned to a
textbook table, to the paper's own recurrence and terminal case (App. B), to
the Gaunt integral of three Legendre polynomials by Gauss-Legendre quadrature
(scipy, no 3j involved), and to their orthogonality sum.  The coupling matrix
is pinned to its meaning: M_ll' = (2l+1)^-1 sum_m sum_m' |int w Y_l'm' Y*_lm|^2
computed by quadrature with scipy's Y_lm for a band-limited window, to the full
sky (M = identity) and to its row sums (the shot-noise bracket of Sec. 2.1).
The bandpower algebra is pinned by what it is built to do: decoupling returns
piecewise-constant spectra exactly, and the normalised convention leaves a
constant (shot-noise) spectrum unchanged.
"""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre, roots_legendre, sph_harm_y


def test_threej_textbook_values(oracle):
    table = {(1, 1, 0): -1 / math.sqrt(3), (1, 1, 2): math.sqrt(2 / 15), (2, 2, 2): -math.sqrt(2 / 35),
             (1, 2, 3): -math.sqrt(3 / 35), (2, 2, 0): 1 / math.sqrt(5), (0, 0, 0): 1.0}
    for (a, b, c), v in table.items():
        for p in ((a, b, c), (b, c, a), (c, a, b), (b, a, c)):      # invariant under permutations
            assert abs(oracle.threej000(*p) - v) < 1e-15


def test_threej_zero_cases(oracle):
    assert oracle.threej000(1, 1, 1) == 0.0            # odd L
    assert oracle.threej000(2, 3, 6) == 0.0            # triangle violated
    assert oracle.threej000(5, 2, 2) == 0.0


def test_threej_paper_terminal_and_recurrence(oracle):
    """App. B: (l l 0; 000) = (-1)^l / sqrt(2l+1), and the ratio recurrence in (l2, l3)."""
    for l in (0, 1, 2, 7, 50, 333, 1000):
        assert abs(oracle.threej000(l, l, 0) - (-1) ** l / math.sqrt(2 * l + 1)) <= 1e-14 / math.sqrt(2 * l + 1)
    rng = np.random.default_rng(3)
    checked = 0
    while checked < 300:
        l1, l2, l3 = (int(v) for v in rng.integers(0, 400, 3))
        L = l1 + l2 + l3
        if L % 2 or l3 < 1 or not (abs(l2 + 1 - (l3 - 1)) <= l1 <= l2 + l3) or abs(l2 - l3) > l1:
            continue
        lhs = oracle.threej000(l1, l2, l3)
        rhs = math.sqrt((L - 2 * l2 - 1) * (L - 2 * l3 + 2) / ((L - 2 * l2) * (L - 2 * l3 + 1))) \
            * oracle.threej000(l1, l2 + 1, l3 - 1)
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
        checked += 1


def test_threej_gaunt_integral_quadrature(oracle):
    """int_{-1}^{1} P_l1 P_l2 P_l3 dx = 2 (l1 l2 l3; 000)^2 (Legendre product integral)."""
    x, g = roots_legendre(80)
    for l1, l2, l3 in [(3, 4, 5), (10, 12, 6), (20, 25, 31), (40, 40, 2), (7, 30, 37), (50, 35, 21)]:
        integral = float(np.sum(g * eval_legendre(l1, x) * eval_legendre(l2, x) * eval_legendre(l3, x)))
        want = 2 * oracle.threej000(l1, l2, l3) ** 2
        assert abs(integral - want) < 1e-11 * want      # quadrature of scipy's P_l: ~1e-14 absolute


def test_threej_orthogonality(oracle):
    for l1, l2 in [(0, 0), (3, 5), (17, 40), (100, 100), (150, 60)]:
        s = sum((2 * l3 + 1) * oracle.threej000(l1, l2, l3) ** 2 for l3 in range(abs(l1 - l2), l1 + l2 + 1))
        assert abs(s - 1.0) < 1e-13


def test_coupling_full_sky_is_identity(oracle):
    W = np.zeros(50)
    W[0] = 4 * math.pi                  # w = 1 everywhere: w_00 = sqrt(4 pi)
    M = oracle.coupling_matrix(W, 200)
    assert np.abs(M - np.eye(201)).max() < 1e-14


def test_coupling_row_sums_shot_noise_bracket(oracle):
    """sum_l' M_ll' = sum_lambda (2 lambda+1) W_lambda / (4 pi) while l + lmax_w <= lmax."""
    rng = np.random.default_rng(5)
    W = rng.uniform(0, 1, 21) * np.exp(-np.arange(21) / 5.0)
    M = oracle.coupling_matrix(W, 120)
    bracket = np.sum((2 * np.arange(21) + 1) * W) / (4 * math.pi)
    rows = M.sum(axis=1)[:100]
    assert np.abs(rows / bracket - 1).max() < 1e-13
    # M_ll' / (2l'+1) is symmetric
    S = M / (2 * np.arange(121) + 1)[None, :]
    assert np.abs(S - S.T).max() < 1e-15 * np.abs(S).max()


def _quadrature_grid(lmax):
    x, g = roots_legendre(lmax + 1)
    nphi = 2 * lmax + 2
    phi = 2 * math.pi * np.arange(nphi) / nphi
    th = np.arccos(x)
    TH, PH = np.meshgrid(th, phi, indexing="ij")
    Wq = np.outer(g, np.full(nphi, 2 * math.pi / nphi))
    return TH, PH, Wq


def test_coupling_equals_its_definition_by_quadrature(oracle):
    """M_ll' from eq. chat against (2l+1)^-1 sum_{m, m'} |int w Y_l'm' Y*_lm dOmega|^2 for a
    band-limited real window w (l <= 3); integrals exact on a Gauss-Legendre x uniform-phi grid."""
    lw, lmax = 3, 8
    TH, PH, Wq = _quadrature_grid(lw + 2 * lmax + 2)
    rng = np.random.default_rng(11)
    w = np.ones_like(TH)
    for l in range(1, lw + 1):
        for m in range(0, l + 1):
            c = rng.normal() * 0.3
            y = sph_harm_y(l, m, TH, PH)
            w += c * (y.real if m == 0 else 2 * y.real)
    # window spectrum W_lambda from w's own harmonic coefficients (quadrature)
    Wl = np.zeros(lw + 1)
    for lam in range(lw + 1):
        s = 0.0
        for m in range(-lam, lam + 1):
            a = np.sum(Wq * w * np.conj(sph_harm_y(lam, m, TH, PH)))
            s += abs(a) ** 2
        Wl[lam] = s / (2 * lam + 1)
    M = oracle.coupling_matrix(Wl, lmax)
    Y = {(l, m): sph_harm_y(l, m, TH, PH) for l in range(lmax + 1) for m in range(-l, l + 1)}
    for l in range(lmax + 1):
        for lp in range(lmax + 1):
            s = 0.0
            for m in range(-l, l + 1):
                for mp in range(-lp, lp + 1):
                    s += abs(np.sum(Wq * w * Y[(lp, mp)] * np.conj(Y[(l, m)]))) ** 2
            assert abs(s / (2 * l + 1) - M[l, lp]) < 1e-12 * max(1.0, abs(M[l, lp]))


def test_bandpowers_recover_piecewise_constant_and_shot_noise(oracle):
    rng = np.random.default_rng(7)
    lw, lmax, dl = 30, 200, 10
    W = np.abs(rng.normal(size=lw + 1)) * np.exp(-np.arange(lw + 1) / 8.0)
    W[0] = 4 * math.pi * 0.4
    M = oracle.coupling_matrix(W, lmax)
    theta, chi = oracle.bin_matrix(lmax, dl)
    nb = theta.shape[0]
    # decoupling: a spectrum constant within each bin comes back exactly
    cb_true = rng.uniform(1, 3, nb)
    cl_true = chi @ cb_true
    cl_hat = M @ cl_true                          # expectation of the pseudo-spectrum (eq. chat)
    cb, window, Mbb = oracle.decoupled_bandpowers(cl_hat, M, theta, chi)
    assert np.abs(cb - cb_true).max() < 1e-11 * cb_true.max()
    assert np.abs(window @ cl_true - cb_true).max() < 1e-11 * cb_true.max()
    # normalised convention: a constant spectrum keeps its amplitude away from the edge
    c0 = 2.5
    cbn, window_n, N = oracle.normalized_bandpowers(M @ np.full(lmax + 1, c0), M, theta, W)
    far = (np.arange(nb) + 1) * dl + lw <= lmax
    assert np.abs(cbn[far] - c0).max() < 1e-12 * c0
    assert np.all(window_n >= 0)


def test_coupling_rows_match_full_matrix(oracle):
    """The row sampler used for large-lmax checks returns rows of the same matrix."""
    W = np.abs(np.random.default_rng(11).normal(size=91))
    M = oracle.coupling_matrix(W, 60)
    rows = [0, 1, 7, 33, 60]
    assert np.array_equal(oracle.coupling_rows(W, 60, rows), M[rows])
    with pytest.raises(ValueError):
        oracle.coupling_rows(W, 60, [61])

