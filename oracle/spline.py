"""Oracle of the interpolated transform of App. A.2 (test infrastructure only).

Plain numpy, written from the appendix in its order and notation:

* y_lm(x) = Y_lm(theta, 0) at the spline nodes, from the oracle's direct sum
  (one unit-weight point at phi = 0 per node, which returns Y*_lm = Y_lm there);
* y'_lm(x) from the derivative relation of App. A.1 (eq. after the l-recurrence),
  carried to the orthonormal functions of Sec. 2.2;
* the cubic Hermite basis c_j0..c_j3 of App. A.2 on each interval
  [x_j, x_{j+1}), with the (x_{j+1} - x_j) factors on the derivative terms
  (the expanded sum of App. A.2 drops them; the spline's definition has them);
* v_ja^(m) = sum_r w_r e^{-i m phi_r} c_ja(x_r) over the points of interval j;
* a_lm = sum_j [v_j0 y(x_j) + v_j1 dx_j y'(x_j) + v_j2 y(x_{j+1}) + v_j3 dx_j y'(x_{j+1})]
  plus, for the points outside the spline region, the exact sum (App. A.2
  splits polar points off; here they take the direct sum instead of a rotation).

Nodes: the paper leaves their placement open.  Here n_nodes nodes are uniform
in theta over [theta_cut, pi - theta_cut], x_j = cos(pi - theta_cut - j h)
ascending in x.  Points with theta < theta_cut or theta > pi - theta_cut are
polar.  A point exactly on an interior node belongs to the interval above it.
"""
import math

import numpy as np

from . import ref


def nodes(n_nodes: int, theta_cut: float):
    """(x_j ascending, theta_j descending, h) for n_nodes nodes uniform in theta."""
    if n_nodes < 2:
        raise ValueError("need at least two nodes")
    h = (math.pi - 2.0 * theta_cut) / (n_nodes - 1)
    th = math.pi - theta_cut - h * np.arange(n_nodes)
    return np.cos(th), th, h


def interval_of(theta, n_nodes: int, theta_cut: float):
    """Interval index j (x_j <= x < x_{j+1}) of each point, or -1 for polar points."""
    theta = np.asarray(theta, dtype=np.float64)
    _, _, h = nodes(n_nodes, theta_cut)
    u = (math.pi - theta_cut - theta) / h           # distance from node 0 in steps, along increasing x
    j = np.floor(u).astype(np.int64)
    j = np.minimum(j, n_nodes - 2)
    polar = (theta < theta_cut) | (theta > math.pi - theta_cut)
    return np.where(polar, -1, j)


def ylm_table(lmax: int, theta_nodes):
    """y_lm(x_j) for every node: [n_nodes, (lmax+1)(lmax+2)/2] real, healpy order."""
    out = np.empty((len(theta_nodes), ref.alm_size(lmax)))
    for j, t in enumerate(theta_nodes):
        out[j] = ref.alm_from_points(np.array([t]), np.zeros(1), np.ones(1), lmax).real
    return out


def dylm_table(lmax: int, x_nodes, y):
    """dy_lm/dx at the nodes from App. A.1's derivative relation.  For the paper's
    Pbar (the recurrence's normalisation) it reads (1-x^2) Pbar'_l = -l x Pbar_l
    + (l+m) sqrt((l-m)/(l+m)) Pbar_{l-1}; the orthonormal y_lm carry the extra
    sqrt((2l+1)/(4 pi)), so (1-x^2) y'_l = -l x y_l + sqrt((2l+1)/(2l-1))
    sqrt((l-m)(l+m)) y_{l-1}, with y_{m-1} = 0."""
    x = np.asarray(x_nodes, dtype=np.float64)
    dy = np.empty_like(y)
    for m in range(lmax + 1):
        base = m * (2 * lmax + 1 - m) // 2
        for l in range(m, lmax + 1):
            yl = y[:, base + l]
            prev = y[:, base + l - 1] if l > m else 0.0
            c = math.sqrt((2 * l + 1) / (2 * l - 1) * (l - m) * (l + m)) if l > m else 0.0
            dy[:, base + l] = (-l * x * yl + c * prev) / (1.0 - x * x)
    return dy


def hermite_basis(t):
    """c_j0..c_j3 of App. A.2 at t = (x - x_j)/(x_{j+1} - x_j): [4, n]."""
    t = np.asarray(t, dtype=np.float64)
    return np.stack([(2 * t + 1) * (1 - t) ** 2, t * (1 - t) ** 2, t * t * (3 - 2 * t), t * t * (t - 1)])


def binned_weights(theta, phi, w, lmax: int, n_nodes: int, theta_cut: float):
    """v[m, j, a] = sum over the points of interval j of w e^{-i m phi} c_ja(x): complex."""
    x_nodes, _, _ = nodes(n_nodes, theta_cut)
    j = interval_of(theta, n_nodes, theta_cut)
    keep = j >= 0
    jj = j[keep]
    x = np.cos(np.asarray(theta, dtype=np.float64)[keep])
    t = (x - x_nodes[jj]) / (x_nodes[jj + 1] - x_nodes[jj])
    c = hermite_basis(t)                                     # [4, n]
    ph = np.asarray(phi, dtype=np.float64)[keep]
    ww = np.asarray(w, dtype=np.float64)[keep]
    v = np.zeros((lmax + 1, n_nodes - 1, 4), dtype=np.complex128)
    for m in range(lmax + 1):
        e = ww * np.exp(-1j * m * ph)
        for a in range(4):
            z = e * c[a]
            v[m, :, a] = (np.bincount(jj, weights=z.real, minlength=n_nodes - 1)
                          + 1j * np.bincount(jj, weights=z.imag, minlength=n_nodes - 1))
    return v


def alm_spline(theta, phi, w, lmax: int, n_nodes: int, theta_cut: float, tables=None):
    """a_lm by the interpolated transform (healpy order, complex128)."""
    x_nodes, th_nodes, _ = nodes(n_nodes, theta_cut)
    if tables is None:
        y = ylm_table(lmax, th_nodes)
        dy = dylm_table(lmax, x_nodes, y)
    else:
        y, dy = tables
    v = binned_weights(theta, phi, w, lmax, n_nodes, theta_cut)
    dx = np.diff(x_nodes)                                    # x_{j+1} - x_j
    out = np.zeros(ref.alm_size(lmax), dtype=np.complex128)
    for m in range(lmax + 1):
        base = m * (2 * lmax + 1 - m) // 2
        sl = slice(base + m, base + lmax + 1)
        vm = v[m]
        out[sl] = (vm[:, 0] @ y[:-1, sl] + (vm[:, 1] * dx) @ dy[:-1, sl]
                   + vm[:, 2] @ y[1:, sl] + (vm[:, 3] * dx) @ dy[1:, sl])
    j = interval_of(theta, n_nodes, theta_cut)
    polar = j < 0
    if polar.any():
        th = np.asarray(theta)[polar]; ph = np.asarray(phi)[polar]; ww = np.asarray(w)[polar]
        out += ref.alm_from_points(th, ph, ww, lmax)
    return out


def alm_spline_entries(theta, phi, w, lmax: int, n_nodes: int, theta_cut: float, pairs):
    """Single coefficients a_lm of the interpolated transform, for sampled checks on
    catalogs too large for the full tables: the node values come from the oracle's
    single-entry sums, the binned weights are formed for each sampled m only."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    x_nodes, th_nodes, _ = nodes(n_nodes, theta_cut)
    j = interval_of(theta, n_nodes, theta_cut)
    keep = j >= 0
    jj = j[keep]
    x = np.cos(theta[keep])
    c = hermite_basis((x - x_nodes[jj]) / (x_nodes[jj + 1] - x_nodes[jj]))
    ph, ww = phi[keep], w[keep]
    dx = np.diff(x_nodes)
    polar = ~keep
    out = []
    vcache = {}
    for l, m in pairs:
        if m not in vcache:
            e = ww * np.exp(-1j * m * ph)
            v = np.zeros((n_nodes - 1, 4), dtype=np.complex128)
            for a in range(4):
                z = e * c[a]
                v[:, a] = (np.bincount(jj, weights=z.real, minlength=n_nodes - 1)
                           + 1j * np.bincount(jj, weights=z.imag, minlength=n_nodes - 1))
            vcache[m] = v
        v = vcache[m]
        ls = np.array([l, max(l - 1, m)])
        ms = np.array([m, m])
        yv = np.empty(n_nodes)
        yp = np.empty(n_nodes)
        for n, t in enumerate(th_nodes):
            vals = ref.alm_entries(np.array([t]), np.zeros(1), np.ones(1), ls, ms).real
            yv[n] = vals[0]
            yp[n] = vals[1] if l > m else 0.0
        cl = math.sqrt((2 * l + 1) / (2 * l - 1) * (l - m) * (l + m)) if l > m else 0.0
        dy = (-l * x_nodes * yv + cl * yp) / (1.0 - x_nodes * x_nodes)
        a = (v[:, 0] @ yv[:-1] + (v[:, 1] * dx) @ dy[:-1] + v[:, 2] @ yv[1:] + (v[:, 3] * dx) @ dy[1:])
        if polar.any():
            a += ref.alm_entries(theta[polar], phi[polar], w[polar], np.array([l]), np.array([m]))[0]
        out.append(a)
    return np.array(out)


def ylm_values(l: int, m: int, theta):
    """y_lm and y_{l-1,m} at each theta (one oracle entry sum per point)."""
    ls = np.array([l, max(l - 1, m)])
    ms = np.array([m, m])
    out = np.empty((2, len(theta)))
    for k, t in enumerate(np.asarray(theta, dtype=np.float64)):
        v = ref.alm_entries(np.array([t]), np.zeros(1), np.ones(1), ls, ms).real
        out[0, k] = v[0]
        out[1, k] = v[1] if l > m else 0.0
    return out


def interpolation_error(l: int, m: int, x_nodes, x_eval):
    """Max |S(x) - y_lm(x)| over x_eval for the Hermite spline of App. A.2 on x_nodes
    (ascending), and max |y_lm| there."""
    x_nodes = np.asarray(x_nodes, dtype=np.float64)
    x_eval = np.asarray(x_eval, dtype=np.float64)
    yn = ylm_values(l, m, np.arccos(x_nodes))
    c = math.sqrt((2 * l + 1) / (2 * l - 1) * (l - m) * (l + m)) if l > m else 0.0
    dyn = (-l * x_nodes * yn[0] + c * yn[1]) / (1.0 - x_nodes * x_nodes)
    j = np.clip(np.searchsorted(x_nodes, x_eval, side="right") - 1, 0, len(x_nodes) - 2)
    dx = x_nodes[j + 1] - x_nodes[j]
    b = hermite_basis((x_eval - x_nodes[j]) / dx)
    s = b[0] * yn[0][j] + b[1] * dx * dyn[j] + b[2] * yn[0][j + 1] + b[3] * dx * dyn[j + 1]
    y = ylm_values(l, m, np.arccos(x_eval))[0]
    return float(np.abs(s - y).max()), float(np.abs(y).max())
