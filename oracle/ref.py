"""ctypes wrapper of the CPU oracle ``libptalm_ref.so`` (test infrastructure only).

Arrays are numpy float64; a_lm come back as complex128 in healpy order
(index(l, m) = m*(2*lmax+1-m)//2 + l).  See ``ptalm_ref.h`` for the contract.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libptalm_ref.so")
_lib = None
_override = None   # set by use_library(); lets a test run the same calls on another build

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def _bind(path):
    lib = ctypes.CDLL(path)
    lib.ptalm_ref_alm_from_points.argtypes = [_dp, _dp, _dp, ctypes.c_int64, ctypes.c_int, _dp, ctypes.c_int]
    lib.ptalm_ref_alm_from_points_ld.argtypes = lib.ptalm_ref_alm_from_points.argtypes + [ctypes.c_int]
    lib.ptalm_ref_alm_entries.argtypes = [_dp, _dp, _dp, ctypes.c_int64, ctypes.c_int, _ip, _ip, _dp, ctypes.c_int]
    lib.ptalm_ref_cl_from_alm.argtypes = [_dp, ctypes.c_int, _dp]
    lib.ptalm_ref_cross_cl.argtypes = [_dp, _dp, ctypes.c_int, _dp]
    lib.ptalm_ref_alm_size.argtypes = [ctypes.c_int]
    lib.ptalm_ref_alm_size.restype = ctypes.c_int64
    lib.ptalm_ref_threej000.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.ptalm_ref_threej000.restype = ctypes.c_double
    lib.ptalm_ref_coupling_matrix.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int]
    lib.ptalm_ref_coupling_rows.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _ip, ctypes.c_int, _dp, ctypes.c_int]
    lib.ptalm_ref_spin_entries.argtypes = [_dp, _dp, _dp, _dp, _dp, ctypes.c_int64, ctypes.c_int, _ip, _ip, _dp,
                                           ctypes.c_int]
    lib.ptalm_ref_spin_alm.argtypes = [_dp, _dp, _dp, _dp, _dp, ctypes.c_int64, ctypes.c_int, _dp, _dp, ctypes.c_int]
    for f in ("ptalm_ref_alm_from_points", "ptalm_ref_alm_from_points_ld", "ptalm_ref_alm_entries", "ptalm_ref_spin_alm",
              "ptalm_ref_cl_from_alm", "ptalm_ref_cross_cl", "ptalm_ref_coupling_matrix", "ptalm_ref_coupling_rows",
              "ptalm_ref_spin_entries"):
        getattr(lib, f).restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _override is not None:
        return _override
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build_ref
        build_ref.build()
    _lib = _bind(_LIB_PATH)
    return _lib


class use_library:
    """Context manager: route this module's calls to another build of the oracle
    (used by the test that plants mistakes in a copy of the source)."""

    def __init__(self, path):
        self.lib = _bind(path)

    def __enter__(self):
        global _override
        self._prev = _override
        _override = self.lib
        return self

    def __exit__(self, *exc):
        global _override
        _override = self._prev
        return False


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(_dp)


def alm_size(lmax: int) -> int:
    return (lmax + 1) * (lmax + 2) // 2


def alm_from_points(theta, phi, w, lmax: int, nthreads: int = 0, long_double: bool = False,
                    fp64_trig: bool = False) -> np.ndarray:
    """a_lm = sum_i w_i conj(Y_lm(theta_i, phi_i)) (eq. alm_def), healpy order, complex128.

    long_double selects the long-double variant; fp64_trig (long-double variant
    only) rounds cos(theta), sin(theta) to double first, as the FP64 variant does.
    """
    lib = _load()
    theta, phi, w = _f64(theta), _f64(phi), _f64(w)
    n = theta.size
    if phi.size != n or w.size != n:
        raise ValueError("theta, phi, w must have the same length")
    out = np.zeros(2 * alm_size(lmax), dtype=np.float64)
    if long_double:
        rc = lib.ptalm_ref_alm_from_points_ld(_ptr(theta), _ptr(phi), _ptr(w), n, lmax, _ptr(out), nthreads,
                                              1 if fp64_trig else 0)
    else:
        rc = lib.ptalm_ref_alm_from_points(_ptr(theta), _ptr(phi), _ptr(w), n, lmax, _ptr(out), nthreads)
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")
    return out.view(np.complex128)


def alm_entries(theta, phi, w, ls, ms, nthreads: int = 0) -> np.ndarray:
    """Selected a_{l,m} over all points (complex128, one per (ls[k], ms[k]))."""
    lib = _load()
    theta, phi, w = _f64(theta), _f64(phi), _f64(w)
    ls = np.ascontiguousarray(ls, dtype=np.int32)
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    out = np.zeros(2 * ls.size, dtype=np.float64)
    rc = lib.ptalm_ref_alm_entries(_ptr(theta), _ptr(phi), _ptr(w), theta.size, ls.size,
                                   ls.ctypes.data_as(_ip), ms.ctypes.data_as(_ip), _ptr(out), nthreads)
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")
    return out.view(np.complex128)


def spin_entries(theta, phi, w, g1, g2, ls, ms, nthreads: int = 0):
    """Selected spin +-2 coefficients over all points: (_{+2}a, _{-2}a), each complex128,
    one per (ls[k], ms[k]), for the field g1 + i g2 (spin +2) and its conjugate (spin -2)."""
    lib = _load()
    theta, phi, w, g1, g2 = (_f64(a) for a in (theta, phi, w, g1, g2))
    ls = np.ascontiguousarray(ls, dtype=np.int32)
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    out = np.zeros(4 * ls.size, dtype=np.float64)
    rc = lib.ptalm_ref_spin_entries(_ptr(theta), _ptr(phi), _ptr(w), _ptr(g1), _ptr(g2), theta.size, ls.size,
                                    ls.ctypes.data_as(_ip), ms.ctypes.data_as(_ip), _ptr(out), nthreads)
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")
    o = out.reshape(-1, 4)
    return o[:, 0] + 1j * o[:, 1], o[:, 2] + 1j * o[:, 3]


def spin_alm(theta, phi, w, g1, g2, lmax: int, nthreads: int = 0):
    """(_{+2}a_lm, _{-2}a_lm) for every coefficient, healpy order, complex128 (0 for l < 2)."""
    lib = _load()
    theta, phi, w, g1, g2 = (_f64(a) for a in (theta, phi, w, g1, g2))
    T = alm_size(lmax)
    p2 = np.zeros(2 * T)
    m2 = np.zeros(2 * T)
    rc = lib.ptalm_ref_spin_alm(_ptr(theta), _ptr(phi), _ptr(w), _ptr(g1), _ptr(g2), theta.size, lmax, _ptr(p2),
                                _ptr(m2), nthreads)
    if rc != 0:
        raise ValueError(f"oracle rejected the arguments (rc={rc})")
    return p2.view(np.complex128), m2.view(np.complex128)


def shear_eb(theta, phi, w, g1, g2, lmax: int, nthreads: int = 0):
    """E and B coefficients of the whole transform: a^E = -(_2a + _-2a)/2, a^B = i (_2a - _-2a)/2."""
    a2, am2 = spin_alm(theta, phi, w, g1, g2, lmax, nthreads)
    return -(a2 + am2) / 2, 1j * (a2 - am2) / 2


def shear_eb_entries(theta, phi, w, g1, g2, ls, ms, nthreads: int = 0):
    """Selected E and B coefficients: a^E = -(_2a + _-2a)/2, a^B = i (_2a - _-2a)/2."""
    a2, am2 = spin_entries(theta, phi, w, g1, g2, ls, ms, nthreads)
    return -(a2 + am2) / 2, 1j * (a2 - am2) / 2


def cl_from_alm(alm, lmax: int) -> np.ndarray:
    """C_l = (2l+1)^-1 sum_{m=-l..l} |a_lm|^2 (eq. pseudoCl)."""
    lib = _load()
    a = np.ascontiguousarray(alm, dtype=np.complex128).view(np.float64)
    if a.size != 2 * alm_size(lmax):
        raise ValueError("alm has the wrong length for lmax")
    out = np.zeros(lmax + 1)
    if lib.ptalm_ref_cl_from_alm(_ptr(a), lmax, _ptr(out)) != 0:
        raise ValueError("bad arguments")
    return out


def cross_cl(alm1, alm2, lmax: int) -> np.ndarray:
    """C^AB_l = (2l+1)^-1 sum_{m=-l..l} Re(a_lm conj(b_lm))."""
    lib = _load()
    a = np.ascontiguousarray(alm1, dtype=np.complex128).view(np.float64)
    b = np.ascontiguousarray(alm2, dtype=np.complex128).view(np.float64)
    if a.size != 2 * alm_size(lmax) or b.size != a.size:
        raise ValueError("alm has the wrong length for lmax")
    out = np.zeros(lmax + 1)
    if lib.ptalm_ref_cross_cl(_ptr(a), _ptr(b), lmax, _ptr(out)) != 0:
        raise ValueError("bad arguments")
    return out


# ---------------------------------------------------------------------------
# Mode coupling and bandpowers (Sec. 2.1 eq. chat, eq. mode_coupling; App. B)
# ---------------------------------------------------------------------------

def threej000(l1: int, l2: int, l3: int) -> float:
    """(l1 l2 l3; 0 0 0), closed form (App. B)."""
    return float(_load().ptalm_ref_threej000(int(l1), int(l2), int(l3)))


def coupling_matrix(Wl, lmax: int, nthreads: int = 0) -> np.ndarray:
    """M[l, l'] = (2l'+1)/(4pi) sum_lambda (2 lambda+1) (l l' lambda; 000)^2 W_lambda (eq. chat),
    0 <= l, l' <= lmax; W given for lambda = 0..len(Wl)-1."""
    Wl = _f64(Wl)
    M = np.zeros((lmax + 1, lmax + 1))
    rc = _load().ptalm_ref_coupling_matrix(_ptr(Wl), Wl.size - 1, lmax, _ptr(M), nthreads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return M


def coupling_rows(Wl, lmax: int, rows, nthreads: int = 0) -> np.ndarray:
    """Rows M[rows[k], 0..lmax] of the coupling matrix."""
    Wl = _f64(Wl)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros((rows.size, lmax + 1))
    rc = _load().ptalm_ref_coupling_rows(_ptr(Wl), Wl.size - 1, lmax, rows.ctypes.data_as(_ip), rows.size,
                                         _ptr(out), nthreads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def bin_matrix(lmax: int, delta_l: int, lmin: int = 0):
    """theta[b, l] = 1/delta_l for l in bin b = [lmin + b delta_l, lmin + (b+1) delta_l) (complete
    bins within lmax only), else 0 (Sec. 2.1: averaging C_l within each bin); and the bin
    indicator chi[l, b]."""
    nb = (lmax + 1 - lmin) // delta_l
    theta = np.zeros((nb, lmax + 1))
    chi = np.zeros((lmax + 1, nb))
    for b in range(nb):
        lo = lmin + b * delta_l
        theta[b, lo:lo + delta_l] = 1.0 / delta_l
        chi[lo:lo + delta_l, b] = 1.0
    return theta, chi


def decoupled_bandpowers(cl_hat, M, theta, chi):
    """Mode-decoupled bandpowers (eq. mode_coupling): M_bb' = sum_{l in b} sum_{l' in b'}
    theta_b^l M_ll', C~_b = sum_b' (M^-1)_bb' C^_b' with C^_b = sum_l theta_b^l C^_l, and the
    window of eq. expectation_value, cal M_bl' = sum_b' (M^-1)_bb' sum_l theta_b'^l M_ll'."""
    Mbb = theta @ M @ chi
    cb = np.linalg.solve(Mbb, theta @ np.asarray(cl_hat))
    window = np.linalg.solve(Mbb, theta @ M)
    return cb, window, Mbb


def normalized_bandpowers(cl_hat, M, theta, Wl):
    """Normalised convention: C~'_b = N sum_l theta_b^l C^_l, cal M'_bl' = N sum_l theta_b^l M_ll',
    with 1/N = sum_l' (2l'+1)/(4pi) W_l' (the shot-noise amplitude factor)."""
    Wl = np.asarray(Wl, dtype=np.float64)
    lam = np.arange(Wl.size)
    N = 1.0 / np.sum((2 * lam + 1) / (4 * np.pi) * Wl)
    return N * (theta @ np.asarray(cl_hat)), N * (theta @ M), N
