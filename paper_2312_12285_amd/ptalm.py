"""Python binding of the ptalm C ABI (``include/ptalm.h``): argument marshalling only.

Every function takes torch tensors that live on the GPU, passes their device
pointers and the current HIP stream to ``libptalm.so``, and returns the output
tensor.  All arithmetic happens in the library's HIP kernels; there is no CPU
or PyTorch fallback: if the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptalm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                      "(or python paper_2312_12285_amd/build.py) first")

_lib = ctypes.CDLL(LIB_PATH)

PTALM_OK, PTALM_EINVAL, PTALM_ENOMEM, PTALM_EDEVICE, PTALM_EBUSY, PTALM_ENOTSUP = 0, -1, -2, -3, -4, -5
FP64, MIXED, FP32, BF16X3 = 0, 1, 2, 3
LMAX_MAX = 16383

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64


class Opts(ctypes.Structure):
    """Mirror of ``struct ptalm_opts``."""
    _fields_ = [("precision", ctypes.c_int), ("n_weights", ctypes.c_int), ("points_per_lane", ctypes.c_int),
                ("l_block", ctypes.c_int), ("n_slices", ctypes.c_int), ("m_ranges", ctypes.c_int),
                ("reduction", ctypes.c_int), ("timing", ctypes.c_int)]


def _sig(name, restype, argtypes):
    f = getattr(_lib, name)
    f.restype = restype
    f.argtypes = argtypes
    return f


_alm_size = _sig("ptalm_alm_size", _i64, [ctypes.c_int])
_alm_index = _sig("ptalm_alm_index", _i64, [ctypes.c_int, ctypes.c_int, ctypes.c_int])
_alm = _sig("ptalm_alm_from_points", ctypes.c_int, [_vp, _vp, _vp, _i64, ctypes.c_int, _vp, _vp])
_alm_ex = _sig("ptalm_alm_from_points_ex", ctypes.c_int,
               [_vp, _vp, _vp, _i64, ctypes.c_int, _vp, ctypes.POINTER(Opts), _vp, ctypes.c_size_t, _vp])
_alm_noalloc = _sig("ptalm_alm_from_points_noalloc", ctypes.c_int, [_vp, _vp, _vp, _i64, ctypes.c_int, _vp, _vp])
NOALLOC_SCRATCH_BYTES = 128 << 20
NOALLOC_LMAX_MAX = 4094
_ws_bytes = _sig("ptalm_workspace_bytes", ctypes.c_size_t, [_i64, ctypes.c_int, ctypes.POINTER(Opts)])
_cl = _sig("ptalm_cl_from_alm", ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp])
_cross = _sig("ptalm_cross_cl", ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp])
_axpy = _sig("ptalm_alm_axpy", ctypes.c_int, [ctypes.c_double, _vp, _vp, ctypes.c_int, _vp])
_fkp = _sig("ptalm_fkp_fields", ctypes.c_int, [_vp, _vp, ctypes.c_int, _vp, _vp, _vp, _vp])
_last_error = _sig("ptalm_last_error", ctypes.c_char_p, [])
_last_timing = _sig("ptalm_last_timing", ctypes.c_int, [ctypes.POINTER(ctypes.c_double)])
_release = _sig("ptalm_release_cache", ctypes.c_int, [])
_prepare = _sig("ptalm_prepare", ctypes.c_int, [ctypes.c_int])
_plan_ranges = _sig("ptalm_plan_m_ranges", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)])
_shot = _sig("ptalm_window_shot_noise", ctypes.c_int, [_vp, _i64, _vp, _vp, _vp])
_coupling = _sig("ptalm_coupling_matrix", ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp])
_bp_count = _sig("ptalm_bandpower_count", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int])
_bandpowers = _sig("ptalm_bandpowers", ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                     ctypes.c_int, ctypes.c_int, _vp, _vp, _vp])
_alm_spline = _sig("ptalm_alm_from_points_spline", ctypes.c_int,
                   [_vp, _vp, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_double, _vp, ctypes.POINTER(Opts), _vp,
                    ctypes.c_size_t, _vp])
_spline_ws = _sig("ptalm_spline_workspace_bytes", ctypes.c_size_t, [_i64, ctypes.c_int, ctypes.c_int])
_prepare_spline = _sig("ptalm_prepare_spline_call", ctypes.c_int, [_i64, ctypes.c_int, ctypes.c_int])
_shear = _sig("ptalm_shear_alm_from_points", ctypes.c_int,
              [_vp, _vp, _vp, _vp, _vp, _i64, ctypes.c_int, _vp, _vp, ctypes.POINTER(Opts), _vp])
_shear_ws = _sig("ptalm_shear_workspace_bytes", ctypes.c_size_t, [_i64, ctypes.c_int, ctypes.POINTER(Opts)])
_prepare_call = _sig("ptalm_prepare_call", ctypes.c_int, [_i64, ctypes.c_int, ctypes.POINTER(Opts)])
_autotune = _sig("ptalm_autotune", ctypes.c_int,
                 [_vp, _vp, _vp, _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(Opts), _vp])


class Request(ctypes.Structure):
    """Mirror of ``struct ptalm_request``."""
    _fields_ = [("theta", _vp), ("phi", _vp), ("w", _vp), ("n", _i64), ("lmax", ctypes.c_int),
                ("precision", ctypes.c_int), ("alm", _vp), ("cl", _vp)]


class RequestStats(ctypes.Structure):
    """Mirror of ``struct ptalm_request_stats`` (times: steady clock = time.monotonic(), seconds)."""
    _fields_ = [("status", ctypes.c_int), ("slot", ctypes.c_int), ("footprint_bytes", ctypes.c_size_t),
                ("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class ServerState(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_size_t), ("arena_in_use", ctypes.c_size_t), ("slots", ctypes.c_int),
                ("running", ctypes.c_int), ("waiting", ctypes.c_int64)]


_srv_create = _sig("ptalm_server_create", ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.c_int,
                                                          ctypes.POINTER(_vp)])
_srv_submit = _sig("ptalm_server_submit", ctypes.c_int, [_vp, ctypes.POINTER(Request), ctypes.POINTER(_i64)])
_srv_poll = _sig("ptalm_server_poll", ctypes.c_int, [_vp, _i64, ctypes.POINTER(ctypes.c_int),
                                                      ctypes.POINTER(RequestStats)])
_srv_wait = _sig("ptalm_server_wait", ctypes.c_int, [_vp, _i64, ctypes.POINTER(RequestStats)])
_srv_query = _sig("ptalm_server_query", ctypes.c_int, [_vp, ctypes.POINTER(ServerState)])
_srv_destroy = _sig("ptalm_server_destroy", ctypes.c_int, [_vp])
_srv_error = _sig("ptalm_server_last_error", ctypes.c_char_p, [])


class PtalmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ptalm error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != PTALM_OK:
        raise PtalmError(rc, _last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f64(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return t


def _need(t, count: int, name: str):
    """The C ABI takes raw pointers, so buffer sizes are checked here, before any launch."""
    if t.numel() < count:
        raise ValueError(f"{name} holds {t.numel()} elements, the call needs {count}")


def _lmax_ok(lmax: int):
    if not (isinstance(lmax, int) and 0 <= lmax <= LMAX_MAX):
        raise ValueError(f"lmax must be an int in [0, {LMAX_MAX}]")


def alm_size(lmax: int) -> int:
    return int(_alm_size(lmax))


def alm_index(lmax: int, l: int, m: int) -> int:
    return int(_alm_index(lmax, l, m))


def plan_m_ranges(lmax: int, n_ranges: int):
    b = (ctypes.c_int * (n_ranges + 1))()
    _check(_plan_ranges(lmax, n_ranges, b))
    return list(b)


def opts(precision=FP64, n_weights=1, points_per_lane=0, l_block=0, n_slices=0, m_ranges=0, reduction=0,
         timing=0) -> Opts:
    """reduction: 0 = tuned default, else 1 + register-stage (1) + pipelined (2)."""
    return Opts(precision, n_weights, points_per_lane, l_block, n_slices, m_ranges, reduction, timing)


def last_timing_ms() -> float:
    """Device milliseconds of the transform kernel(s) of the last call made with timing=1
    on this thread (HIP events recorded by the library on the call's stream)."""
    v = ctypes.c_double()
    _check(_last_timing(ctypes.byref(v)))
    return v.value


def alm_from_points(theta, phi, w, lmax: int, out=None, options: Opts | None = None, workspace=None, stream=None):
    """a_lm = sum_i w_i Y*_lm(theta_i, phi_i); returns float64 [n_weights, 2T] ((re, im) interleaved,
    healpy order), or [2T] for one weight vector.  w may be [n] or [n_weights, n]."""
    _dev_f64(theta, "theta"); _dev_f64(phi, "phi"); _dev_f64(w, "w")
    n = theta.numel()
    if phi.numel() != n or w.numel() % max(n, 1) != 0:
        raise ValueError("theta, phi and w rows must have the same length")
    nw = w.shape[0] if w.dim() == 2 else 1
    if w.dim() == 2 and w.shape[1] != n:
        raise ValueError("w must be [n] or [n_weights, n]")
    T = alm_size(lmax)
    shape = (nw, 2 * T) if w.dim() == 2 else (2 * T,)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=theta.device)
    else:
        _dev_f64(out, "out")
        if out.numel() != nw * 2 * T:
            raise ValueError("out has the wrong size")
    if options is None and nw == 1 and workspace is None:
        _check(_alm(_ptr(theta), _ptr(phi), _ptr(w), n, lmax, _ptr(out), _stream(stream)))
    else:
        o = options if options is not None else opts()
        o.n_weights = nw
        ws_ptr, ws_len = (None, 0) if workspace is None else (_ptr(workspace), workspace.numel() * workspace.element_size())
        _check(_alm_ex(_ptr(theta), _ptr(phi), _ptr(w), n, lmax, _ptr(out), ctypes.byref(o), ws_ptr, ws_len,
                       _stream(stream)))
    return out


def alm_from_points_noalloc(theta, phi, w, lmax: int, out, stream=None):
    """The no-allocation transform (FP64, one weight vector): the library's static scratch
    holds the partial sums, so the call allocates nothing; `out` (2T doubles) must be given and
    prepare(lmax) must have run on this device.  Calls on one device must not overlap in time."""
    _dev_f64(theta, "theta"); _dev_f64(phi, "phi"); _dev_f64(w, "w"); _dev_f64(out, "out")
    n = theta.numel()
    if phi.numel() != n or w.numel() != n:
        raise ValueError("theta, phi and w must have the same length")
    _lmax_ok(lmax)
    _need(out, 2 * alm_size(lmax), "out")
    _check(_alm_noalloc(_ptr(theta), _ptr(phi), _ptr(w), n, lmax, _ptr(out), _stream(stream)))
    return out


def workspace_bytes(n: int, lmax: int, options: Opts | None = None) -> int:
    o = options if options is not None else opts()
    return int(_ws_bytes(n, lmax, ctypes.byref(o)))


def cl_from_alm(alm, lmax: int, out=None, stream=None):
    """C_l = (2l+1)^-1 sum_{m=-l..l} |a_lm|^2 (float64 [lmax+1])."""
    _dev_f64(alm, "alm")
    _lmax_ok(lmax)
    _need(alm, 2 * alm_size(lmax), "alm")
    if out is None:
        out = torch.empty(lmax + 1, dtype=torch.float64, device=alm.device)
    _dev_f64(out, "out")
    _need(out, lmax + 1, "out")
    _check(_cl(_ptr(alm), lmax, _ptr(out), _stream(stream)))
    return out


def cross_cl(alm1, alm2, lmax: int, out=None, stream=None):
    """C^AB_l = (2l+1)^-1 sum_{m=-l..l} Re(a_lm conj(b_lm)) (float64 [lmax+1])."""
    _dev_f64(alm1, "alm1"); _dev_f64(alm2, "alm2")
    _lmax_ok(lmax)
    _need(alm1, 2 * alm_size(lmax), "alm1"); _need(alm2, 2 * alm_size(lmax), "alm2")
    if out is None:
        out = torch.empty(lmax + 1, dtype=torch.float64, device=alm1.device)
    _dev_f64(out, "out")
    _need(out, lmax + 1, "out")
    _check(_cross(_ptr(alm1), _ptr(alm2), lmax, _ptr(out), _stream(stream)))
    return out


def alm_axpy(alpha: float, x, y, lmax: int, stream=None):
    """y <- y + alpha x (in place); returns y."""
    _dev_f64(x, "x"); _dev_f64(y, "y")
    _lmax_ok(lmax)
    _need(x, 2 * alm_size(lmax), "x"); _need(y, 2 * alm_size(lmax), "y")
    _check(_axpy(float(alpha), _ptr(x), _ptr(y), lmax, _stream(stream)))
    return y


def fkp_fields(alm_data, alm_randoms, lmax: int, stream=None):
    """(delta, window, alpha): alpha = a00(d)/a00(r) on the device, delta = a(d) - alpha a(r),
    window = alpha a(r)."""
    _dev_f64(alm_data, "alm_data"); _dev_f64(alm_randoms, "alm_randoms")
    _lmax_ok(lmax)
    _need(alm_data, 2 * alm_size(lmax), "alm_data"); _need(alm_randoms, 2 * alm_size(lmax), "alm_randoms")
    delta = torch.empty_like(alm_data)
    window = torch.empty_like(alm_data)
    alpha = torch.empty(1, dtype=torch.float64, device=alm_data.device)
    _check(_fkp(_ptr(alm_data), _ptr(alm_randoms), lmax, _ptr(delta), _ptr(window), _ptr(alpha), _stream(stream)))
    return delta, window, alpha


def prepare(lmax: int):
    """Build the per-lmax coefficient tables on the current device ahead of first use."""
    _check(_prepare(lmax))


def window_shot_noise(w, alpha=None, out=None, stream=None):
    """alpha^2 sum_i w_i^2 / (4 pi) (device scalar tensor); alpha a 1-element device tensor or None."""
    _dev_f64(w, "w")
    if alpha is not None:
        _dev_f64(alpha, "alpha")
        _need(alpha, 1, "alpha")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=w.device)
    _dev_f64(out, "out")
    _need(out, 1, "out")
    _check(_shot(_ptr(w), w.numel(), None if alpha is None else _ptr(alpha), _ptr(out), _stream(stream)))
    return out


def coupling_matrix(Wl, lmax: int, shot=None, out=None, stream=None):
    """Mode-coupling matrix M[l, l'] (eq. chat) from the window spectrum Wl[0..lmax_w]; float64
    [(lmax+1), (lmax+1)].  shot: optional 1-element device tensor subtracted from W first."""
    _dev_f64(Wl, "Wl")
    _lmax_ok(lmax)
    if shot is not None:
        _dev_f64(shot, "shot")
        _need(shot, 1, "shot")
    if out is None:
        out = torch.empty((lmax + 1, lmax + 1), dtype=torch.float64, device=Wl.device)
    _dev_f64(out, "out")
    _need(out, (lmax + 1) ** 2, "out")
    _check(_coupling(_ptr(Wl), Wl.numel() - 1, None if shot is None else _ptr(shot), lmax, _ptr(out),
                     _stream(stream)))
    return out


def bandpower_count(lmax: int, lmin: int, delta_l: int) -> int:
    return int(_bp_count(lmax, lmin, delta_l))


def bandpowers(cl_hat, M, lmax: int, delta_l: int, lmin: int = 0, mode: int = 0, Wl=None, stream=None):
    """(cb, window): mode 0 mode-decoupled (eq. mode_coupling), 1 normalised."""
    _dev_f64(cl_hat, "cl_hat"); _dev_f64(M, "M")
    _lmax_ok(lmax)
    _need(cl_hat, lmax + 1, "cl_hat"); _need(M, (lmax + 1) ** 2, "M")
    nb = bandpower_count(lmax, lmin, delta_l)
    cb = torch.empty(max(nb, 1), dtype=torch.float64, device=M.device)
    window = torch.empty((max(nb, 1), lmax + 1), dtype=torch.float64, device=M.device)
    if Wl is not None:
        _dev_f64(Wl, "Wl")
    _check(_bandpowers(_ptr(cl_hat), _ptr(M), None if Wl is None else _ptr(Wl), -1 if Wl is None else Wl.numel() - 1,
                       lmax, lmin, delta_l, mode, _ptr(cb), _ptr(window), _stream(stream)))
    return cb, window


def spline_workspace_bytes(n: int, lmax: int, n_nodes: int) -> int:
    return int(_spline_ws(n, lmax, n_nodes))


def prepare_spline_call(n: int, lmax: int, n_nodes: int):
    """Build the tables a later interpolated transform of these sizes needs (for capture)."""
    _check(_prepare_spline(n, lmax, n_nodes))


def alm_from_points_spline(theta, phi, w, lmax: int, n_nodes: int, theta_cut: float, out=None,
                           options: Opts | None = None, workspace=None, stream=None):
    """a_lm by the interpolated transform of App. A.2 (cubic Hermite splines on n_nodes nodes
    uniform in theta over [theta_cut, pi - theta_cut]; the polar caps by the exact sum).
    Same layout as alm_from_points with one weight vector.  workspace: optional device
    buffer of spline_workspace_bytes(n, lmax, n_nodes) bytes (then nothing is allocated)."""
    _dev_f64(theta, "theta"); _dev_f64(phi, "phi"); _dev_f64(w, "w")
    n = theta.numel()
    if phi.numel() != n or w.numel() != n:
        raise ValueError("theta, phi and w must have the same length")
    T = alm_size(lmax)
    if out is None:
        out = torch.empty(2 * T, dtype=torch.float64, device=theta.device)
    else:
        _dev_f64(out, "out")
        if out.numel() != 2 * T:
            raise ValueError("out has the wrong size")
    ws_ptr, ws_len = (None, 0) if workspace is None else (_ptr(workspace), workspace.numel() * workspace.element_size())
    _check(_alm_spline(_ptr(theta), _ptr(phi), _ptr(w), n, lmax, n_nodes, float(theta_cut), _ptr(out),
                       None if options is None else ctypes.byref(options), ws_ptr, ws_len, _stream(stream)))
    return out


def shear_alm_from_points(theta, phi, w, g1, g2, lmax: int, out_e=None, out_b=None, options: Opts | None = None,
                          stream=None):
    """E and B modes of a weighted shear catalog through the spin +-2 harmonics:
    a^E = -(_2a + _-2a)/2, a^B = i(_2a - _-2a)/2 with _{+-2}a_lm = sum_i w_i (g1 +- i g2)_i _{+-2}Y*_lm.
    Returns (alm_E, alm_B), each float64 [2T] in the layout of alm_from_points."""
    for name, a in (("theta", theta), ("phi", phi), ("w", w), ("g1", g1), ("g2", g2)):
        _dev_f64(a, name)
    n = theta.numel()
    if any(a.numel() != n for a in (phi, w, g1, g2)):
        raise ValueError("theta, phi, w, g1 and g2 must have the same length")
    T = alm_size(lmax)
    outs = []
    for o in (out_e, out_b):
        if o is None:
            o = torch.empty(2 * T, dtype=torch.float64, device=theta.device)
        else:
            _dev_f64(o, "out")
            if o.numel() != 2 * T:
                raise ValueError("out has the wrong size")
        outs.append(o)
    o = options if options is not None else opts()
    _check(_shear(_ptr(theta), _ptr(phi), _ptr(w), _ptr(g1), _ptr(g2), n, lmax, _ptr(outs[0]), _ptr(outs[1]),
                  ctypes.byref(o), _stream(stream)))
    return outs[0], outs[1]


def shear_workspace_bytes(n: int, lmax: int, options: Opts | None = None) -> int:
    o = options if options is not None else opts()
    return int(_shear_ws(n, lmax, ctypes.byref(o)))


def prepare_call(n: int, lmax: int, options: Opts | None = None):
    """Build everything a later call with these arguments needs, so that it can be captured
    into a HIP graph (under capture the library allocates nothing and needs a workspace)."""
    o = options if options is not None else opts()
    _check(_prepare_call(n, lmax, ctypes.byref(o)))


def autotune(theta, phi, w, lmax: int, precision: int = FP64, stream=None) -> Opts:
    """Time every compiled kernel variant of `precision` on these points and return the
    fastest options; the library also keeps them as the defaults for (precision,
    n_weights, lmax) on this device."""
    _dev_f64(theta, "theta"); _dev_f64(phi, "phi"); _dev_f64(w, "w")
    n = theta.numel()
    nw = w.shape[0] if w.dim() == 2 else 1
    if phi.numel() != n or w.numel() != nw * n:
        raise ValueError("theta, phi and w rows must have the same length")
    best = Opts()
    _check(_autotune(_ptr(theta), _ptr(phi), _ptr(w), n, lmax, precision, nw, ctypes.byref(best), _stream(stream)))
    return best


class Server:
    """Continuous-batching request server of the library (ptalm_server_*): requests wait in
    arrival order and are admitted as stream slots and arena memory free up; admitted
    requests run concurrently on the device."""

    def __init__(self, arena_bytes: int, slots: int = 4, device: int | None = None):
        dev = torch.cuda.current_device() if device is None else device
        h = _vp()
        rc = _srv_create(dev, arena_bytes, slots, ctypes.byref(h))
        if rc != PTALM_OK:
            raise PtalmError(rc, _srv_error().decode())
        self._h = h
        self._keep = {}        # ticket -> tensors the request reads or writes

    def submit(self, theta, phi, w, lmax: int, precision: int = FP64, alm=None, cl=None):
        """Queue one catalog (device tensors, complete on the current stream: it is
        synchronized first).  Returns (ticket, alm, cl)."""
        _dev_f64(theta, "theta"); _dev_f64(phi, "phi"); _dev_f64(w, "w")
        n = theta.numel()
        if phi.numel() != n or w.numel() != n:
            raise ValueError("theta, phi and w must have the same length")
        T = alm_size(lmax)
        if alm is None:
            alm = torch.empty(2 * T, dtype=torch.float64, device=theta.device)
        if cl is False:
            cl = None
        elif cl is None:
            cl = torch.empty(lmax + 1, dtype=torch.float64, device=theta.device)
        torch.cuda.current_stream().synchronize()
        req = Request(theta.data_ptr(), phi.data_ptr(), w.data_ptr(), n, lmax, precision, alm.data_ptr(),
                      None if cl is None else cl.data_ptr())
        t = _i64()
        rc = _srv_submit(self._h, ctypes.byref(req), ctypes.byref(t))
        if rc != PTALM_OK:
            raise PtalmError(rc, _srv_error().decode())
        self._keep[t.value] = (theta, phi, w, alm, cl)
        return t.value, alm, cl

    def poll(self, ticket: int):
        """None while running; the stats (RequestStats) once done."""
        done = ctypes.c_int()
        st = RequestStats()
        rc = _srv_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(st))
        if not done.value and rc == PTALM_OK:
            return None
        self._keep.pop(ticket, None)
        if rc != PTALM_OK:
            raise PtalmError(rc, _srv_error().decode())
        return st

    def wait(self, ticket: int):
        st = RequestStats()
        rc = _srv_wait(self._h, ticket, ctypes.byref(st))
        self._keep.pop(ticket, None)
        if rc != PTALM_OK:
            raise PtalmError(rc, _srv_error().decode())
        return st

    def state(self) -> ServerState:
        st = ServerState()
        _check_srv(_srv_query(self._h, ctypes.byref(st)))
        return st

    def close(self):
        if getattr(self, "_h", None):
            _srv_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_srv(rc):
    if rc != PTALM_OK:
        raise PtalmError(rc, _srv_error().decode())


def release_cache():
    _check(_release())


def last_error() -> str:
    return _last_error().decode()


def as_complex(alm):
    """View a float64 (re, im)-interleaved a_lm tensor as complex128."""
    return torch.view_as_complex(alm.view(*alm.shape[:-1], -1, 2))
