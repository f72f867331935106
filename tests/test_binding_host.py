"""Host checks of the Python binding's argument checks (no GPU): the C ABI takes raw
pointers, so the binding must refuse buffers too small for lmax before any call into the
library.  The device-tensor check is bypassed so CPU tensors stand in for device ones, and
every library entry point is replaced by a sentinel that fails the test if reached."""
import os
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.fixture()
def ptalm(monkeypatch):
    from paper_2312_12285_amd import ptalm as mod

    def must_not_call(*a, **k):
        raise AssertionError("the library was called with an undersized buffer")

    monkeypatch.setattr(mod, "_dev_f64", lambda t, name: t)
    monkeypatch.setattr(mod, "_stream", lambda s: None)
    for name in ("_cl", "_cross", "_axpy", "_fkp", "_shot", "_coupling", "_bandpowers"):
        monkeypatch.setattr(mod, name, must_not_call)
    return mod


def f64(n):
    return torch.zeros(n, dtype=torch.float64)


LMAX = 64
T = (LMAX + 1) * (LMAX + 2) // 2


def test_spectra_refuse_short_alm(ptalm):
    short = f64(2 * T - 1)
    with pytest.raises(ValueError, match="alm"):
        ptalm.cl_from_alm(short, LMAX, out=f64(LMAX + 1))
    with pytest.raises(ValueError, match="alm2"):
        ptalm.cross_cl(f64(2 * T), short, LMAX, out=f64(LMAX + 1))
    with pytest.raises(ValueError, match="out"):
        ptalm.cl_from_alm(f64(2 * T), LMAX, out=f64(LMAX))
    # an lmax-8 array passed with lmax 64 (the mismatch that would read past the buffer)
    with pytest.raises(ValueError):
        ptalm.cl_from_alm(f64(2 * 45), LMAX, out=f64(LMAX + 1))


def test_axpy_and_fkp_refuse_short_operands(ptalm):
    with pytest.raises(ValueError, match="y"):
        ptalm.alm_axpy(2.0, f64(2 * T), f64(2 * T - 2), LMAX)
    with pytest.raises(ValueError, match="x"):
        ptalm.alm_axpy(2.0, f64(10), f64(2 * T), LMAX)
    with pytest.raises(ValueError, match="alm_randoms"):
        ptalm.fkp_fields(f64(2 * T), f64(2 * T - 1), LMAX)


def test_bad_lmax_is_refused(ptalm):
    for bad in (-1, 16384):
        with pytest.raises(ValueError, match="lmax"):
            ptalm.cl_from_alm(f64(8), bad, out=f64(8))


def test_coupling_and_bandpowers_refuse_short_buffers(ptalm):
    with pytest.raises(ValueError, match="out"):
        ptalm.coupling_matrix(f64(200), LMAX, out=f64((LMAX + 1) ** 2 - 1))
    with pytest.raises(ValueError, match="shot"):
        ptalm.coupling_matrix(f64(200), LMAX, shot=f64(0))
    with pytest.raises(ValueError, match="M"):
        ptalm.bandpowers(f64(LMAX + 1), f64(LMAX * LMAX), LMAX, 8)
    with pytest.raises(ValueError, match="cl_hat"):
        ptalm.bandpowers(f64(LMAX), f64((LMAX + 1) ** 2), LMAX, 8)
    with pytest.raises(ValueError, match="alpha"):
        ptalm.window_shot_noise(f64(100), alpha=f64(0))
