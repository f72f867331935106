"""The reduced-precision workload's own oracle check: the first 1e5 points of the 1e8-point
masked random catalog (seed 31, unit weights; the bench catalog's prefix) at lmax 3072,
against the CPU oracle summed over all 1e5 points.

The oracle runs on four 25,000-point chunks (one test each, so no single test is long) and
the reference is their sum (linearity of eq. alm_def; chunking moves the oracle by rounding
only, ~1e-16).  Gates: FP64 per-l norm-wise <= 1e-10 for every l plus the element-wise gate;
MIXED (FP64 recurrence, FP32 products, compensated FP64 final reduction) global norm-wise
<= 1e-6 with its per-l curve stated; the FP32-recurrence form's curve is stated against its
bound of max(1e-6, 8 (l+1) 2^-24) per l."""
import sys

import numpy as np
import pytest

from conftest import ell_of_index, per_l_rel_err

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N, LMAX, CHUNK = 100_000, 3072, 25_000
_ref = {}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cat():
    from paper_2312_12285_amd import synth
    return synth.masked_randoms(N, seed=31)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2312_12285_amd import ptalm
    return ptalm


def gpu(lib, cat, lo, hi, precision):
    import torch
    t, p, w = (torch.as_tensor(np.ascontiguousarray(a[lo:hi])).cuda() for a in (cat.theta, cat.phi, cat.w))
    out = lib.alm_from_points(t, p, w, LMAX, options=lib.opts(precision=precision))
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.complex128).copy()


def curve(err):
    pick = [0, 1, 2, 10, 100, 500, 1000, 1500, 2000, 2500, 3000, LMAX]
    return ", ".join(f"l={l}: {err[l]:.2e}" for l in pick)


def element_err(a, ref):
    L = ell_of_index(LMAX)
    nrm = np.sqrt(np.bincount(L, weights=np.abs(ref) ** 2, minlength=LMAX + 1))
    return float((np.abs(a - ref) / np.maximum(nrm[L] / np.sqrt(L + 1.0), 1e-300)).max())


@pytest.mark.parametrize("k", range(N // CHUNK))
def test_fp64_chunk_against_oracle(lib, oracle, cat, k):
    """FP64 GPU result of chunk k against the oracle on the same chunk (the reference of the
    tests below is the sum of these oracle chunks)."""
    lo, hi = k * CHUNK, (k + 1) * CHUNK
    say(f"case: C3 prefix chunk {k} points [{lo}, {hi}) lmax {LMAX}")
    ref = oracle.alm_from_points(cat.theta[lo:hi], cat.phi[lo:hi], cat.w[lo:hi], LMAX)
    _ref[k] = ref
    a = gpu(lib, cat, lo, hi, lib.FP64)
    err = per_l_rel_err(a, ref, LMAX)
    assert err.max() <= 1e-10 and element_err(a, ref) <= 1e-10


def reference():
    if len(_ref) != N // CHUNK:
        pytest.fail("the oracle chunks did not all run (run this module whole)")
    return sum(_ref[k] for k in range(N // CHUNK))


def test_fp64_1e5_points(lib, cat, measured):
    ref = reference()
    a = gpu(lib, cat, 0, N, lib.FP64)
    err = per_l_rel_err(a, ref, LMAX)
    el = element_err(a, ref)
    measured.append(f"C3 1e5-point prefix, lmax {LMAX}, FP64 vs oracle: max per-l {err.max():.2e} "
                    f"(l={err.argmax()}), element {el:.2e}; {curve(err)}")
    assert err.max() <= 1e-10 and el <= 1e-10


def test_mixed_1e5_points(lib, cat, measured):
    ref = reference()
    a = gpu(lib, cat, 0, N, lib.MIXED)
    err = per_l_rel_err(a, ref, LMAX)
    glob = float(np.sqrt(np.sum(np.abs(a - ref) ** 2) / np.sum(np.abs(ref) ** 2)))
    measured.append(f"C3 1e5-point prefix, lmax {LMAX}, MIXED vs oracle: global {glob:.2e}, max per-l "
                    f"{err.max():.2e} (l={err.argmax()}); {curve(err)}")
    assert glob <= 1e-6


def test_fp32_1e5_points(lib, cat, measured):
    ref = reference()
    a = gpu(lib, cat, 0, N, lib.FP32)
    err = per_l_rel_err(a, ref, LMAX)
    glob = float(np.sqrt(np.sum(np.abs(a - ref) ** 2) / np.sum(np.abs(ref) ** 2)))
    measured.append(f"C3 1e5-point prefix, lmax {LMAX}, FP32 recurrence vs oracle: global {glob:.2e}, max per-l "
                    f"{err.max():.2e} (l={err.argmax()}); {curve(err)}")
    l = np.arange(LMAX + 1)
    assert np.all(err <= np.maximum(1e-6, 8.0 * (l + 1) * 2.0 ** -24))
