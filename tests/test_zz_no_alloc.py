"""The no-allocation transform (ptalm_alm_from_points_noalloc) against the allocating one,
through the C ABI: two calls in a row on one device, the second with a smaller input, each
within the FP64 parity gate of the allocating call (per-l norm-wise 1e-10 and element-wise);
the limits it refuses; and the set-up it needs."""
import sys

import numpy as np
import pytest

from conftest import ell_of_index, per_l_rel_err

pytestmark = pytest.mark.gpu

GATE = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2312_12285_amd import ptalm
    return ptalm


def check(a, ref, lmax, what):
    err = per_l_rel_err(a, ref, lmax)
    L = ell_of_index(lmax)
    nrm = np.sqrt(np.bincount(L, weights=np.abs(ref) ** 2, minlength=lmax + 1))
    elem = np.abs(a - ref) / np.maximum(nrm[L] / np.sqrt(L + 1.0), 1e-300)
    say(f"{what}: max per-l err {err.max():.3e}, max element err {elem.max():.3e}")
    assert err.max() <= GATE and elem.max() <= GATE


def test_noalloc_matches_the_allocating_transform_twice(lib):
    import torch
    from paper_2312_12285_amd import synth
    cases = [(300_000, 1024, 71), (5_000, 96, 72)]     # the second call is smaller in n and lmax
    outs = []
    for n, lmax, seed in cases:
        say(f"case: no-alloc n={n} lmax={lmax} seed={seed}")
        cat = synth.masked_galaxies(n, seed_pos=seed, seed_w=seed + 100)
        t, p, w = (torch.as_tensor(a).cuda() for a in (cat.theta, cat.phi, cat.w))
        lib.prepare(lmax)
        out = torch.full((2 * lib.alm_size(lmax),), float("nan"), dtype=torch.float64, device="cuda")
        lib.alm_from_points_noalloc(t, p, w, lmax, out)
        ref = lib.alm_from_points(t, p, w, lmax)
        torch.cuda.synchronize()
        outs.append((out.cpu().numpy().view(np.complex128).copy(), ref.cpu().numpy().view(np.complex128).copy(),
                     lmax))
    for k, (a, ref, lmax) in enumerate(outs):
        assert np.isfinite(a).all()
        check(a, ref, lmax, f"call {k}")


def test_noalloc_edge_cases(lib):
    import torch
    lmax = 64
    lib.prepare(lmax)
    out = torch.full((2 * lib.alm_size(lmax),), 7.0, dtype=torch.float64, device="cuda")
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    lib.alm_from_points_noalloc(e, e, e, lmax, out)             # n = 0: all zero
    torch.cuda.synchronize()
    assert not out.cpu().numpy().any()
    # one point at the north pole: a_lm = w sqrt((2l+1)/4pi) delta_m0
    one = torch.tensor([0.0], dtype=torch.float64, device="cuda")
    wt = torch.tensor([2.5], dtype=torch.float64, device="cuda")
    lib.alm_from_points_noalloc(one, one, wt, lmax, out)
    torch.cuda.synchronize()
    a = out.cpu().numpy().view(np.complex128)
    l = np.arange(lmax + 1)
    np.testing.assert_allclose(a[:lmax + 1].real, 2.5 * np.sqrt((2 * l + 1) / (4 * np.pi)), rtol=1e-13)
    assert np.abs(a[lmax + 1:]).max() <= 1e-13 and not a[:lmax + 1].imag.any()


def test_noalloc_refusals(lib):
    import torch
    t = torch.zeros(10, dtype=torch.float64, device="cuda")
    big = lib.NOALLOC_LMAX_MAX + 1
    out = torch.empty(2 * lib.alm_size(big), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.PtalmError) as ei:
        lib.alm_from_points_noalloc(t, t, t, big, out)
    assert ei.value.code == lib.PTALM_EINVAL and "NOALLOC" in str(ei.value)
    lmax = 1237                                                # not prepared on this device
    out = torch.empty(2 * lib.alm_size(lmax), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.PtalmError) as ei:
        lib.alm_from_points_noalloc(t, t, t, lmax, out)
    assert ei.value.code == lib.PTALM_EBUSY and "ptalm_prepare" in str(ei.value)
