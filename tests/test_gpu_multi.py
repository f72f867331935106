"""Multi-weight forms: several weight vectors sharing one position set.

* FP64 multi-weight (one FP64 transform per weight vector) against the oracle
  at the 1e-10 gate.
* Split-bf16 MFMA form (PTALM_BF16X3): three bf16 products with FP32
  accumulation leave ~2^-16 relative error per product; gated at 1e-4 global
  norm-wise per weight vector and stated per l.
"""
import numpy as np
import pytest

from conftest import per_l_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    from paper_2312_12285_amd import ptalm
    return ptalm


def run(lib, th, ph, W, lmax, **opt):
    import torch
    t, p = [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in (th, ph)]
    w = torch.as_tensor(np.ascontiguousarray(W, dtype=np.float64)).cuda()
    out = lib.alm_from_points(t, p, w, lmax, options=lib.opts(**opt))
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.complex128).reshape(W.shape[0], -1).copy()


def catalog(n, nw, seed=41):
    from paper_2312_12285_amd.synth import multi_weight_positions
    return multi_weight_positions(n, nw, seed_pos=seed, seed_w0=4100)


@pytest.mark.parametrize("nw", [16, 32])
def test_bf16x3_small(lib, oracle, nw):
    th, ph, W = catalog(2000 + 37, nw)          # 3 full groups of 512 points and a ragged one
    lmax = 100
    a = run(lib, th, ph, W, lmax, precision=lib.BF16X3)
    worst = 0.0
    for v in range(nw):
        ref = oracle.alm_from_points(th, ph, W[v], lmax)
        g = np.linalg.norm(a[v] - ref) / np.linalg.norm(ref)
        worst = max(worst, g)
    print(f"bf16x3 nw={nw}: worst global rel err over weight vectors {worst:.2e}", flush=True)
    assert worst <= 1e-4


def test_bf16x3_slices_and_determinism(lib, oracle):
    th, ph, W = catalog(3000, 16, seed=43)
    lmax = 64
    a1 = run(lib, th, ph, W, lmax, precision=lib.BF16X3, n_slices=3)
    a2 = run(lib, th, ph, W, lmax, precision=lib.BF16X3, n_slices=3)
    assert np.array_equal(a1.view(np.float64), a2.view(np.float64))
    a3 = run(lib, th, ph, W, lmax, precision=lib.BF16X3, n_slices=1)
    for v in (0, 7, 15):
        ref = oracle.alm_from_points(th, ph, W[v], lmax)
        for a in (a1, a3):
            assert np.linalg.norm(a[v] - ref) / np.linalg.norm(ref) <= 1e-4


def test_bf16x3_poles_and_edges(lib, oracle):
    """Points exactly at the poles and on the equator, lmax 0 and 1."""
    th = np.array([0.0, np.pi, np.pi / 2, 1e-5, np.pi - 1e-5] * 60)
    ph = np.linspace(0.0, 6.0, th.size)
    rng = np.random.default_rng(3)
    W = rng.lognormal(0, 0.2, (16, th.size))
    for lmax in (0, 1, 33):
        a = run(lib, th, ph, W, lmax, precision=lib.BF16X3)
        for v in (0, 15):
            ref = oracle.alm_from_points(th, ph, W[v], lmax)
            assert np.all(np.isfinite(a[v]))
            assert np.linalg.norm(a[v] - ref) / np.linalg.norm(ref) <= 1e-4


def test_fp64_multi_weight_loop(lib, oracle):
    th, ph, W = catalog(1500, 4, seed=44)
    lmax = 80
    a = run(lib, th, ph, W, lmax, precision=lib.FP64)
    for v in range(4):
        ref = oracle.alm_from_points(th, ph, W[v], lmax)
        assert per_l_rel_err(a[v], ref, lmax).max() <= 1e-10


def test_bf16x3_rejects_unsupported_weight_counts(lib):
    import torch
    th, ph, W = catalog(100, 8)
    t, p = [torch.as_tensor(a).cuda() for a in (th, ph)]
    w = torch.as_tensor(W).cuda()
    with pytest.raises(lib.PtalmError):
        lib.alm_from_points(t, p, w, 10, options=lib.opts(precision=lib.BF16X3))


def test_bf16x3_workload_prefix_lmax2048(lib, oracle):
    """First 1000 positions of the multi-weight workload at lmax 2048, 4 of the 32
    weight vectors against the oracle (the oracle costs n*T per vector)."""
    th, ph, W = catalog(1000, 32)
    lmax = 2048
    a = run(lib, th, ph, W, lmax, precision=lib.BF16X3)
    for v in (0, 11, 22, 31):
        ref = oracle.alm_from_points(th, ph, W[v], lmax)
        g = np.linalg.norm(a[v] - ref) / np.linalg.norm(ref)
        pl = per_l_rel_err(a[v], ref, lmax)
        print(f"bf16x3 lmax2048 v={v}: global {g:.2e}, per-l max {pl.max():.2e} at l={pl.argmax()}", flush=True)
        assert g <= 1e-4
