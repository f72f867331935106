"""Autotuner and HIP-graph capture of the transform.

* ptalm_autotune times every compiled variant of a form on a sample and keeps
  the fastest as the default; a later call with default options must then give
  bitwise the result of the explicit tuned options, and that result must pass
  the form's gate against the oracle.
* A transform captured into a HIP graph (caller workspace, tables prepared) is
  replayed several times with eager work between replays (the weights change
  in place); every replay must equal, bitwise, an eager call on the same inputs
  (the kernels are deterministic for a fixed decomposition).
* Capture without a workspace, or of an lmax whose tables were not prepared,
  is refused before anything is enqueued.
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
    yield ptalm
    ptalm.release_cache()      # forget tuned defaults for the tests that follow


def dev(*arrays):
    import torch
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrays]


def as_np(t):
    return t.cpu().numpy().view(np.complex128).copy()


def test_autotune_fp64_then_defaults_follow(lib, oracle):
    import torch
    from paper_2312_12285_amd.synth import masked_randoms
    cat = masked_randoms(30_000, seed=31)
    th, ph, w = cat.theta, cat.phi, cat.w
    lmax = 256
    t, p, wd = dev(th, ph, w)
    best = lib.autotune(t, p, wd, lmax, precision=lib.FP64)
    print(f"autotune fp64 lmax {lmax}: points_per_lane {best.points_per_lane}, l_block {best.l_block}, "
          f"reduction {best.reduction}", flush=True)
    assert best.precision == lib.FP64 and best.points_per_lane > 0 and best.l_block > 0 and best.reduction > 0
    explicit = lib.alm_from_points(t, p, wd, lmax, options=lib.opts(points_per_lane=best.points_per_lane,
                                                                     l_block=best.l_block, reduction=best.reduction))
    default = lib.alm_from_points(t, p, wd, lmax)
    torch.cuda.synchronize()
    assert torch.equal(explicit, default)
    ref = oracle.alm_from_points(th, ph, w, lmax)
    assert per_l_rel_err(as_np(default), ref, lmax).max() <= 1e-10


def test_autotune_bf16x3(lib, oracle):
    import torch
    from paper_2312_12285_amd.synth import multi_weight_positions
    th, ph, W = multi_weight_positions(20_000, 16, seed_pos=45, seed_w0=4500)
    lmax = 128
    t, p, wd = dev(th, ph, W)
    best = lib.autotune(t, p, wd, lmax, precision=lib.BF16X3)
    print(f"autotune bf16x3 lmax {lmax}: n_slices {best.n_slices}", flush=True)
    assert best.n_slices in (1, 2, 4, 8)
    out = lib.alm_from_points(t, p, wd, lmax, options=lib.opts(precision=lib.BF16X3))
    torch.cuda.synchronize()
    a = as_np(out).reshape(16, -1)
    for v in (0, 15):
        ref = oracle.alm_from_points(th, ph, W[v], lmax)
        assert np.linalg.norm(a[v] - ref) / np.linalg.norm(ref) <= 1e-4


@pytest.mark.parametrize("form", ["fp64", "bf16x3"])
def test_graph_replays_equal_eager_calls(lib, form):
    import torch
    from paper_2312_12285_amd.synth import multi_weight_positions
    nw = 1 if form == "fp64" else 16
    n, lmax = 5_000 + 123, 96
    th, ph, W = multi_weight_positions(n, max(nw, 1), seed_pos=47, seed_w0=4700)
    t, p = dev(th, ph)
    w = dev(W[0] if nw == 1 else W)[0]
    o = lib.opts(precision=lib.FP64 if form == "fp64" else lib.BF16X3, n_weights=nw)
    lib.prepare_call(n, lmax, o)
    ws = torch.empty(lib.workspace_bytes(n, lmax, o), dtype=torch.uint8, device="cuda")
    out = torch.empty((nw, 2 * lib.alm_size(lmax)) if nw > 1 else (2 * lib.alm_size(lmax),),
                      dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):        # one eager call on the capture stream first
        lib.alm_from_points(t, p, w, lmax, out=out, options=o, workspace=ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        lib.alm_from_points(t, p, w, lmax, out=out, options=o, workspace=ws)
    for rep in range(3):
        w.mul_(1.0 + 0.25 * rep)         # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        eager = lib.alm_from_points(t, p, w, lmax, options=lib.opts(precision=o.precision, n_weights=nw))
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {rep} differs from the eager call"


def test_capture_refusals(lib):
    import torch
    n, lmax = 1000, 77
    t, p, w = dev(np.full(n, 1.0), np.zeros(n), np.ones(n))
    o = lib.opts()
    ws = torch.empty(lib.workspace_bytes(n, lmax, o), dtype=torch.uint8, device="cuda")
    out = torch.empty(2 * lib.alm_size(lmax), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(lib.PtalmError) as ei:
        with torch.cuda.graph(g):
            lib.alm_from_points(t, p, w, lmax, out=out, options=o)            # no workspace
    assert ei.value.code == lib.PTALM_EINVAL
    g2 = torch.cuda.CUDAGraph()
    with pytest.raises(lib.PtalmError) as ei:
        with torch.cuda.graph(g2):
            lib.alm_from_points(t, p, w, lmax, out=out, options=o, workspace=ws)   # lmax 77 never prepared
    assert ei.value.code == lib.PTALM_EBUSY
    torch.cuda.synchronize()
