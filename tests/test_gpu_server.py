"""Served form: continuous batching in the library's request server.

* A mix of catalogs of uneven size, lmax and precision, submitted together to
  a server with several slots, runs concurrently on the device, and every
  request's a_lm and C_l are bitwise those of the same call made alone (each
  request keeps its solo work plan); two of them also pass the oracle gate.
* With an arena smaller than the mix, admission never holds more scratch than
  the arena, admits in arrival order, and still completes everything.
* Requests run as work items (chunks of point slices): a small request
  submitted behind two large ones completes first, and all three are bitwise
  their solo results.
* Requests that can never fit, or that ask for a form the server does not
  run, are refused at submission; destroying a server completes pending work.
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


MIX = [  # (n, lmax, precision name, seed)
    (400_000, 512, "FP64", 61), (0, 64, "FP64", 62), (1, 8, "FP64", 63), (20_000, 256, "FP64", 64),
    (150_000, 128, "MIXED", 65), (513, 0, "FP64", 66), (300_000, 256, "FP32", 67), (64_000, 512, "FP64", 68),
    (250_000, 384, "FP64", 69), (5_000, 64, "FP64", 70), (120_000, 512, "MIXED", 71), (90_000, 200, "FP64", 72),
]


def catalog(n, seed):
    from paper_2312_12285_amd.synth import uniform_in_mask, lognormal_weights
    if n == 0:
        return np.zeros(0), np.zeros(0), np.zeros(0)
    t, p = uniform_in_mask(n, seed)
    return t, p, lognormal_weights(n, 0.3, seed + 1000)


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def overlapped(stats):
    for i, a in enumerate(stats):
        for b in stats[i + 1:]:
            if a.admit_s < b.done_s and b.admit_s < a.done_s:
                return True
    return False


def test_mix_runs_concurrently_and_equals_solo(lib, oracle):
    import torch
    cats = [catalog(n, seed) for n, _, _, seed in MIX]
    inputs = [(dev(t), dev(p), dev(w)) for t, p, w in cats]
    torch.cuda.synchronize()
    with lib.Server(arena_bytes=4 << 30, slots=4) as srv:
        subs = []
        for (n, lmax, prec, _), (t, p, w) in zip(MIX, inputs):
            subs.append(srv.submit(t, p, w, lmax, precision=getattr(lib, prec)))
        stats = [srv.wait(tk) for tk, _, _ in subs]
    assert all(s.status == 0 for s in stats)
    assert overlapped(stats), "no two requests were on the device at the same time"
    for (n, lmax, prec, _), (t, p, w), (tk, alm, cl), st in zip(MIX, inputs, subs, stats):
        solo = lib.alm_from_points(t, p, w, lmax, options=lib.opts(precision=getattr(lib, prec)))
        solo_cl = lib.cl_from_alm(solo, lmax)
        torch.cuda.synchronize()
        assert torch.equal(alm, solo), f"request n={n} lmax={lmax} {prec}: served result differs from solo"
        assert torch.equal(cl, solo_cl)
        assert st.admit_s >= st.submit_s and st.done_s >= st.admit_s
    for k in (3, 9):                      # two FP64 requests against the oracle
        n, lmax, _, _ = MIX[k]
        t, p, w = cats[k]
        ref = oracle.alm_from_points(t, p, w, lmax)
        got = subs[k][1].cpu().numpy().view(np.complex128)
        assert per_l_rel_err(got, ref, lmax).max() <= 1e-10


def test_admission_budget_and_order(lib):
    import torch
    reqs = [(200_000, 256, 81 + k) for k in range(10)]
    cats = [catalog(n, seed) for n, _, seed in reqs]
    inputs = [(dev(t), dev(p), dev(w)) for t, p, w in cats]
    foot = lib.workspace_bytes(200_000, 256, lib.opts())
    arena = 3 * ((foot + 255) // 256 * 256)       # room for three at a time
    torch.cuda.synchronize()
    with lib.Server(arena_bytes=arena, slots=8) as srv:
        subs = [srv.submit(t, p, w, lmax) for (n, lmax, _), (t, p, w) in zip(reqs, inputs)]
        stats = [srv.wait(tk) for tk, _, _ in subs]
    assert all(s.status == 0 and s.footprint_bytes == foot for s in stats)
    for s in stats:                       # scratch held at each admission <= arena
        held = sum(o.footprint_bytes for o in stats if o.admit_s <= s.admit_s < o.done_s)
        assert held <= arena
        assert sum(1 for o in stats if o.admit_s <= s.admit_s < o.done_s) <= 3
    admits = [s.admit_s for s in stats]   # tickets were submitted in list order
    assert all(a <= b for a, b in zip(admits, admits[1:])), "admission overtook an earlier request"
    for (n, lmax, _), (t, p, w), (tk, alm, cl) in zip(reqs[:2], inputs[:2], subs[:2]):
        solo = lib.alm_from_points(t, p, w, lmax)
        torch.cuda.synchronize()
        assert torch.equal(alm, solo)


def test_small_request_overtakes_large_ones(lib):
    import torch
    cats = [catalog(2_000_000, 95), catalog(2_000_000, 96), catalog(10_000, 97)]
    lmaxes = (1024, 1024, 64)
    ins = [(dev(t), dev(p), dev(w)) for t, p, w in cats]
    torch.cuda.synchronize()
    with lib.Server(arena_bytes=4 << 30, slots=2) as srv:
        subs = [srv.submit(t, p, w, lmax) for (t, p, w), lmax in zip(ins, lmaxes)]
        stats = [srv.wait(tk) for tk, _, _ in subs]
    assert all(s.status == 0 for s in stats)
    print("done after submission (s):", [round(s.done_s - s.submit_s, 4) for s in stats], flush=True)
    assert stats[2].done_s < min(stats[0].done_s, stats[1].done_s), "the small request waited for the large ones"
    for (tk, alm, cl), (t, p, w), lmax in zip(subs, ins, lmaxes):
        solo = lib.alm_from_points(t, p, w, lmax)
        torch.cuda.synchronize()
        assert torch.equal(alm, solo)


def test_refusals_and_shutdown(lib):
    import torch
    t, p, w = [dev(a) for a in catalog(50_000, 91)]
    with lib.Server(arena_bytes=1 << 20, slots=2) as srv:
        with pytest.raises(lib.PtalmError) as ei:
            srv.submit(t, p, w, 1024)             # scratch far beyond 1 MiB
        assert ei.value.code == lib.PTALM_EBUSY
        with pytest.raises(lib.PtalmError) as ei:
            srv.submit(t, p, w, 64, precision=lib.BF16X3)
        assert ei.value.code == lib.PTALM_EINVAL
        with pytest.raises(lib.PtalmError):
            srv.submit(t, p, w, 20000)
    srv = lib.Server(arena_bytes=256 << 20, slots=2)
    subs = [srv.submit(t, p, w, lmax) for lmax in (32, 64, 96)]
    srv.close()                                   # completes the pending requests
    for (tk, alm, cl), lmax in zip(subs, (32, 64, 96)):
        solo = lib.alm_from_points(t, p, w, lmax)
        torch.cuda.synchronize()
        assert torch.equal(alm, solo)
