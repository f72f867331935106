#!/usr/bin/env python3
"""Throughput benchmark of the direct point-to-harmonic transform on one MI355X.

A step is one pass of the whole path over one synthetic catalog resident in
HBM: the transform a_lm = sum_i w_i Y*_lm (ptalm_alm_from_points) followed by
its pseudo-spectrum (ptalm_cl_from_alm); the two-catalog workload adds the FKP
field (alpha, delta = a_d - alpha a_r, window = alpha a_r) and both spectra.
The metric is point.(l,m) terms per second: terms = n * (lmax+1)(lmax+2)/2 per
transform.  Prints ONE JSON line.

Workloads (--workload):
  randoms3072  1e8 uniform-in-mask randoms, unit weights, lmax 3072   (default)
  galaxies1024 2e6 clustered galaxies (lognormal weights) + 2e7 randoms, lmax 1024
  fullsky64    1e4 uniform full-sky points, unit weights, lmax 64
  multi2048    1e7 masked positions shared by 32 lognormal weight vectors, lmax 2048,
               split-bf16 MFMA form; tuned by the library's autotuner on a prefix,
               then each step replays one captured HIP graph (transform + 32 spectra)
  spline3072   the randoms3072 catalog through the interpolated transform of App. A.2:
               cubic Hermite splines on pi (lmax+1) + 1 nodes uniform in theta (the
               spacing of 2 (lmax+1) nodes uniform in x at the equator), polar caps
               theta < 1 deg by the exact sum; value = point.(l,m) terms of the exact sum
               it replaces per second; error vs the exact GPU sum on the first 2e6 points
  shear3072    1e7 clustered masked galaxies (lognormal weights) with shear components
               g1, g2 ~ N(0, 0.26^2), lmax 3072: the spin +-2 transform to E and B
               (ptalm_shear_alm_from_points) and the EE, BB, EB spectra; value =
               point.(l,m) terms per second, one term covering both spins
  spline1000   the configuration the paper times its own method on (1e8 points, lmax ~1000,
               2048 nodes uniform in x, ~30 s on 4 A100s): 1e8 full-sky uniform points,
               lmax 1000, 3217 nodes uniform in theta (the same equatorial spacing), 1 deg
               caps; the paper's equivalent rate (1.7e12 terms/s on other hardware) is quoted
               beside it as context, not as a baseline
  coupling3072 mode coupling and bandpowers from a window spectrum W_l (l <= 6144) and a
               pseudo-spectrum (l <= 3072): shot noise of 1e8 unit-weight randoms scaled by
               alpha, M_ll' (l, l' <= 3072) with the shot noise removed from W, decoupled
               and normalised bandpowers (delta_l 25 from l = 2); value = terms of the
               coupling sum (l, l', lambda) per second
  served       a Poisson stream (50/s) of 500 masked catalogs, n log-uniform in
               [1e4, 1e7], lmax uniform in {128, ..., 2048}, through the library's
               request server; value = terms/s of the stream, with p50/p99 latency,
               the same trace time-scaled to 0.7x the measured capacity, and a
               burst of the first 100 requests served vs run one after another

Besides value, the line carries the roofline of the transform kernel (the FP64
work it executes, 6.5 flops per term, over its device time measured with HIP
events the library records on the launch stream, and the fraction of VALU issue
slots its 3.5 instructions per term fill), the CPU oracle timed on a bounded
prefix of the same catalog, and a sampled parity check of the full result
against oracle entries computed over every point.  The default workload adds
one mixed-precision step on the same catalog (rate and error per l against the
FP64 result) when the budget leaves room for it.

Wall-clock budget: the whole run, from process start, is kept within
--time-budget seconds (480 by default).  --steps and --warmup are upper
limits: the first step measures a step's duration, the checks run after it,
and only the warmup and timed steps that still fit are run (at least one
timed).  The line reports the steps actually timed (steps, warmup) beside the
requested ones (steps_requested, warmup_requested).
"""
import argparse
import json
import math
import os
import sys
import time

START = time.monotonic()      # the wall-clock budget counts from here (torch import and generation included)

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

FP64_PEAK_TFLOPS = 78.6       # MI355X FP64 vector peak (256 CUs x 2.4 GHz x 128 flop/clk/CU)
BF16_PEAK_TFLOPS = 2500.0     # MI355X dense bf16 matrix peak
MULTI_FLOPS_PER_TERM = 4      # per (point, l, m, weight vector): re and im multiply-adds
FLOPS_PER_TERM = 6.5          # FP64 flops the direct kernel executes per term: 3 FMA + 0.5 MUL
VALU_INSTS_PER_TERM = 3.5     # its FP64 VALU instructions per term (split recurrence 1.5, accumulate 2)
VALU_ISSUE_PER_S = 256 * 2.4e9 * 64   # lane-instructions/s: 256 CUs, 4 SIMDs x 16 lanes, 2.4 GHz
SPIN_FLOPS_PER_TERM = 16      # spin +-2: two step factors, two chains, four accumulate FMAs
METRIC = "point\u00b7(l,m) terms/s FP64 vs mixed at stated rel err; served p50/p99 latency"
UNIT = "point\u00b7(l,m) terms/s"

WORKLOADS = {
    "randoms3072": dict(desc="masked randoms n=1e8, unit weights, lmax=3072", lmax=3072),
    "galaxies1024": dict(desc="masked galaxies n=2e6 (2% jittered copies, lognormal sigma=0.3) + masked randoms "
                              "n=2e7, lmax=1024, C_l of galaxies - alpha randoms and W_l", lmax=1024),
    "fullsky64": dict(desc="full-sky uniform n=1e4, unit weights, lmax=64", lmax=64),
    "served": dict(desc="Poisson stream 50/s of masked catalogs, n log-uniform [1e4, 1e7], lmax uniform in "
                        "{128,256,512,1024,2048}, lognormal sigma=0.3 weights, through the request server", lmax=2048),
    "spline3072": dict(desc="masked randoms n=1e8, unit weights, lmax=3072, interpolated transform (App. A.2): "
                            "pi (lmax+1) + 1 = 9655 spline nodes uniform in theta, polar caps < 1 deg by the exact sum", lmax=3072),
    "shear3072": dict(desc="masked galaxies n=1e7 (2% jittered copies, lognormal sigma=0.3) with shear g1, g2 ~ "
                           "N(0, 0.26^2), lmax=3072, spin +-2 transform to E and B modes + EE/BB/EB spectra", lmax=3072),
    "spline1000": dict(desc="the paper's timing configuration: full-sky n=1e8 uniform points, unit weights, lmax=1000, "
                            "interpolated transform (App. A.2) with 3217 nodes uniform in theta (the equatorial "
                            "spacing of 2048 nodes uniform in x), polar caps < 1 deg by the exact sum", lmax=1000,
                       nodes=3217),
    "coupling3072": dict(desc="mode coupling lmax=3072 from W_l to 6144 (shot noise of n=1e8 unit-weight randoms "
                              "removed), decoupled and normalised bandpowers delta_l=25 from l=2", lmax=3072),
    "multi2048": dict(desc="one masked position set n=1e7 shared by 32 lognormal weight vectors (sigma=0.2), "
                           "lmax=2048, split-bf16 MFMA form", lmax=2048),
}


LONG_STEP_S = 20.0   # steps at least this long report their end as they finish


class Budget:
    """Wall-clock budget of one bench run, counted from process start.  --steps and --warmup are
    upper limits: a step whose measured duration no longer fits is not started."""

    def __init__(self, seconds):
        self.end = START + seconds

    def left(self):
        return self.end - time.monotonic()


def run_steps(step, sync, warmup, steps, budget, reserve_s=0.0, after_first=None, label="step",
              optional=None, min_timed_with_optional=2):
    """Up to `warmup` untimed and `steps` timed steps, inside the budget, timed steps first.
    The first step runs alone (synchronized) to measure a step's duration; `after_first`
    (checks that read a finished step's output) runs right after it when that step is a
    warmup.  Then the steps that still fit are shared out: timed steps first (at least one),
    further warmups only with time to spare.  `reserve_s` seconds are kept free for work after
    the timed steps, and, when optional = (k, s) is given, k step durations plus s seconds more
    for an optional run after them if at least `min_timed_with_optional` timed steps still fit
    beside it.  Returns a dict: warmup_done, steps (timed), elapsed_s (over the timed steps),
    step_s (duration of one step), optional (whether that time was kept free)."""
    done_w = 0
    step_s = None
    timed = 0
    if warmup > 0:
        print(f"[bench] warmup {label} 0", file=sys.stderr, flush=True)
        t = time.monotonic()
        step()
        sync()
        step_s = time.monotonic() - t
        done_w = 1
        if after_first is not None:
            after_first()

    def fitting(extra):
        return int(max(0.0, budget.left() - reserve_s - extra) // (step_s * 1.05)) if step_s > 0 else steps + warmup

    def optional_s():
        return 0.0 if optional is None else optional[0] * step_s * 1.05 + optional[1]

    sync()
    t0 = time.perf_counter()
    if step_s is None:          # no warmup: the first timed step measures the duration
        step()
        sync()
        step_s = time.perf_counter() - t0
        timed = 1
        print(f"[bench] timed {label} 0 done ({step_s:.2f} s)", file=sys.stderr, flush=True)
        n = max(0, min(steps - timed, fitting(0.0)))
        keep_optional = optional is not None and timed + fitting(optional_s()) >= min_timed_with_optional
        if keep_optional:
            n = max(0, min(steps - timed, fitting(optional_s())))
    else:
        keep_optional = optional is not None and fitting(optional_s()) >= min_timed_with_optional
        fit = fitting(optional_s() if keep_optional else 0.0)
        n = max(1, min(steps, fit))
        more_w = max(0, min(warmup - done_w, fit - n))
        for _ in range(more_w):
            print(f"[bench] warmup {label} {done_w}", file=sys.stderr, flush=True)
            step()
            if step_s >= LONG_STEP_S:
                sync()
            done_w += 1
        sync()
        t0 = time.perf_counter()
    if n > 0:
        print(f"[bench] timing {n} {'more ' if timed else ''}{label}(s) ({timed + n} of {steps} requested fit the "
              f"budget)", file=sys.stderr, flush=True)
    for i in range(n):
        step()
        if step_s >= LONG_STEP_S:
            # a long step ends with a synchronization and a progress line (one wait per
            # step of tens of seconds costs nothing measurable; short steps stay queued)
            sync()
            print(f"[bench] timed {label} {timed + i + 1} of {timed + n} done", file=sys.stderr, flush=True)
    sync()
    elapsed = time.perf_counter() - t0
    timed += n
    print(f"[bench] {timed} timed {label}(s) in {elapsed:.2f} s", file=sys.stderr, flush=True)
    return {"warmup_done": done_w, "steps": timed, "elapsed_s": elapsed, "step_s": step_s,
            "optional": keep_optional}


PROFILES = os.path.join(HERE, "profiles")
# the kernel and the work plan that decides its launch, per workload with a recorded traffic
# summary (a change to either voids the record)
CSRC = os.path.join(HERE, "paper_2312_12285_amd", "csrc")
TRAFFIC_SOURCES = {
    "randoms3072": (["alm_direct.hip", "wave_common.h"],
                    ("api.hip", "// Default kernel variant and decomposition.", "size_t align256(size_t b)")),
    "spline3072": (["spline.hip", "wave_common.h"], None),
    "spline1000": (["spline.hip", "wave_common.h"], None),
    "shear3072": (["spin.hip", "wave_common.h"],
                  ("api.hip", "// Default spin kernels:", "size_t ptalm_shear_workspace_bytes(")),
    "coupling3072": (["coupling.hip"], None),
    "multi2048": (["alm_multi.hip"],
                  ("api.hip", "// Default kernel variant and decomposition.", "size_t align256(size_t b)")),
}


def kernel_source_hash(workload="randoms3072"):
    """sha256 (first 16 hex digits) of the dominant kernel's sources and of the part of
    api.hip that picks its launch, for a workload with a recorded traffic summary."""
    import hashlib
    files, plan = TRAFFIC_SOURCES[workload]
    h = hashlib.sha256()
    for name in files:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    if plan is not None:
        name, start, end = plan
        with open(os.path.join(CSRC, name)) as f:
            text = f.read()
        h.update(text[text.index(start):text.index(end)].encode())
    return h.hexdigest()[:16]


def copy_calibration():
    """A plain 1 GiB device-to-device copy (1 GiB read, 1 GiB written): counter runs scale the
    FETCH_SIZE and WRITE_SIZE of the measured kernel by what the counters read for it."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def recorded_traffic(workload, variant):
    """HBM bytes per launch of the workload's dominant kernel from the committed rocprofv3
    PMC summary (FETCH_SIZE, WRITE_SIZE scaled by a copy-kernel calibration), or None when
    no summary exists for this workload/variant or its sources changed since."""
    if workload not in TRAFFIC_SOURCES:
        return None
    path = os.path.join(PROFILES, f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash(workload) or rec.get("variant") != variant:
        return None
    return rec.get("hbm_bytes_per_launch")


def tri(lmax):
    return (lmax + 1) * (lmax + 2) // 2


def make_catalogs(name, scale):
    from paper_2312_12285_amd import synth
    if name in ("randoms3072", "spline3072"):
        return [("randoms", synth.masked_randoms(int(1e8 * scale), seed=31))]
    if name == "spline1000":
        import numpy as np
        t, p = synth.uniform_sphere(int(1e8 * scale), 33)
        return [("points", synth.Catalog(t, p, np.ones(t.size)))]
    if name == "galaxies1024":
        return [("galaxies", synth.masked_galaxies(int(2e6 * scale), seed_pos=21, seed_w=22)),
                ("randoms", synth.masked_randoms(int(2e7 * scale), seed=23))]
    if name == "shear3072":
        return [("galaxies", synth.masked_galaxies(int(1e7 * scale), seed_pos=61, seed_w=62))]
    if name == "fullsky64":
        return [("points", synth.fullsky_uniform(10_000, seed=1))]
    if name == "multi2048":
        t, p, W = synth.multi_weight_positions(int(1e7 * scale), 32, seed_pos=41, seed_w0=4100)
        return [("positions", synth.Catalog(t, p, W))]
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(cats, lmax, seconds_target):
    """The oracle, untuned, on a prefix of the first catalog sized for ~seconds_target."""
    from oracle import ref
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    cat = cats[0][1]
    T = tri(lmax)
    k = max(64, min(cat.n, 512))
    t0 = time.time()
    ref.alm_from_points(cat.theta[:k], cat.phi[:k], cat.w[:k], lmax, nthreads=nthreads)
    dt = time.time() - t0
    rate = k * T / dt
    k2 = int(min(cat.n, max(k, rate * seconds_target / T)))
    if k2 > k:
        t0 = time.time()
        ref.alm_from_points(cat.theta[:k2], cat.phi[:k2], cat.w[:k2], lmax, nthreads=nthreads)
        dt = time.time() - t0
        k = k2
        rate = k * T / dt
    return {"value": rate, "unit": UNIT, "cores": nthreads, "kind": "oracle",
            "sample": f"first {k} points of the {cats[0][0]} catalog at lmax {lmax} ({k * T:.3g} terms, {dt:.1f} s)"}


def sampled_parity(cat, lmax, alm_dev):
    """Compare a few a_lm of the full result with oracle entries summed over every point."""
    import numpy as np
    from oracle import ref
    from paper_2312_12285_amd import ptalm
    pairs = [(0, 0), (1, 0), (1, 1), (lmax, lmax), (lmax, lmax - 1), (lmax, lmax - 3),
             (lmax // 2, lmax // 2 - 2), (min(40, lmax), min(17, lmax))]
    ls = np.array([p[0] for p in pairs]); ms = np.array([p[1] for p in pairs])
    t0 = time.time()
    want = ref.alm_entries(cat.theta, cat.phi, cat.w, ls, ms)
    dt = time.time() - t0
    a = ptalm.as_complex(alm_dev).cpu().numpy()
    got = np.array([a[ptalm.alm_index(lmax, l, m)] for l, m in pairs])
    # each entry against the size of a typical coefficient at its l
    cl = ptalm.cl_from_alm(alm_dev, lmax).cpu().numpy()
    scale = np.sqrt(np.maximum(cl[ls], 1e-300))
    rel = np.abs(got - want) / scale
    return {"entries": [f"({l},{m})" for l, m in pairs], "max_err_over_rms_l": float(rel.max()),
            "oracle_seconds": round(dt, 1)}


def per_l_errors(got, ref, lmax):
    """Per-l norm-wise relative error over m, the global norm-wise error, and a few l."""
    import numpy as np
    L = np.concatenate([np.arange(m, lmax + 1) for m in range(lmax + 1)])
    num = np.bincount(L, weights=np.abs(got - ref) ** 2, minlength=lmax + 1)
    den = np.bincount(L, weights=np.abs(ref) ** 2, minlength=lmax + 1)
    per_l = np.sqrt(num / np.maximum(den, 1e-300))
    pick = sorted({0, 1, 10, 100, lmax // 4, lmax // 2, lmax})
    return {"global": float(np.sqrt(num.sum() / den.sum())), "max_per_l": float(per_l.max()),
            "l_of_max": int(per_l.argmax()), "per_l": {str(l): float(per_l[l]) for l in pick}}


def precision_errors(args, cat, lmax, alm_dev, prec):
    """Error of a reduced-precision result: against the FP64 GPU path on the full catalog
    (itself gated against the oracle), and against the oracle on the first 1e4 points."""
    import numpy as np
    import torch
    from oracle import ref
    from paper_2312_12285_amd import ptalm
    t = torch.as_tensor(cat.theta).cuda(); p = torch.as_tensor(cat.phi).cuda(); w = torch.as_tensor(cat.w).cuda()
    full64 = ptalm.alm_from_points(t, p, w, lmax)
    got = ptalm.as_complex(alm_dev).cpu().numpy()
    out = {"vs_fp64_gpu_full_catalog": per_l_errors(got, ptalm.as_complex(full64).cpu().numpy(), lmax)}
    k = min(cat.n, 10_000)
    sub = ptalm.alm_from_points(t[:k].contiguous(), p[:k].contiguous(), w[:k].contiguous(), lmax,
                                options=ptalm.opts(precision=prec))
    want = ref.alm_from_points(cat.theta[:k], cat.phi[:k], cat.w[:k], lmax)
    out[f"vs_oracle_first_{k}_points"] = per_l_errors(ptalm.as_complex(sub).cpu().numpy(), want, lmax)
    return out


def run_multi(args, cats, lmax):
    """multi2048: autotune on a prefix, capture transform + spectra once, replay per step."""
    import numpy as np
    import torch
    from paper_2312_12285_amd import ptalm, synth
    T = tri(lmax)
    cat = cats[0][1]
    n, nw = cat.n, cat.w.shape[0]
    t = torch.as_tensor(cat.theta).cuda()
    p = torch.as_tensor(cat.phi).cuda()
    w = torch.as_tensor(cat.w).cuda()
    if args.multi_slices > 0:
        n_slices = args.multi_slices
        o = ptalm.opts(precision=ptalm.BF16X3, n_weights=nw, n_slices=n_slices)
    else:
        k = min(n, 1_000_000)
        print(f"[bench] autotune on the first {k} positions", file=sys.stderr, flush=True)
        best = ptalm.autotune(t[:k].contiguous(), p[:k].contiguous(), w[:, :k].contiguous(), lmax,
                              precision=ptalm.BF16X3)
        torch.cuda.synchronize()
        n_slices = best.n_slices
        o = ptalm.opts(precision=ptalm.BF16X3, n_weights=nw)      # auto fields take the tuned choice
    ptalm.prepare_call(n, lmax, o)
    ws = torch.empty(ptalm.workspace_bytes(n, lmax, o), dtype=torch.uint8, device="cuda")
    out = torch.empty((nw, 2 * T), dtype=torch.float64, device="cuda")
    cls = torch.empty((nw, lmax + 1), dtype=torch.float64, device="cuda")

    def body():
        ptalm.alm_from_points(t, p, w, lmax, out=out, options=o, workspace=ws)
        for v in range(nw):
            ptalm.cl_from_alm(out[v], lmax, out=cls[v])

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        body()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    print("[bench] capturing one step into a HIP graph", file=sys.stderr, flush=True)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        body()
    evs = []

    def step():
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        b.record()
        evs.append((a, b))

    res = run_steps(step, torch.cuda.synchronize, args.warmup, args.steps, Budget(args.time_budget),
                    reserve_s=30.0 + args.cpu_seconds, label="graph replay")
    elapsed, steps = res["elapsed_s"], res["steps"]
    step_ms = float(np.mean([a.elapsed_time(b) for a, b in evs[res["warmup_done"]:]]))
    weight_terms = nw * n * T
    value = weight_terms * steps / elapsed
    useful = MULTI_FLOPS_PER_TERM * weight_terms
    achieved = useful / (step_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / BF16_PEAK_TFLOPS, 4),
                # the slice count moves this kernel's traffic by under 5%: one record serves every S
                "traffic": recorded_traffic(args.workload if args.scale == 1.0 else None, f"bf16x3,nw={nw}"),
                "kernel": "alm_multi_kernel<32>", "kernel_ms_per_launch": round(step_ms, 3),
                "timed_span": "whole replayed graph (transform + 32 spectra), events on the replay stream",
                "flops_per_weight_term": MULTI_FLOPS_PER_TERM, "issued_mfma_flops_per_useful": 3}
    line = {"metric": METRIC, "value": value, "unit": UNIT + " (summed over the weight vectors)",
            "n_gpus": 1, "steps": steps, "warmup": res["warmup_done"], "steps_requested": args.steps,
            "warmup_requested": args.warmup, "ms_per_step": round(1e3 * elapsed / steps, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16x3 split products, f32 accumulate, f64 recurrence", "data": "synthetic",
            "config": {"workload": WORKLOADS[args.workload]["desc"], "lmax": lmax, "points": n, "weight_vectors": nw,
                       "position_terms_per_step": n * T, "weight_terms_per_step": weight_terms,
                       "n_slices": n_slices, "n_slices_from": "flag" if args.multi_slices > 0 else "autotune",
                       "hip_graph": True},
            "roofline": roofline}
    if not args.no_check:
        print("[bench] sampled parity against oracle entries (weight vectors 0 and 31)", file=sys.stderr, flush=True)
        line["parity"] = {f"w{v}": sampled_parity(synth.Catalog(cat.theta, cat.phi, cat.w[v]), lmax, out[v])
                          for v in (0, nw - 1)}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, weight vector 0)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline([("positions with weight vector 0",
                                              synth.Catalog(cat.theta, cat.phi, cat.w[0]))], lmax, args.cpu_seconds)
    print(json.dumps(line), flush=True)


SPLINE_CUT_DEG = 1.0
SPLINE_FLOPS_PER_TERM = 22      # per (point, m) of the binning: 4 complex x real multiply-adds + the phase rotation
PAPER_SHT_RATE = 1.7e12         # the paper's own method: 1e8 points x T(1000) / ~30 s on 4 A100s (context)


def spline_nodes(lmax):
    return int(round(math.pi * (lmax + 1))) + 1


def run_spline(args, cats, lmax):
    """spline3072 / spline1000: the interpolated transform."""
    import numpy as np
    import torch
    from oracle import ref, spline
    from paper_2312_12285_amd import ptalm
    cat = cats[0][1]
    n = cat.n
    wl = WORKLOADS[args.workload]
    nodes = wl.get("nodes") or spline_nodes(lmax)
    cut = math.radians(SPLINE_CUT_DEG)
    t = torch.as_tensor(cat.theta).cuda(); p = torch.as_tensor(cat.phi).cuda(); w = torch.as_tensor(cat.w).cuda()
    T = tri(lmax)
    out = torch.empty(2 * T, dtype=torch.float64, device="cuda")
    ptalm.prepare(lmax)     # the polar part's direct-sum tables, outside the timed region
    opt = ptalm.opts(timing=1)
    evs, bin_ms = [], []

    def step():
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        ptalm.alm_from_points_spline(t, p, w, lmax, nodes, cut, out=out, options=opt)
        b.record()
        evs.append((a, b))
        bin_ms.append(ptalm.last_timing_ms())
        ptalm.cl_from_alm(out, lmax)

    res = run_steps(step, torch.cuda.synchronize, args.warmup, args.steps, Budget(args.time_budget),
                    reserve_s=90.0 + args.cpu_seconds)
    elapsed, steps, wd = res["elapsed_s"], res["steps"], res["warmup_done"]
    call_ms = float(np.mean([a.elapsed_time(b) for a, b in evs[wd:]]))
    k_ms = float(np.mean(bin_ms[wd:]))
    theta = cat.theta
    n_polar = int(((theta < cut) | (theta > math.pi - cut)).sum())
    flops = SPLINE_FLOPS_PER_TERM * (n - n_polar) * (lmax + 1)
    achieved = flops / (k_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": recorded_traffic(args.workload if args.scale == 1.0 else None, "bin_kernel"),
                "kernel": "bin_kernel (per-m binned Hermite weights)", "kernel_ms_per_launch": round(k_ms, 3),
                "flops_per_point_m": SPLINE_FLOPS_PER_TERM, "call_ms": round(call_ms, 3),
                "call_tflops": round(flops / (call_ms * 1e-3) / 1e12, 3)}
    line = {"metric": METRIC, "value": n * T * steps / elapsed, "unit": UNIT + " (of the exact sum replaced)",
            "n_gpus": 1, "steps": steps, "warmup": wd, "steps_requested": args.steps,
            "warmup_requested": args.warmup, "ms_per_step": round(1e3 * elapsed / steps, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": wl["desc"], "lmax": lmax, "points": n, "nodes": nodes,
                       "theta_cut_deg": SPLINE_CUT_DEG, "polar_points": n_polar},
            "roofline": roofline}
    if args.workload == "spline1000":
        # the paper's own method on the configuration it is timed on: other hardware, so context only
        line["paper_context"] = {"value": PAPER_SHT_RATE, "unit": UNIT + " (of the exact sum replaced)",
                                 "what": "the paper's interpolated transform, 1e8 points, lmax ~1000, 2048 nodes, "
                                         "~30 s on 4 A100s, as the exact-sum rate it replaces"}
    if not args.no_check:
        print("[bench] error vs the exact GPU sum on the first 2e6 points", file=sys.stderr, flush=True)
        k = min(n, 2_000_000)
        a_s = ptalm.alm_from_points_spline(t[:k].contiguous(), p[:k].contiguous(), w[:k].contiguous(), lmax, nodes, cut)
        a_d = ptalm.alm_from_points(t[:k].contiguous(), p[:k].contiguous(), w[:k].contiguous(), lmax)
        line["interpolation_error_first_2e6"] = per_l_errors(ptalm.as_complex(a_s).cpu().numpy(),
                                                             ptalm.as_complex(a_d).cpu().numpy(), lmax)
        print("[bench] sampled parity with the oracle's interpolated transform (full catalog)", file=sys.stderr,
              flush=True)
        pairs = [(0, 0), (2, 1), (100, 0), (lmax // 2, lmax // 4), (lmax, 0), (lmax, lmax - lmax // 40)]
        t1 = time.time()
        want = spline.alm_spline_entries(cat.theta, cat.phi, cat.w, lmax, nodes, cut, pairs)
        a = ptalm.as_complex(out).cpu().numpy()
        got = np.array([a[ptalm.alm_index(lmax, l, m)] for l, m in pairs])
        clh = ptalm.cl_from_alm(out, lmax).cpu().numpy()
        scale = np.sqrt(np.maximum(clh[[l for l, _ in pairs]], 1e-300))
        line["parity"] = {"entries": [f"({l},{m})" for l, m in pairs],
                          "max_err_over_rms_l": float((np.abs(got - want) / scale).max()),
                          "oracle_seconds": round(time.time() - t1, 1)}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle interpolated transform, sampled coefficients)", file=sys.stderr,
              flush=True)
        pairs = [(lmax, 0), (lmax, lmax // 2), (2 * lmax // 3, 100), (lmax // 3, lmax // 3 - 1), (lmax // 6, 7),
                 (lmax, lmax), (10, 5), (lmax // 2, 1)]
        k = min(n, int(7e6 * 3073 / (lmax + 1)))
        t1 = time.time()
        spline.alm_spline_entries(cat.theta[:k], cat.phi[:k], cat.w[:k], lmax, nodes, cut, pairs)
        dt = time.time() - t1
        nthreads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        line["cpu_baseline"] = {"value": k * len(pairs) / dt, "unit": UNIT + " (of the exact sum replaced)",
                                "cores": nthreads, "kind": "oracle",
                                "sample": f"{len(pairs)} coefficients (l, m) of the first {k} points, lmax {lmax}, "
                                          f"{nodes} nodes ({dt:.1f} s; node values by the C oracle, binning in numpy)"}
    print(json.dumps(line), flush=True)


SHEAR_PAIRS = [(2, 0), (2, 2), (3, 1), (100, 37), (1536, 700), (3072, 3072), (3072, 3000), (3071, 1)]


def run_shear(args, cats, lmax):
    """shear3072: spin +-2 transform to E/B of a shear catalog and its three spectra."""
    import numpy as np
    import torch
    from oracle import ref
    from paper_2312_12285_amd import ptalm, synth
    cat = cats[0][1]
    n = cat.n
    g1, g2 = synth.shear_components(n, seed=63)
    d = [torch.as_tensor(a).cuda() for a in (cat.theta, cat.phi, cat.w, g1, g2)]
    T = tri(lmax)
    e = torch.empty(2 * T, dtype=torch.float64, device="cuda")
    b = torch.empty(2 * T, dtype=torch.float64, device="cuda")
    cls = [torch.empty(lmax + 1, dtype=torch.float64, device="cuda") for _ in range(3)]
    opt = ptalm.opts(points_per_lane=args.points_per_lane, l_block=args.l_block, timing=1)
    kernel_ms = []

    def step():
        ptalm.shear_alm_from_points(*d, lmax, out_e=e, out_b=b, options=opt)
        kernel_ms.append(ptalm.last_timing_ms())
        ptalm.cl_from_alm(e, lmax, out=cls[0])
        ptalm.cl_from_alm(b, lmax, out=cls[1])
        ptalm.cross_cl(e, b, lmax, out=cls[2])

    res = run_steps(step, torch.cuda.synchronize, args.warmup, args.steps, Budget(args.time_budget),
                    reserve_s=40.0 + args.cpu_seconds)
    elapsed, steps, wd = res["elapsed_s"], res["steps"], res["warmup_done"]
    terms = n * T
    k_ms = float(np.mean(kernel_ms[wd:]))
    achieved = SPIN_FLOPS_PER_TERM * terms / (k_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": recorded_traffic(args.workload if args.scale == 1.0 else None,
                                            f"kp={args.points_per_lane or 'default'},lb={args.l_block or 'default'}"),
                "kernel": "spin_direct_kernel<4, 8>" if not (args.points_per_lane or args.l_block) else
                          f"spin_direct_kernel<{args.points_per_lane or 4}, {args.l_block or 8}>",
                "kernel_ms_per_launch": round(k_ms, 3), "flops_per_term": SPIN_FLOPS_PER_TERM}
    line = {"metric": METRIC, "value": terms * steps / elapsed, "unit": UNIT + " (spin +-2, both spins per term)",
            "n_gpus": 1, "steps": steps, "warmup": wd, "steps_requested": args.steps,
            "warmup_requested": args.warmup, "ms_per_step": round(1e3 * elapsed / steps, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": WORKLOADS["shear3072"]["desc"], "lmax": lmax, "points": n, "terms_per_step": terms},
            "roofline": roofline}
    if not args.no_check:
        print("[bench] sampled parity against the oracle's spin entries (every point)", file=sys.stderr, flush=True)
        t1 = time.time()
        ls = [l for l, _ in SHEAR_PAIRS]
        ms = [m for _, m in SHEAR_PAIRS]
        we, wb = ref.shear_eb_entries(cat.theta, cat.phi, cat.w, g1, g2, ls, ms)
        ge, gb = ptalm.as_complex(e).cpu().numpy(), ptalm.as_complex(b).cpu().numpy()
        idx = [ptalm.alm_index(lmax, l, m) for l, m in SHEAR_PAIRS]
        cle, clb = cls[0].cpu().numpy(), cls[1].cpu().numpy()
        err = max(float((np.abs(ge[idx] - we) / np.sqrt(cle[ls])).max()),
                  float((np.abs(gb[idx] - wb) / np.sqrt(clb[ls])).max()))
        line["parity"] = {"entries": [f"({l},{m})" for l, m in SHEAR_PAIRS], "max_err_over_rms_l": err,
                          "oracle_seconds": round(time.time() - t1, 1)}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle spin transform on a prefix)", file=sys.stderr, flush=True)
        nthreads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        k = 64
        t1 = time.time()
        ref.shear_eb(cat.theta[:k], cat.phi[:k], cat.w[:k], g1[:k], g2[:k], lmax, nthreads=nthreads)
        dt = time.time() - t1
        k2 = int(min(n, max(k, k * args.cpu_seconds / max(dt, 1e-3))))
        if k2 > k:
            t1 = time.time()
            ref.shear_eb(cat.theta[:k2], cat.phi[:k2], cat.w[:k2], g1[:k2], g2[:k2], lmax, nthreads=nthreads)
            dt = time.time() - t1
            k = k2
        line["cpu_baseline"] = {"value": k * T / dt, "unit": UNIT + " (spin +-2, both spins per term)",
                                "cores": nthreads, "kind": "oracle",
                                "sample": f"first {k} galaxies at lmax {lmax} ({k * T:.3g} terms, {dt:.1f} s)"}
    print(json.dumps(line), flush=True)


def spline_error_table():
    """Pointwise interpolation error of y_lm(x) for the configurations of the paper's figure on
    it (l = 500; m = 0, 125, 250; N_x = N_l/2, N_l, 2 N_l with N_l = 501), with the nodes
    uniform in x over [-1, 1] and with the same number uniform in theta, evaluated on
    |x| <= 3/4 (the paper's equatorial region).  CPU only (the oracle)."""
    import numpy as np
    from oracle import spline
    l, Nl = 500, 501
    x_eval = np.linspace(-0.75, 0.75, 6001)
    rows = []
    for nx in (Nl // 2, Nl, 2 * Nl):
        xu = np.linspace(-1.0, 1.0, nx)
        xu = xu[np.abs(xu) < 0.9]
        th = np.linspace(math.pi, 0.0, nx)
        xt = np.cos(th)
        xt = xt[np.abs(xt) < 0.9]
        for m in (0, 125, 250):
            eu, amp = spline.interpolation_error(l, m, xu, x_eval)
            et, _ = spline.interpolation_error(l, m, xt, x_eval)
            rows.append({"N_x": nx, "l": l, "m": m, "max_abs_err_x_uniform": eu, "max_abs_err_theta_uniform": et,
                         "max_abs_y": amp})
    return rows


COUPLING_LW = 6144
COUPLING_DL, COUPLING_LMIN = 25, 2
COUPLING_RANDOMS = 100_000_000


def coupling_terms(lmax, lmax_w, rows=None):
    """Terms (l, l', lambda) of the coupling sum (eq. chat) over rows l (all if None) and all
    l' <= lmax: lambda runs over |l - l'| .. min(l + l', lmax_w) in steps of 2."""
    import numpy as np
    ls = np.arange(lmax + 1) if rows is None else np.asarray(rows)
    lp = np.arange(lmax + 1)
    lo = np.abs(ls[:, None] - lp[None, :])
    hi = np.minimum(ls[:, None] + lp[None, :], lmax_w)
    return int(np.maximum((hi - lo) // 2 + 1, 0).sum())


def run_coupling(args):
    """coupling3072: shot noise, coupling matrix, both bandpower conventions per step."""
    import numpy as np
    import torch
    from oracle import ref
    from paper_2312_12285_amd import ptalm, synth
    lmax, lw = WORKLOADS["coupling3072"]["lmax"], COUPLING_LW
    n_r = int(COUPLING_RANDOMS * args.scale)
    W = synth.window_spectrum(lw, seed=5)
    cl = synth.pseudo_spectrum(lmax, seed=6)
    Wd = torch.as_tensor(W).cuda()
    cld = torch.as_tensor(cl).cuda()
    wr = torch.ones(n_r, dtype=torch.float64, device="cuda")
    alpha = torch.tensor([0.02], dtype=torch.float64, device="cuda")
    shot = torch.empty(1, dtype=torch.float64, device="cuda")
    M = torch.empty((lmax + 1, lmax + 1), dtype=torch.float64, device="cuda")
    terms = coupling_terms(lmax, lw)
    diag = sum(min(2 * l, lw) // 2 + 1 for l in range(lmax + 1))
    half_terms = (terms + diag) // 2      # each unordered pair (l, l') once: the contraction's work
    cms = []

    def step():
        ptalm.window_shot_noise(wr, alpha, out=shot)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        ptalm.coupling_matrix(Wd, lmax, shot=shot, out=M)
        b.record()
        cms.append((a, b))
        cb, win = ptalm.bandpowers(cld, M, lmax, COUPLING_DL, lmin=COUPLING_LMIN, mode=0)
        cbn, winn = ptalm.bandpowers(cld, M, lmax, COUPLING_DL, lmin=COUPLING_LMIN, mode=1, Wl=Wd)
        return cb, cbn

    res = run_steps(step, torch.cuda.synchronize, args.warmup, args.steps, Budget(args.time_budget),
                    reserve_s=30.0 + args.cpu_seconds)
    elapsed, steps, wd = res["elapsed_s"], res["steps"], res["warmup_done"]
    k_ms = float(np.mean([a.elapsed_time(b) for a, b in cms[wd:]]))
    flops = 2.0 * half_terms       # one multiply-add per term of the contraction, each unordered (l, l') once
    achieved = flops / (k_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": recorded_traffic(args.workload, "tables+mfma per call"),
                "kernel": "coupling_t_kernel + coupling_mfma_kernel (one ptalm_coupling_matrix call)",
                "kernel_ms_per_launch": round(k_ms, 4), "flops_per_term": 2,
                "terms_per_launch": half_terms}
    line = {"metric": "coupling-sum terms (l,l',lambda)/s, mode coupling + bandpowers", "value": terms * steps / elapsed,
            "unit": "(l,l',lambda) terms/s", "n_gpus": 1, "steps": steps, "warmup": wd,
            "steps_requested": args.steps, "warmup_requested": args.warmup,
            "ms_per_step": round(1e3 * elapsed / steps, 3), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": WORKLOADS["coupling3072"]["desc"], "lmax": lmax, "lmax_w": lw,
                       "randoms": n_r, "delta_l": COUPLING_DL, "lmin": COUPLING_LMIN,
                       "bins": ptalm.bandpower_count(lmax, COUPLING_LMIN, COUPLING_DL), "terms_per_step": terms},
            "roofline": roofline}
    if not args.no_check:
        print("[bench] sampled rows of M against the oracle", file=sys.stderr, flush=True)
        s = float(shot.cpu()[0])
        want_shot = 0.02 ** 2 * n_r / (4 * math.pi)
        rows = [0, 1, 1024, 2047, 3072]
        t1 = time.time()
        want = ref.coupling_rows(W - s, lmax, rows)
        got = M.cpu().numpy()[rows]
        line["parity"] = {"rows": rows, "max_rel_err": float((np.abs(got - want) / np.abs(want)).max()),
                          "shot_rel_err": abs(s - want_shot) / want_shot, "oracle_seconds": round(time.time() - t1, 1)}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle coupling rows)", file=sys.stderr, flush=True)
        nthreads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
        rows = list(range(0, lmax + 1, 128))
        t1 = time.time()
        ref.coupling_rows(W, lmax, rows, nthreads=nthreads)
        dt = time.time() - t1
        k = coupling_terms(lmax, lw, rows)
        if dt < args.cpu_seconds / 3:
            rows = list(range(0, lmax + 1, 64))
            t1 = time.time()
            ref.coupling_rows(W, lmax, rows, nthreads=nthreads)
            dt = time.time() - t1
            k = coupling_terms(lmax, lw, rows)
        line["cpu_baseline"] = {"value": k / dt, "unit": "(l,l',lambda) terms/s", "cores": nthreads, "kind": "oracle",
                                "sample": f"{len(rows)} rows of M (every {rows[1] - rows[0]}th l) at lmax {lmax}, "
                                          f"{k:.3g} terms, {dt:.1f} s"}
    print(json.dumps(line), flush=True)


def _served_catalogs(reqs, workers):
    """Host generation of every request's catalog in a fork pool (before the GPU is touched)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    from paper_2312_12285_amd import synth
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        return list(ex.map(synth.served_catalog, reqs, chunksize=2))


def run_served(args):
    """served: replay the request trace through ptalm.Server (see the module docstring)."""
    import numpy as np
    from paper_2312_12285_amd import synth
    K = args.served_requests
    reqs = synth.served_trace(K, 50.0, 51)
    workers = max(1, min(16, os.cpu_count() or 1))
    t0 = time.time()
    cats = _served_catalogs(reqs, workers)
    print(f"[bench] generated {K} catalogs ({sum(r.n for r in reqs):.3g} points) in {time.time() - t0:.1f} s "
          f"with {workers} processes", file=sys.stderr, flush=True)
    import torch
    from paper_2312_12285_amd import ptalm
    prec = {"fp64": ptalm.FP64, "mixed": ptalm.MIXED, "fp32": ptalm.FP32}[args.precision]
    dev = [(torch.as_tensor(c.theta).cuda(), torch.as_tensor(c.phi).cuda(), torch.as_tensor(c.w).cuda())
           for c in cats]
    outs = [(torch.empty(2 * tri(r.lmax), dtype=torch.float64, device="cuda"),
             torch.empty(r.lmax + 1, dtype=torch.float64, device="cuda")) for r in reqs]
    for lmax in sorted({r.lmax for r in reqs}):
        ptalm.prepare(lmax)
    torch.cuda.synchronize()
    terms = np.array([r.n * tri(r.lmax) for r in reqs], dtype=np.float64)
    arena = int(args.served_arena_gb * (1 << 30))

    def replay(arrivals, order, label):
        with ptalm.Server(arena_bytes=arena, slots=args.served_slots) as srv:
            start = time.monotonic()
            tickets = {}
            last_note = start
            for k in order:
                dt = start + arrivals[k] - time.monotonic()
                if dt > 0:
                    time.sleep(dt)
                t, p, w = dev[k]
                tickets[k] = srv.submit(t, p, w, reqs[k].lmax, precision=prec, alm=outs[k][0], cl=outs[k][1])[0]
                if time.monotonic() - last_note > 15:
                    last_note = time.monotonic()
                    print(f"[bench] {label}: submitted {len(tickets)}/{len(order)}", file=sys.stderr, flush=True)
            stats = {}
            while len(stats) < len(order):
                for k in order:
                    if k not in stats:
                        st = srv.poll(tickets[k])
                        if st is not None:
                            stats[k] = st
                time.sleep(0.002)
                if time.monotonic() - last_note > 15:
                    last_note = time.monotonic()
                    print(f"[bench] {label}: completed {len(stats)}/{len(order)}", file=sys.stderr, flush=True)
        lat = np.array([stats[k].done_s - (start + arrivals[k]) for k in order])
        slow = lat / (terms[order] / capacity_hint)       # latency over the request's time alone at capacity
        makespan = max(stats[k].done_s for k in order) - start
        tot = float(terms[order].sum())
        print(f"[bench] {label}: makespan {makespan:.1f} s, {tot / makespan:.3e} terms/s", file=sys.stderr, flush=True)
        return {"requests": len(order), "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
                "p99_latency_s": round(float(np.percentile(lat, 99)), 4), "makespan_s": round(makespan, 3),
                "terms_per_s": tot / makespan,
                "offered_terms_per_s": tot / max(1e-9, float(arrivals[order].max() - arrivals[order].min())),
                "max_queue_wait_s": round(float(max(stats[k].admit_s - (start + arrivals[k]) for k in order)), 4),
                "p50_slowdown": round(float(np.percentile(slow, 50)), 2),
                "p99_slowdown": round(float(np.percentile(slow, 99)), 2),
                "p99_of_requests_above_1e12_terms_s": round(float(np.percentile(lat[terms[order] > 1e12], 99)), 4)
                if (terms[order] > 1e12).any() else None}

    arrivals = np.array([r.arrival_s for r in reqs])
    order = list(range(K))
    capacity_hint = 5.8e12          # FP64 terms/s of one device, for the slowdown figures only
    res = replay(arrivals, order, "trace at 50/s")
    capacity = res["terms_per_s"]
    offered = float(terms.sum() / arrivals.max())
    scale = offered / (0.7 * capacity)
    res_07 = replay(arrivals * scale, order, "trace time-scaled to 0.7x capacity")
    res_07["time_scale"] = round(scale, 4)

    B = min(100, K)
    burst = replay(np.zeros(K), list(range(B)), f"burst of the first {B}")
    served_alms = {k: outs[k][0].clone() for k in range(B)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(B):
        t, p, w = dev[k]
        ptalm.alm_from_points(t, p, w, reqs[k].lmax, out=outs[k][0], options=ptalm.opts(precision=prec))
        ptalm.cl_from_alm(outs[k][0], reqs[k].lmax, out=outs[k][1])
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t0
    same = sum(bool(torch.equal(served_alms[k], outs[k][0])) for k in range(B))
    seq_rate = float(terms[:B].sum()) / seq_s
    print(f"[bench] sequential {B}: {seq_s:.1f} s; served == solo for {same}/{B}", file=sys.stderr, flush=True)

    line = {"metric": METRIC, "value": capacity, "unit": UNIT, "n_gpus": 1, "steps": 1, "warmup": 0,
            "ms_per_step": round(1e3 * res["makespan_s"], 1), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": {"fp64": "f64", "mixed": "f64 recurrence + f32 products",
                                           "fp32": "f32 + f64"}[args.precision], "data": "synthetic",
            "config": {"workload": WORKLOADS["served"]["desc"], "requests": K, "rate_hz": 50.0,
                       "points": int(sum(r.n for r in reqs)), "terms": float(terms.sum()), "slots": args.served_slots,
                       "arena_bytes": arena, "precision": args.precision},
            "served": {"trace_50hz": res, "trace_0.7x_capacity": res_07,
                       "burst": {"requests": B, "served_terms_per_s": burst["terms_per_s"],
                                 "sequential_terms_per_s": seq_rate,
                                 "served_over_sequential": round(burst["terms_per_s"] / seq_rate, 4),
                                 "served_equals_solo": f"{same}/{B} bitwise"}},
            "roofline": {"bound": "alu", "achieved": round(FLOPS_PER_TERM * capacity / 1e12, 3),
                         "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(FLOPS_PER_TERM * capacity / 1e12 / FP64_PEAK_TFLOPS, 4), "traffic": None,
                         "kernel": "alm_direct_kernel (all requests; aggregate over concurrent launches)"}}
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, request 0)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline([("request 0", cats[0])], reqs[0].lmax, args.cpu_seconds)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="randoms3072", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "fp32"])
    ap.add_argument("--points-per-lane", type=int, default=0)
    ap.add_argument("--l-block", type=int, default=0)
    ap.add_argument("--scale", type=float, default=1.0, help="catalog size factor (1 = the named workload)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--time-budget", type=float, default=480.0,
                    help="wall-clock seconds for the whole run from process start; --steps and --warmup are "
                         "upper limits inside it (at least one step is timed)")
    ap.add_argument("--no-mixed-record", dest="mixed_record", action="store_false",
                    help="default workload: skip the extra mixed-precision step run when the budget has room")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--served-requests", type=int, default=500)
    ap.add_argument("--served-slots", type=int, default=4)
    ap.add_argument("--served-arena-gb", type=float, default=16.0)
    ap.add_argument("--spline-error-table", action="store_true",
                    help="print the oracle's pointwise spline interpolation errors (CPU only) and exit")
    ap.add_argument("--multi-slices", type=int, default=0,
                    help="multi2048: point slice count (0: autotune on the first 1e6 positions)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain 1 GiB device copy first (counter runs scale FETCH/WRITE_SIZE by it)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); sharding the catalog over several GPUs is "
              "not built", file=sys.stderr)
        sys.exit(2)
    if args.spline_error_table:
        print(json.dumps(spline_error_table()))
        return
    if args.workload == "served":        # generates its catalogs in worker processes before touching the GPU
        return run_served(args)

    import numpy as np
    import torch
    from paper_2312_12285_amd import ptalm
    if args.copy_calibration and args.workload == "coupling3072":
        copy_calibration()
    if args.workload == "coupling3072":
        return run_coupling(args)

    wl = WORKLOADS[args.workload]
    lmax = wl["lmax"]
    T = tri(lmax)
    print(f"[bench] generating {args.workload} (scale {args.scale})", file=sys.stderr, flush=True)
    t0 = time.time()
    cats = make_catalogs(args.workload, args.scale)
    print(f"[bench] generated in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    if args.copy_calibration:
        copy_calibration()
    if args.workload == "multi2048":
        return run_multi(args, cats, lmax)
    if args.workload in ("spline3072", "spline1000"):
        return run_spline(args, cats, lmax)
    if args.workload == "shear3072":
        return run_shear(args, cats, lmax)
    dev = []
    for name, c in cats:
        dev.append((name, torch.as_tensor(c.theta).cuda(), torch.as_tensor(c.phi).cuda(),
                    torch.as_tensor(c.w).cuda(), c.n))
    prec = {"fp64": ptalm.FP64, "mixed": ptalm.MIXED, "fp32": ptalm.FP32}[args.precision]
    opt = ptalm.opts(precision=prec, points_per_lane=args.points_per_lane, l_block=args.l_block, timing=1)
    outs = [torch.empty(2 * T, dtype=torch.float64, device="cuda") for _ in dev]
    cls = [torch.empty(lmax + 1, dtype=torch.float64, device="cuda") for _ in range(2)]
    kernel_ms = []

    def step():
        ms = 0.0
        for (name, t, p, w, n), out in zip(dev, outs):
            ptalm.alm_from_points(t, p, w, lmax, out=out, options=opt)
            ms += ptalm.last_timing_ms()
        if len(dev) == 2:
            delta, window, alpha = ptalm.fkp_fields(outs[0], outs[1], lmax)
            ptalm.cl_from_alm(delta, lmax, out=cls[0])
            ptalm.cl_from_alm(window, lmax, out=cls[1])
        else:
            ptalm.cl_from_alm(outs[0], lmax, out=cls[0])
        kernel_ms.append(ms)

    # build the per-lmax tables outside the timed region
    ptalm.prepare(lmax)
    torch.cuda.synchronize()
    budget = Budget(args.time_budget)
    line = {}
    checks_done = []

    def checks():
        """Parity and the CPU baseline read a finished step's output (every step computes the
        same result bitwise), so they run after the first warmup, before the timed steps."""
        if not args.no_check:
            print("[bench] sampled parity against oracle entries", file=sys.stderr, flush=True)
            line["parity"] = sampled_parity(cats[-1][1], lmax, outs[-1])
            if prec != ptalm.FP64:
                print("[bench] precision error against the FP64 path and the oracle", file=sys.stderr, flush=True)
                line["precision_error"] = precision_errors(args, cats[-1][1], lmax, outs[-1], prec)
        if not args.no_cpu_baseline:
            print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
            line["cpu_baseline"] = cpu_baseline(cats, lmax, min(args.cpu_seconds, max(2.0, budget.left() / 8)))
        checks_done.append(True)

    # parity (8 oracle entries over every point) and the CPU baseline, if they still run after the
    # timed steps (no warmup requested): ~30 s per 1e8 points + the baseline sample
    reserve = 0.0 if args.warmup > 0 else (3e-7 * sum(n for *_, n in dev) + args.cpu_seconds + 10.0)
    want_mixed = args.precision == "fp64" and args.mixed_record and args.scale == 1.0 and len(dev) == 1
    res = run_steps(step, torch.cuda.synchronize, args.warmup, args.steps, budget,
                    reserve_s=reserve + 10.0, after_first=checks if args.warmup > 0 else None,
                    label="step", optional=(1.0, 15.0) if want_mixed else None)
    if not checks_done:
        kernel_ms_timed = list(kernel_ms)
        checks()
    else:
        kernel_ms_timed = kernel_ms[res["warmup_done"]:]
    elapsed = res["elapsed_s"]
    steps = res["steps"]

    terms_per_step = sum(n for *_, n in dev) * T
    ms_per_step = 1e3 * elapsed / steps
    value = terms_per_step * steps / elapsed
    k_ms = float(np.mean(kernel_ms_timed[:steps])) / len(dev)     # average transform-kernel launch
    launch_terms = terms_per_step / len(dev)
    achieved = FLOPS_PER_TERM * launch_terms / (k_ms * 1e-3) / 1e12
    variant = f"kp={args.points_per_lane or 'default'},lb={args.l_block or 'default'},{args.precision}"
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": recorded_traffic(args.workload if args.scale == 1.0 else None, variant),
                "kernel": "alm_direct_kernel<" + {"fp64": "double, double", "mixed": "double, float",
                                                  "fp32": "float, float"}[args.precision] + ", ...>",
                "kernel_ms_per_launch": round(k_ms, 3), "flops_per_term": FLOPS_PER_TERM,
                "flops_per_term_note": "executed: 3 FMA + 0.5 MUL per term (split recurrence + two accumulates)",
                "valu_issue_frac": round(VALU_INSTS_PER_TERM * launch_terms / (k_ms * 1e-3) / VALU_ISSUE_PER_S, 4)}

    line.update({"metric": METRIC, "value": value, "unit": UNIT,
                 "n_gpus": 1, "steps": steps, "warmup": res["warmup_done"], "steps_requested": args.steps,
                 "warmup_requested": args.warmup, "ms_per_step": round(ms_per_step, 3),
                 "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                 "dtype": {"fp64": "f64", "mixed": "f64 recurrence + f32 products",
                           "fp32": "f32 + f64"}[args.precision], "data": "synthetic",
                 "config": {"workload": wl["desc"], "lmax": lmax, "points": sum(n for *_, n in dev),
                            "terms_per_step": terms_per_step, "precision": args.precision,
                            "points_per_lane": args.points_per_lane or "default",
                            "l_block": args.l_block or "default"},
                 "roofline": roofline,
                 "time_budget_s": args.time_budget})
    if want_mixed and (res["optional"] or budget.left() > 1.05 * res["step_s"] + 15.0):
        print("[bench] mixed-precision step on the same catalog", file=sys.stderr, flush=True)
        line["mixed"] = mixed_record(dev[0], outs[0], lmax, terms_per_step, k_ms)
    elif want_mixed:
        line["mixed"] = {"skipped": f"no room in the {args.time_budget:.0f} s budget for one more step"}
    line["wall_s"] = round(time.monotonic() - START, 1)
    print(json.dumps(line), flush=True)


def mixed_record(d, out64, lmax, terms, fp64_kernel_ms):
    """One MIXED (FP64 recurrence, FP32 products) transform of the same catalog: its rate, kernel
    time and error per l against the FP64 result of the timed steps."""
    import numpy as np
    import torch
    from paper_2312_12285_amd import ptalm
    _, t, p, w, n = d
    out = torch.empty_like(out64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ptalm.alm_from_points(t, p, w, lmax, out=out, options=ptalm.opts(precision=ptalm.MIXED, timing=1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_ms = ptalm.last_timing_ms()
    err = per_l_errors(ptalm.as_complex(out).cpu().numpy(), ptalm.as_complex(out64).cpu().numpy(), lmax)
    return {"value": terms / wall, "unit": UNIT, "steps": 1, "kernel_ms_per_launch": round(k_ms, 3),
            "dtype": "f64 recurrence + f32 products",
            "speedup_over_fp64_kernel": round(fp64_kernel_ms / k_ms, 4), "error_vs_fp64": err}


if __name__ == "__main__":
    main()
