#!/usr/bin/env python3
"""Throughput of the TREVR2 hot path on one MI355X, in receiver-ray segments/s.

A step is one pass of the whole path over one scene resident in HBM: build
the radiation tree (Morton sort, topology, moments, transmission tables),
compute J at the active elements, and run the adjoint for a fixed seeded
dE/dJ (gradients with respect to L, kappa and rho).  The segment count (per
active element and ray: 1 + absorbing cells with a chord beyond r_pp +
sources on the ray) is the library's counter, equal to the oracle's by
test; `value` is segments per step over the step time (build + forward +
adjoint), and the forward alone and forward + adjoint on a resident tree
are reported beside it.

Workload: the clumpy medium -- 2^18 elements drawn from a log-normal density
field (P(k) ~ k^-3, sigma_ln rho = 1.5), 10% sources with log-normal
luminosities, 3 bands (opacity 1:10:100), N_side 2 (48 rays), theta 0.75,
leaf 8, all elements active.

Prints one JSON line (see the keys below).  `--gpus N` with N > 1 is not
supported: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "receiver-ray segments/sec (fwd, fwd+adjoint) at J rel. err ≤1e-4 vs FP64"
PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32
PEAK_HBM_GBS = 8000.0


def flop_model(c: dict, B: int, nray: int) -> float:
    """Algorithmic floating-point operations of one compute_J (each add,
    multiply, divide, square root and exponential counts one):
      far source at a receiver      37 + 6B per (receiver, source entry)
      cell-ray intersection         20 + 2B per (bucket, absorber entry)
      p-p column along a ray        24      per (receiver, ray, p-p element)
      p-p source path               35      per (receiver, p-p source, p-p element)"""
    return (c["src_pairs"] * (37 + 6 * B) + c["absorber_entries"] * (20 + 2 * B)
            + nray * c["near_pairs"] * 24 + c["near_src_triples"] * 35)


def near_flops(c: dict, nray: int) -> float:
    """The p-p part of flop_model (the work of the near-field kernel)."""
    return nray * c["near_pairs"] * 24 + c["near_src_triples"] * 35


def far_flops(c: dict, B: int) -> float:
    return c["src_pairs"] * (37 + 6 * B) + c["absorber_entries"] * (20 + 2 * B)


def far_adjoint_flops(c: dict, B: int) -> float:
    """Arithmetic of the far-field adjoint kernel: per (receiver, source
    entry) the forward term (37 + 6B) plus its derivatives (intensity-kernel
    slope 14, dK/dr and dK/dh 6, position 4, 13 per band); per (bucket,
    absorber entry) two sweeps of the hit arithmetic (2 x (20 + 2B)) and the
    cell-absorption adjoint (4B)."""
    return c["src_pairs"] * (61 + 19 * B) + c["absorber_entries"] * (40 + 8 * B)


def measured_traffic(kernel: str):
    """HBM-side bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE/WRITE_SIZE runs (profiles/), or None when the kernel source
    changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_clumpy2e18_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def batched_bench(args, dev):
    """The batched workload: 64 independent scenes (log-uniform 2^12..2^17
    elements, uniform or log-normal media, 1-4 bands, N_side 1/2/4), all
    active, computed by the batched calls replayed from HIP graphs (forward;
    forward + adjoint); against it the plain path, every scene's own tree
    called in turn.  Also the same graph replayed with per-scene active
    fractions of 1%, 10% or 100% written into its active buffer."""
    import numpy as np
    import torch
    from paper_2310_15235_amd import api, scenes

    def note(msg):
        print(f"[batched] {msg}", file=sys.stderr, flush=True)

    scs = scenes.batched_scenes(64)
    torch.cuda.synchronize()
    b0 = time.perf_counter()
    F = api.Forest(scs, device=dev)
    torch.cuda.synchronize()
    b1 = time.perf_counter()
    note(f"forest of {F.S} scenes built and planned in {b1 - b0:.2f} s")
    a = F.flat_active([None] * F.S)
    gJ = torch.as_tensor(np.random.default_rng(11).normal(size=int(F.boff[-1])), device=dev)
    J = F.new_J()
    outs = (torch.empty_like(gJ), torch.empty_like(gJ),
            torch.empty(int(F.offsets[-1]), dtype=torch.float64, device=dev))
    chosen, tune_ms = F.autotune(a, reps=1)   # forward only: the adjoint's p-p work follows it
    note(f"autotuned: configuration {chosen}, forward ms {[round(float(t), 1) for t in tune_ms]}")
    F.compute_J(a, out=J)
    F.compute_J_backward(gJ, a, out=outs)
    F.check()
    seg = F.counters(-1)["segments"]
    note("eager forward + adjoint done")
    torch.cuda.synchronize()
    g_f, g_fa = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_f):
        F.compute_J(a, out=J)
    with torch.cuda.graph(g_fa):
        F.compute_J(a, out=J)
        F.compute_J_backward(gJ, a, out=outs)

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / k

    k = max(1, min(args.steps, 2))   # each replay takes seconds at this size
    ms_f = timed(g_f.replay, k)
    note(f"graph forward {ms_f:.1f} ms")
    ms_fa = timed(g_fa.replay, k)
    note(f"graph forward + adjoint {ms_fa:.1f} ms")
    # mixed individual time steps: per-scene active fractions in one buffer
    rng = np.random.default_rng(7)
    fr = rng.choice([0.01, 0.1, 1.0], size=F.S)
    acts = [scenes.active_subset(s, f, 300 + i) if f < 1.0 else None
            for i, (s, f) in enumerate(zip(scs, fr))]
    a.copy_(F.flat_active(acts))
    F.compute_J(a, out=J)
    F.check()
    seg_mixed = F.counters(-1)["segments"]
    ms_fa_mixed = timed(g_fa.replay, k)
    note(f"graph forward + adjoint, mixed active sets {ms_fa_mixed:.1f} ms")
    a.copy_(F.flat_active([None] * F.S))
    # the plain path: each scene's own tree, one after another
    trees = [F.scene_tree(s) for s in range(F.S)]
    Jp, gLp, gkp, grp = F.split(J), F.split(outs[0]), F.split(outs[1]), F.split(outs[2])
    gJp = F.split(gJ)
    ap_ = F.split(a)
    bgs = [None if not s.background else torch.as_tensor(s.bg, device=dev) for s in scs]

    def plain_f():
        for s, T in enumerate(trees):
            T.compute_J(ap_[s], bgs[s], out=Jp[s])

    def plain_fa():
        for s, T in enumerate(trees):
            T.compute_J(ap_[s], bgs[s], out=Jp[s])
            T.compute_J_backward(gJp[s], ap_[s], bgs[s], out=(gLp[s], gkp[s], grp[s]))

    plain_fa()
    ms_pf = timed(plain_f, k)
    note(f"plain forward {ms_pf:.1f} ms")
    ms_pfa = timed(plain_fa, k)
    note(f"plain forward + adjoint {ms_pfa:.1f} ms")
    for T in trees:
        T.check()
    F.close()
    n_tot = int(F.offsets[-1])
    return {
        "workload": "64 scenes, 2^12..2^17 elements each (log-uniform), uniform or log-normal "
                    "media, 1-4 bands, N_side 1/2/4, theta 0.75, leaf 8, all active",
        "scenes": F.S, "elements": n_tot, "segments_per_step": seg,
        "timed_replays": k,
        "graph": True,
        "fwd": {"value": seg / (ms_f * 1e-3), "ms": ms_f},
        "fwd_adjoint": {"value": seg / (ms_fa * 1e-3), "ms": ms_fa},
        "plain_fwd": {"value": seg / (ms_pf * 1e-3), "ms": ms_pf},
        "plain_fwd_adjoint": {"value": seg / (ms_pfa * 1e-3), "ms": ms_pfa},
        "mixed_active": {"segments_per_step": seg_mixed,
                         "fwd_adjoint": {"value": seg_mixed / (ms_fa_mixed * 1e-3),
                                         "ms": ms_fa_mixed},
                         "fractions": "1% / 10% / 100% per scene"},
        "build_and_plan_ms": (b1 - b0) * 1e3,
        "autotune": {"chosen": chosen, "candidate_fwd_ms": [float(t) for t in tune_ms],
                     "candidates": "bit 2: bucket order (cost / scene), bit 1: persistent "
                                   "grid (full / half), bit 0: p-p boxes (16 / 8)"},
    }


def measured_counters(kernel: str):
    """VALU issue utilisation, L2 hit rate and LDS figures of `kernel` from
    the committed rocprofv3 counter runs (profiles/), or None when the kernel
    source changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_clumpy2e18_counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return {k: rec[k] for k in ("valu_issue_util", "l2_hit_rate", "lds_instr_per_valu",
                                "lds_bank_conflicts_per_lds_instr")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=float, default=0.05,
                    help="fraction of receivers the oracle evaluates for the CPU baseline")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched 64-scene measurement")
    ap.add_argument("--no-keep-depths", action="store_true",
                    help="skip the forward + adjoint timing with the depth cache")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched 64-scene measurement and print its record")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy first (a kernel of known "
                         "traffic, for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU (this build has no multi-GPU path)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2310_15235_amd import api, scenes

    dev = torch.device("cuda:0")
    if args.only_batched:
        print(json.dumps({"batched": batched_bench(args, dev)}), flush=True)
        return
    sc = scenes.config_clumpy()
    n, B, nray = sc.n, sc.n_bands, 12 * sc.nside ** 2
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev)
    x, y, z, m, rho = f32(sc.x), f32(sc.y), f32(sc.z), f32(sc.m), f32(sc.rho)
    kappa, lum = f32(sc.kappa), f32(sc.lum)
    active = torch.as_tensor(sc.active, device=dev)
    flags = api.THICK_CORR | api.NEAR_FIELD
    kw = dict(nside=sc.nside, leaf_size=sc.leaf_size, theta=sc.theta, flags=flags, box=sc.box)
    J = torch.zeros((B, n), dtype=torch.float64, device=dev)
    gJ = torch.as_tensor(np.random.default_rng(7).normal(size=(B, n)), device=dev)
    grads = (torch.empty((B, n), dtype=torch.float64, device=dev),
             torch.empty((B, n), dtype=torch.float64, device=dev),
             torch.empty((n,), dtype=torch.float64, device=dev))
    if args.calibrate_copy:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    scratch = [None]   # one scratch buffer kept across steps, as a time-stepping caller would

    def step():
        T = api.Tree(x, y, z, m, rho, kappa, lum, scratch=scratch[0], **kw)
        T.compute_J(active, None, out=J)
        T.compute_J_backward(gJ, active, None, out=grads)
        scratch[0] = T.scratch
        return T

    # warm-up (also sizes the scratch buffer once)
    for _ in range(max(args.warmup, 1)):
        T = step()
        T.check()
        counters = T.counters()
        T.close()
    seg = counters["segments"]

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        T = step()
        T.close()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps

    # forward alone and forward + adjoint on a resident tree, with per-phase
    # HIP event timing recorded by the library on its stream
    T = api.Tree(x, y, z, m, rho, kappa, lum, scratch=scratch[0], **kw)
    T.compute_J(active, None, out=J)
    T.compute_J_backward(gJ, active, None, out=grads)
    T.profile(True)
    torch.cuda.synchronize()
    f0 = time.perf_counter()
    for _ in range(args.steps):
        T.compute_J(active, None, out=J)
    torch.cuda.synchronize()
    f1 = time.perf_counter()
    prof_fwd = T.profile_read()
    T.profile(True)
    torch.cuda.synchronize()
    a0 = time.perf_counter()
    for _ in range(args.steps):
        T.compute_J(active, None, out=J)
        T.compute_J_backward(gJ, active, None, out=grads)
    torch.cuda.synchronize()
    a1 = time.perf_counter()
    prof = T.profile_read()
    T.check()
    ms_fwd = (f1 - f0) * 1e3 / args.steps
    ms_fwd_adj = (a1 - a0) * 1e3 / args.steps
    T.close()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    T = api.Tree(x, y, z, m, rho, kappa, lum, scratch=scratch[0], **kw)
    ev1.record()
    torch.cuda.synchronize()
    ms_build = ev0.elapsed_time(ev1)
    T.close()

    # forward + adjoint again with the depth cache (KEEP_DEPTHS): the forward
    # keeps the far sources' cell optical depths and the adjoint reads them
    # instead of recomputing every ray's prefixes (the default above)
    ms_fwd_adj_keep = None
    if not args.no_keep_depths:
        kw_keep = dict(kw, flags=flags | api.KEEP_DEPTHS)
        T = api.Tree(x, y, z, m, rho, kappa, lum, **kw_keep)
        T.compute_J(active, None, out=J)
        T.compute_J_backward(gJ, active, None, out=grads)
        torch.cuda.synchronize()
        k0 = time.perf_counter()
        for _ in range(args.steps):
            T.compute_J(active, None, out=J)
            T.compute_J_backward(gJ, active, None, out=grads)
        torch.cuda.synchronize()
        k1 = time.perf_counter()
        T.check()
        T.close()
        ms_fwd_adj_keep = (k1 - k0) * 1e3 / args.steps

    # the dominant single kernel of a step: the far-field reduction or its
    # adjoint (the p-p phases are two kernels each and shorter)
    kname = max(("reduce", "adj_reduce"), key=lambda k: prof[k][0])
    red_ms, red_calls = prof[kname]
    flops = far_flops(counters, B) if kname == "reduce" else far_adjoint_flops(counters, B)
    per_launch = flops / max(red_calls / args.steps, 1)
    achieved = per_launch / (red_ms / max(red_calls, 1) * 1e-3) / 1e12
    kernel = {"reduce": "k_far", "adj_reduce": "k_far_bwd"}[kname]
    roofline = {"kernel": kernel, "bound": "alu",
                "achieved": achieved,
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                "traffic": measured_traffic(kernel),
                "counters": measured_counters(kernel),
                "launches_per_step": red_calls / args.steps,
                "avg_launch_ms": red_ms / max(red_calls, 1),
                "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
                "fwd_kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof_fwd.items()
                                           if v[1]}}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        nthreads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
        act = scenes.active_subset(sc, args.cpu_sample, 123)
        c0 = time.perf_counter()
        O = oracle.OracleTree(sc)
        c1 = time.perf_counter()
        _, oc = O.compute_J(act, nthreads=nthreads)
        c2 = time.perf_counter()
        tb, tj = c1 - c0, c2 - c1
        frac = act.sum() / n
        cpu = {"value": oc["segments"] / (tj + frac * tb), "unit": "segments/s",
               "cores": nthreads, "kind": "oracle",
               "sample": f"{int(act.sum())} of {n} receivers ({args.cpu_sample:.0%}) of the same "
                         f"scene; full tree build {tb:.2f} s prorated by that fraction, "
                         f"J {tj:.2f} s"}

    batched = None if args.no_batched else batched_bench(args, dev)

    out = {
        "metric": METRIC,
        "value": seg / (ms_step * 1e-3),
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "clumpy log-normal medium: 2^18 elements, 10% sources, 3 bands "
                               "(kappa 1:10:100), N_side 2 (48 rays), theta 0.75, leaf 8, "
                               "all active",
                   "n": n, "bands": B, "nside": sc.nside, "active": int(sc.active.sum()),
                   "segments_per_step": seg},
        "fwd": {"value": seg / (ms_fwd * 1e-3), "ms": ms_fwd},
        "fwd_adjoint": {"value": seg / (ms_fwd_adj * 1e-3), "ms": ms_fwd_adj},
        "fwd_adjoint_keep_depths": None if ms_fwd_adj_keep is None else
            {"value": seg / (ms_fwd_adj_keep * 1e-3), "ms": ms_fwd_adj_keep},
        "build_ms": ms_build,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "counters": counters,
        "batched": batched,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
