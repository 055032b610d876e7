#!/usr/bin/env python3
"""Throughput of the TREVR2 hot path on one MI355X, in receiver-ray segments/s.

A step is one pass of the whole path over one scene resident in HBM: build
the radiation tree (Morton sort, topology, moments, transmission tables) and
compute J at the active elements.  The segment count (per active element
and ray: 1 + absorbing cells with a chord beyond r_pp + sources on the ray)
is the library's counter, equal to the oracle's by test.

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=float, default=0.05,
                    help="fraction of receivers the oracle evaluates for the CPU baseline")
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
    sc = scenes.config_clumpy()
    n, B, nray = sc.n, sc.n_bands, 12 * sc.nside ** 2
    f32 = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=dev)
    x, y, z, m, rho = f32(sc.x), f32(sc.y), f32(sc.z), f32(sc.m), f32(sc.rho)
    kappa, lum = f32(sc.kappa), f32(sc.lum)
    active = torch.as_tensor(sc.active, device=dev)
    flags = api.THICK_CORR | api.NEAR_FIELD
    kw = dict(nside=sc.nside, leaf_size=sc.leaf_size, theta=sc.theta, flags=flags, box=sc.box)
    J = torch.zeros((B, n), dtype=torch.float64, device=dev)
    if args.calibrate_copy:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        T = api.Tree(x, y, z, m, rho, kappa, lum, **kw)
        T.compute_J(active, None, out=J)
        return T

    # warm-up (also sizes the scratch buffer once)
    for _ in range(args.warmup):
        T = step()
        T.check()
        counters = T.counters()
        T.close()
    if args.warmup == 0:
        T = step()
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

    # forward alone on a resident tree, and per-kernel HIP event timing
    T = api.Tree(x, y, z, m, rho, kappa, lum, **kw)
    T.compute_J(active, None, out=J)
    T.profile(True)
    torch.cuda.synchronize()
    f0 = time.perf_counter()
    for _ in range(args.steps):
        T.compute_J(active, None, out=J)
    torch.cuda.synchronize()
    f1 = time.perf_counter()
    prof = T.profile_read()
    T.check()
    ms_fwd = (f1 - f0) * 1e3 / args.steps
    T.close()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    T = api.Tree(x, y, z, m, rho, kappa, lum, **kw)
    ev1.record()
    torch.cuda.synchronize()
    ms_build = ev0.elapsed_time(ev1)
    T.close()

    # the dominant kernel by time
    kname, (red_ms, red_calls) = max(((k, v) for k, v in prof.items() if k in ("near", "reduce")),
                                     key=lambda kv: kv[1][0])
    flops = far_flops(counters, B) if kname == "reduce" else near_flops(counters, nray)
    per_launch = flops / max(red_calls / args.steps, 1)
    achieved = per_launch / (red_ms / max(red_calls, 1) * 1e-3) / 1e12
    roofline = {"kernel": {"near": "k_pp_rays+k_pp_src", "reduce": "k_far"}[kname], "bound": "alu",
                "achieved": achieved,
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                "traffic": measured_traffic("k_far") if kname == "reduce" else None,
                "launches_per_step": red_calls / args.steps,
                "avg_launch_ms": red_ms / max(red_calls, 1),
                "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()}}

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
        "fwd_only": {"value": seg / (ms_fwd * 1e-3), "ms": ms_fwd},
        "build_ms": ms_build,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "counters": counters,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
