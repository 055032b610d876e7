#!/usr/bin/env python3
"""Throughput of the TREVR2 hot path on one MI355X, in receiver-ray segments/s.

Headline (`value`): batched forward + adjoint.  A step is one replay of a HIP
graph holding the batched forward (J of every active element of 64
independent scenes) and its adjoint (gradients of a fixed seeded
<dE/dJ, J> with respect to L, kappa and rho), with the scenes' trees and
inputs resident in HBM.  Segments (per active element and ray: 1 + absorbing
cells with a chord beyond r_pp + sources on the ray) are the library's
counter, equal to the oracle's by test; `value` = segments per step / step
time.

Workload: 64 scenes of log-uniform size 2^12..2^17 elements (2.2M in all),
each a uniform or a log-normal medium (C1 / C2 generators), 1-4 bands, N_side
1, 2 or 4, theta 0.75, leaf 8, all elements active.  The forest keeps the p-p
job log (the forward's culled p-p source jobs, read by the adjoint), sized
from the forward's own count of its entries.

Beside it (extra keys): the batched forward alone, the same graph with mixed
per-scene active fractions, the plain path (each scene's own tree called in
turn), the single-scene clumpy 2^18 workload, the diffuse 2^21 workload at 1%,
10% and 100% active, the cost of 10 bands against 1, the roofline of the
dominant kernel, the traversal-byte HBM fraction, and the oracle's CPU rate.

Prints one JSON line.  `--gpus N` with N > 1 is not supported: this build
runs on one GPU.
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
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E


def note(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ----------------------------------------------------------- work models
# Algorithmic floating-point operations (each add, multiply, divide, square
# root and exponential counts one), per unit of work the oracle counts:
#   far source at a receiver        37 + 6B   per (receiver, source entry)
#   cell-ray intersection           20 + 2B   per (bucket, absorber entry)
#   p-p column along a ray          24        per (receiver, ray, p-p element)
#   p-p source path                 29 + 2B   per hit: a (receiver, source,
#                                   element) triple whose element absorbs on
#                                   the path (its exact test 25, the column 4,
#                                   a multiply-add per band); the kernel finds
#                                   the hits by conservative culling, so
#                                   triples that cannot be hits are not work
# and for the adjoint kernels the forward arithmetic again plus the
# derivatives:
#   far source                      61 + 19B  (kernel slope 14, dK/dr, dK/dh 6,
#                                              position 4, 13 per band)
#   cell-ray intersection           40 + 8B   (two sweeps + absorption adjoint)
#   p-p column                      24 + 8    (column slope in h, kappa term)
#   p-p source path                 35 + 5B   per hit (column slope in h,
#                                              kappa and h adjoints per band)
def kernel_flops(c: dict, B: int, nray: int) -> dict:
    return {
        "k_pp_src": c["near_src_hits"] * (29.0 + 2 * B),
        "k_pp_rays": nray * c["near_pairs"] * 24.0,
        "k_far": c["src_pairs"] * (37 + 6 * B) + c["absorber_entries"] * (20 + 2 * B),
        "k_pp_src_bwd": c["near_src_hits"] * (35.0 + 5 * B),
        "k_pp_rays_bwd": nray * c["near_pairs"] * 32.0,
        "k_far_bwd": c["src_pairs"] * (61 + 19 * B) + c["absorber_entries"] * (40 + 8 * B),
    }


# Traversal bytes (HBM roofline model): per bucket, each accepted cell is read
# once (box 24 B, luminosity centre 12 B, luminosity 4B B), each (cell, ray)
# intersection reads its transmission average (4B B), each active receiver
# is read and its J written (20 + 8B B).
def traversal_bytes(c: dict, B: int) -> float:
    return (c["cells"] * (36 + 4 * B) + c["absorber_entries"] * 4 * B
            + c["active"] * (20 + 8 * B))


# Which profile slots time which kernel (the p-p columns are the near-field
# phase minus the p-p source kernel).
def kernel_ms(prof: dict) -> dict:
    g = lambda k: prof[k][0]
    n = lambda k: prof[k][1]
    return {
        "k_pp_src": (g("pp_src"), n("pp_src")),
        "k_pp_rays": (g("near") - g("pp_src"), n("pp_src")),
        "k_far": (g("reduce"), n("reduce")),
        "k_pp_src_bwd": (g("adj_pp_src"), n("adj_pp_src")),
        "k_pp_rays_bwd": (g("adj_near") - g("adj_pp_src"), n("adj_pp_src")),
        "k_far_bwd": (g("adj_reduce"), n("adj_reduce")),
    }


def committed_profile(kernel: str, workload: str, kind: str):
    """Figures of `kernel` from the committed rocprofv3 runs (profiles/),
    or None when the kernel's sources changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{kind}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in rec["sources"]:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ------------------------------------------------------------- batched C4
def batched(args, dev, extras: bool):
    import numpy as np
    import torch
    from paper_2310_15235_amd import api, scenes

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
    chosen, tune_ms = F.autotune(a, reps=1)   # forward: the adjoint's p-p work follows it
    note(f"autotuned: configuration {chosen}, forward ms {[round(float(t), 1) for t in tune_ms]}")
    F.compute_J(a, out=J)
    F.check()
    per_scene = [F.counters(s) for s in range(F.S)]
    seg = sum(c["segments"] for c in per_scene)
    # the p-p job log: room for every bucket's jobs (the forward's count) plus
    # partly used blocks (32 KiB per persistent wavefront and band count)
    log_entries = sum(c["pp_log_entries"] for c in per_scene)
    F.set_job_log(2 * log_entries + (1 << 30))
    note(f"p-p job log: {log_entries} entries, {F.job_log_bytes / 2 ** 30:.2f} GiB")
    F.compute_J(a, out=J)
    F.compute_J_backward(gJ, a, out=outs)
    F.check()

    # kernel times of one forward + adjoint (HIP events on the stream the
    # library launches on), and the algorithmic work of each kernel
    F.profile(True)
    F.compute_J(a, out=J)
    F.compute_J_backward(gJ, a, out=outs)
    prof = F.profile_read()
    F.profile(False)
    F.check()
    kms = kernel_ms(prof)
    flops = {}
    tbytes = 0.0
    for s, c in enumerate(per_scene):
        c = dict(c, active=scs[s].n)
        for k, v in kernel_flops(c, scs[s].n_bands, 12 * scs[s].nside ** 2).items():
            flops[k] = flops.get(k, 0.0) + v
        tbytes += traversal_bytes(c, scs[s].n_bands)
    dom = max(kms, key=lambda k: kms[k][0])
    d_ms, d_launch = kms[dom]
    achieved = flops[dom] / (d_ms * 1e-3) / 1e12
    note(f"dominant kernel {dom}: {d_ms:.1f} ms in {d_launch} launches, {achieved:.2f} TFLOP/s")

    torch.cuda.synchronize()
    g_f, g_fa = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(g_f):
        F.compute_J(a, out=J)
    with torch.cuda.graph(g_fa):
        F.compute_J(a, out=J)
        F.compute_J_backward(gJ, a, out=outs)

    # headline: W warm-up replays, then K replays timed together
    for _ in range(args.warmup):
        g_fa.replay()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record()
        g_fa.replay()
        e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    per_replay = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
    note(f"graph forward + adjoint: {ms_step:.1f} ms per step (median replay "
         f"{per_replay[len(per_replay) // 2]:.1f} ms)")
    Jg = J.cpu().numpy()

    def timed(fn, k):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(k):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    ms_f = timed(g_f.replay, 3)
    note(f"graph forward {ms_f:.1f} ms")
    rec = {
        "seg": seg, "ms_step": ms_step, "per_replay_ms": {"median": per_replay[len(per_replay) // 2],
                                                          "min": per_replay[0]},
        "fwd_ms": ms_f, "prof": prof, "kernel_ms": kms, "flops": flops,
        "dominant": dom, "achieved": achieved, "launches": d_launch, "dom_ms": d_ms,
        "traversal_bytes": tbytes, "build_and_plan_ms": (b1 - b0) * 1e3,
        "job_log": {"entries": log_entries, "bytes": F.job_log_bytes,
                    "scratch_bytes": int(F.scratch.numel())},
        "autotune": {"chosen": chosen, "candidate_fwd_ms": [float(t) for t in tune_ms],
                     "candidates": "bit 2: bucket order (cost / scene), bit 1: persistent "
                                   "grid (full / half), bit 0: p-p boxes (16 / 8)"},
        "J": Jg, "scenes": scs, "forest": F, "n_total": int(F.offsets[-1]),
    }
    if extras:
        # mixed individual time steps: per-scene active fractions in one buffer
        rng = np.random.default_rng(7)
        fr = rng.choice([0.01, 0.1, 1.0], size=F.S)
        acts = [scenes.active_subset(s, f, 300 + i) if f < 1.0 else None
                for i, (s, f) in enumerate(zip(scs, fr))]
        a.copy_(F.flat_active(acts))
        F.compute_J(a, out=J)
        F.check()
        seg_mixed = F.counters(-1)["segments"]
        ms_mixed = timed(g_fa.replay, 1)
        note(f"graph forward + adjoint, mixed active sets {ms_mixed:.1f} ms")
        a.copy_(F.flat_active([None] * F.S))
        # the plain path: each scene's own tree, one after another
        trees = [F.scene_tree(s) for s in range(F.S)]
        Jp, gLp, gkp, grp = F.split(J), F.split(outs[0]), F.split(outs[1]), F.split(outs[2])
        gJp, ap_ = F.split(gJ), F.split(a)
        bgs = [None if not s.background else torch.as_tensor(s.bg, device=dev) for s in scs]

        def plain_f():
            for s, T in enumerate(trees):
                T.compute_J(ap_[s], bgs[s], out=Jp[s])

        def plain_fa():
            for s, T in enumerate(trees):
                T.compute_J(ap_[s], bgs[s], out=Jp[s])
                T.compute_J_backward(gJp[s], ap_[s], bgs[s], out=(gLp[s], gkp[s], grp[s]))

        ms_pf = timed(plain_f, 1)
        ms_pfa = timed(plain_fa, 1)
        note(f"plain forward {ms_pf:.1f} ms, forward + adjoint {ms_pfa:.1f} ms")
        for T in trees:
            T.check()
        rec.update(seg_mixed=seg_mixed, ms_mixed=ms_mixed, ms_plain_f=ms_pf, ms_plain_fa=ms_pfa)
    return rec


def c4_cpu_baseline(rec, per_scene_recv=24, one_core_scenes=16):
    """The oracle (OpenMP over buckets) on a bounded sample: `per_scene_recv`
    random receivers of every scene, each scene's tree built in full and its
    build time prorated by the sampled fraction; the same with one thread on
    the first scenes.  Returns the record and the sampled J for the
    self-check."""
    import numpy as np
    import oracle
    from paper_2310_15235_amd import scenes as S
    scs = rec["scenes"]
    nthreads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))

    def run(idx, nt, k):
        seg, t_j, t_b = 0, 0.0, 0.0
        samples = []
        for s in idx:
            sc = scs[s]
            rng = np.random.default_rng(500 + s)
            act = np.zeros(sc.n, np.uint8)
            act[rng.choice(sc.n, size=min(k, sc.n), replace=False)] = 1
            c0 = time.perf_counter()
            O = oracle.OracleTree(sc)
            c1 = time.perf_counter()
            Jo, oc = O.compute_J(act, nthreads=nt)
            c2 = time.perf_counter()
            seg += oc["segments"]
            t_j += c2 - c1
            t_b += (c1 - c0) * act.sum() / sc.n
            samples.append((s, act, Jo))
        return seg, t_j, t_b, samples

    seg, t_j, t_b, samples = run(range(len(scs)), nthreads, per_scene_recv)
    seg1, t_j1, t_b1, _ = run(range(one_core_scenes), 1, per_scene_recv // 3)
    return {"value": seg / (t_j + t_b), "unit": "segments/s", "cores": nthreads,
            "kind": "oracle",
            "sample": f"{per_scene_recv} random receivers of each of the {len(scs)} scenes "
                      f"(forward; the oracle has no adjoint), every tree built in full with its "
                      f"build time prorated by the sampled fraction: {seg} segments, J "
                      f"{t_j:.2f} s + build {t_b:.3f} s",
            "single_core": {"value": seg1 / (t_j1 + t_b1), "cores": 1,
                            "sample": f"{per_scene_recv // 3} receivers of each of the first "
                                      f"{one_core_scenes} scenes"},
            "cpu_model": cpu_model()}, samples


def self_check(rec, samples):
    """The headline's own J against the oracle's at the sampled receivers."""
    import numpy as np
    F = rec["forest"]
    Jg = rec["J"]
    worst, count = 0.0, 0
    for s, act, Jo in samples:
        g = Jg[int(F.boff[s]):int(F.boff[s + 1])].reshape(F.B[s], F.n[s])
        a = act.astype(bool)
        floor = 1e-12 * np.abs(Jo[:, a]).max(axis=1, keepdims=True)
        e = np.abs(g[:, a] - Jo[:, a]) / np.maximum(np.abs(Jo[:, a]), np.maximum(floor, 1e-300))
        worst = max(worst, float(e.max()))
        count += int(a.sum())
    return {"receivers": count, "max_rel_err": worst, "tol": 1e-4, "pass": worst <= 1e-4}


# ------------------------------------------------------- one-scene legs
def single_tree(sc, dev, reps=3, active=None, label="", extra_flags=0):
    """Forward and forward + adjoint on a resident tree (median of `reps`),
    tree build time, per-phase kernel times, counters; extra_flags (the
    adjoint's depth cache) are or-ed into the scene's options."""
    import numpy as np
    import torch
    from paper_2310_15235_amd import api
    n, B = sc.n, sc.n_bands
    act = torch.as_tensor(sc.active if active is None else active, device=dev)
    bg = None if not sc.background else torch.as_tensor(sc.bg, device=dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    T = api.Tree.from_scene(sc, device=dev, extra_flags=extra_flags)
    ev1.record()
    torch.cuda.synchronize()
    ms_build = ev0.elapsed_time(ev1)
    J = torch.zeros((B, n), dtype=torch.float64, device=dev)
    gJ = torch.as_tensor(np.random.default_rng(7).normal(size=(B, n)), device=dev)
    grads = (torch.empty((B, n), dtype=torch.float64, device=dev),
             torch.empty((B, n), dtype=torch.float64, device=dev),
             torch.empty((n,), dtype=torch.float64, device=dev))
    T.compute_J(act, bg, out=J)
    T.compute_J_backward(gJ, act, bg, out=grads)
    T.check()
    c = T.counters()

    def med(fn):
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    ms_f = med(lambda: T.compute_J(act, bg, out=J))
    T.profile(True)
    ms_fa = med(lambda: (T.compute_J(act, bg, out=J), T.compute_J_backward(gJ, act, bg,
                                                                             out=grads)))
    prof = T.profile_read()
    T.profile(False)
    T.check()
    T.close()
    seg = c["segments"]
    note(f"{label}: build {ms_build:.1f} ms, forward {ms_f:.2f} ms, forward + adjoint "
         f"{ms_fa:.2f} ms, {seg} segments")
    return {"segments": seg, "build_ms": ms_build,
            "fwd": {"value": seg / (ms_f * 1e-3), "ms": ms_f},
            "fwd_adjoint": {"value": seg / (ms_fa * 1e-3), "ms": ms_fa},
            "kernel_ms_per_step": {k: v[0] / reps for k, v in prof.items() if v[1]},
            "counters": c}


def bands_cost(dev):
    """Section 3.1: ten bands cost about 1.3x one band.  The clumpy 2^18
    geometry with 1 band and with 10 (opacities 1..100), forward time on a
    resident tree."""
    import numpy as np
    from paper_2310_15235_amd import scenes
    out = {}
    for nb in (1, 10):
        bands = tuple(float(10 ** (2 * k / 9)) for k in range(nb)) if nb > 1 else (1.0,)
        sc = scenes.lognormal_scene(n=2 ** 18, seed=2, grid=64, bands=bands, nside=2,
                                    name=f"clumpy_b{nb}")
        r = single_tree(sc, dev, reps=3, label=f"clumpy 2^18, {nb} band(s)")
        out[f"B{nb}"] = {"fwd_ms": r["fwd"]["ms"], "fwd_adjoint_ms": r["fwd_adjoint"]["ms"]}
    out["fwd_ratio"] = out["B10"]["fwd_ms"] / out["B1"]["fwd_ms"]
    out["fwd_adjoint_ratio"] = out["B10"]["fwd_adjoint_ms"] / out["B1"]["fwd_adjoint_ms"]
    out["paper"] = "10 bands cost about 1.3x one band (Section 3.1, serial CPU run)"
    return out


def complex_source_cost(dev, reps=3):
    """Section 2.7 (the complex source model): its tree build costs about 40%
    more wall clock in the paper's test problems.  The clumpy 2^18 scene
    built and run forward with and without the model (medians of `reps`;
    the build includes the inputs' upload, the same for both)."""
    import numpy as np
    import torch
    from paper_2310_15235_amd import api, scenes
    sc = scenes.config_clumpy()
    act = torch.as_tensor(sc.active, device=dev)
    out = {}
    for name, flag in (("standard", 0), ("complex", api.COMPLEX_SOURCE)):
        tb, tf = [], []
        for _ in range(reps):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            torch.cuda.synchronize()
            e0.record()
            T = api.Tree.from_scene(sc, device=dev, extra_flags=flag)
            e1.record()
            J = T.compute_J(act)
            e2.record()
            torch.cuda.synchronize()
            T.check()
            T.close()
            tb.append(e0.elapsed_time(e1))
            tf.append(e1.elapsed_time(e2))
        out[name] = {"build_ms": float(np.median(tb)), "fwd_ms": float(np.median(tf))}
    out["build_ratio"] = out["complex"]["build_ms"] / out["standard"]["build_ms"]
    out["paper"] = "the complex source model's tree build: about +40% wall clock (Section 2.7)"
    note(f"complex source model: build {out['standard']['build_ms']:.2f} -> "
         f"{out['complex']['build_ms']:.2f} ms, forward {out['standard']['fwd_ms']:.2f} -> "
         f"{out['complex']['fwd_ms']:.2f} ms")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the batched headline (for profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 256 MiB device-to-device copy first (a kernel of known "
                         "traffic, for scaling HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU (this build has no multi-GPU path)",
              file=sys.stderr)
        sys.exit(2)
    args.steps = max(1, args.steps)

    import torch
    from paper_2310_15235_amd import scenes

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    extras = not args.headline_only
    rec = batched(args, dev, extras)
    seg = rec["seg"]
    dom = rec["dominant"]
    traffic = committed_profile(dom, "batched64", "traffic")
    counters = committed_profile(dom, "batched64", "counters")
    roofline = {"kernel": dom, "bound": "alu", "achieved": rec["achieved"],
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": rec["achieved"] / PEAK_FP32_TFLOPS,
                "traffic": None if traffic is None else traffic["bytes_per_launch"],
                "counters": None if counters is None else
                {k: counters[k] for k in counters if k not in ("sources", "sources_sha256")},
                "launches_per_step": rec["launches"],
                "avg_launch_ms": rec["dom_ms"] / max(rec["launches"], 1),
                "algorithmic_flops_per_launch": rec["flops"][dom] / max(rec["launches"], 1),
                "kernel_ms_per_step": {k: v[0] for k, v in rec["kernel_ms"].items()},
                "timing": "HIP events on the library's stream around each launch, one eager "
                          "forward + adjoint of the same forest"}
    fa_s = rec["ms_step"] * 1e-3
    hbm = {"traversal_bytes_per_step": 2 * rec["traversal_bytes"],
           "achieved_GBs": 2 * rec["traversal_bytes"] / fa_s / 1e9,
           "peak_GBs": PEAK_HBM_GBS,
           "frac": 2 * rec["traversal_bytes"] / fa_s / 1e9 / PEAK_HBM_GBS,
           "model": "per bucket: accepted cells x (36 + 4B) B + (cell, ray) intersections x 4B B "
                    "+ active receivers x (20 + 8B) B, read once by the forward and once by "
                    "the adjoint"}
    cpu = None
    check = None
    if not args.no_cpu_baseline:
        note("CPU baseline (oracle) on sampled receivers of the 64 scenes")
        cpu, samples = c4_cpu_baseline(rec)
        check = self_check(rec, samples)
        note(f"self-check against the oracle: {check}")
        if not check["pass"]:
            print("warning: batched J differs from the oracle beyond 1e-4", file=sys.stderr)
    out = {
        "metric": METRIC,
        "value": seg / fa_s,
        "unit": "segments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "batched forward + adjoint, HIP-graph replay: 64 scenes of "
                               "2^12..2^17 elements (log-uniform, 2.2M in all), uniform or "
                               "log-normal media, 1-4 bands, N_side 1/2/4, theta 0.75, leaf 8, "
                               "all active; p-p job log on",
                   "scenes": len(rec["scenes"]), "elements": rec["n_total"],
                   "segments_per_step": seg, "pp_job_log_bytes": rec["job_log"]["bytes"]},
        "fwd_adjoint": {"value": seg / fa_s, "ms": rec["ms_step"],
                        "replay_ms": rec["per_replay_ms"]},
        "fwd": {"value": seg / (rec["fwd_ms"] * 1e-3), "ms": rec["fwd_ms"]},
        "roofline": roofline,
        "hbm_traversal": hbm,
        "cpu_baseline": cpu,
        "self_check": check,
        "build_and_plan_ms": rec["build_and_plan_ms"],
        "autotune": rec["autotune"],
        "job_log": rec["job_log"],
    }
    if extras:
        out["mixed_active"] = {"segments_per_step": rec["seg_mixed"],
                               "fwd_adjoint": {"value": rec["seg_mixed"] / (rec["ms_mixed"] * 1e-3),
                                               "ms": rec["ms_mixed"]},
                               "fractions": "1% / 10% / 100% per scene"}
        out["plain"] = {"fwd": {"value": seg / (rec["ms_plain_f"] * 1e-3), "ms": rec["ms_plain_f"]},
                        "fwd_adjoint": {"value": seg / (rec["ms_plain_fa"] * 1e-3),
                                        "ms": rec["ms_plain_fa"]},
                        "what": "each scene's own tree with the single-tree calls, in turn"}
        rec["forest"].close()
        out["clumpy2e18"] = single_tree(scenes.config_clumpy(), dev, reps=3,
                                        label="clumpy 2^18")
        from paper_2310_15235_amd import api
        kd = single_tree(scenes.config_clumpy(), dev, reps=3, label="clumpy 2^18, depth cache",
                         extra_flags=api.KEEP_DEPTHS)
        out["clumpy2e18"]["keep_depths"] = {k: kd[k] for k in ("fwd", "fwd_adjoint")}
        sc3 = scenes.config_diffuse(active_frac=1.0)
        diffuse = {}
        for frac in (0.01, 0.1, 1.0):
            act = None if frac == 1.0 else scenes.active_subset(sc3, frac, 17)
            r = single_tree(sc3, dev, reps=2, active=act, label=f"diffuse 2^21, {frac:.0%} active")
            diffuse[f"{frac:g}"] = {k: r[k] for k in ("segments", "build_ms", "fwd",
                                                      "fwd_adjoint", "kernel_ms_per_step")}
        out["diffuse2e21"] = diffuse
        out["bands_cost"] = bands_cost(dev)
        out["complex_source_cost"] = complex_source_cost(dev)
    else:
        rec["forest"].close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
