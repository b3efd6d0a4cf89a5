"""Throughput of the gfx950 DG shallow-water step on one MI355X.

Workload: graded unstructured coastal mesh of ~4M triangles (p = 1) with a
Holland hurricane (60 hPa, Rmax 40 km, 5 m/s across the shelf), M2 tide on
the open boundary, Manning n = 0.025 and wetting/drying, FP64 - synthetic
inputs shaped like the paper's Harvey/TX2008 case.

A step is one SSP-RK(2,2) time step (two stages) over the whole mesh;
metric = element-stage updates per second = n_elems x 2 x steps / time.

Prints one JSON line with the metric (FP64), the roofline of the dominant
kernel (algorithmic bytes / HIP-event duration on the solver's stream,
against 8 TB/s), the same workload in mixed precision (FP32 momentum and
flux arithmetic, FP64 elevation and wet/dry) under "variants", and the
FP64 CPU oracle timed on a bounded sample of the same workload on the host
cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "elem-stage updates/s @4M tri p=1, FP64 vs mixed/batched; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Algorithmic bytes of one element-stage of the whole path (FP64), every
# array loaded once: state in 72 + RK base (second stage only) 36 + state out
# 72 + vertex bathymetry 24 + inverse Jacobian and area 40 + neighbour ids and
# orientation 13 + edge normal and length 36 (1.5 edges per element) +
# Manning n 8 + nodal forcing 12 (0.5 nodes per element) + wet/dry status 2.
B_ALG_FP64 = 315.0
# Mixed precision: momentum modes in FP32 (state in 24 + 24, RK base 12 + 12,
# state out 24 + 24), gradients of the basis 16 + area 8, edge normal and
# length in FP32 18, Manning n 4; bathymetry, neighbour data, nodal forcing
# and wet/dry status as in FP64.
B_ALG_MIXED = 217.0


def algorithmic_bytes(kernel: str, ne: int, ned: int, nn: int, precision: str = "fp64") -> float:
    """Algorithmic bytes of one launch: k_stage carries the whole stage
    (B_ALG_FP64 or B_ALG_MIXED per element); k_forcing reads node
    coordinates and writes the nodal wind stress and pressure (40 B per
    node)."""
    if kernel == "k_stage":
        return (B_ALG_MIXED if precision == "mixed" else B_ALG_FP64) * ne
    if kernel == "k_forcing":
        return 40.0 * nn
    raise KeyError(kernel)


def cpu_baseline(wl, target_s=12.0):
    """The FP64 oracle on the same mesh and forcing, on the host cores."""
    from oracle.oracle import Oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = Oracle(wl.mesh, wl.params, wl.forcing)
    o.set_state(wl.w0, 0.0, wl.postprocess_initial)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter() - t0
    more = max(0, min(50, int(target_s / max(t1, 1e-3)) - 1))
    t0 = time.perf_counter()
    if more:
        o.step(more)
    t2 = time.perf_counter() - t0
    steps, secs = (more, t2) if more else (1, t1)
    rate = wl.mesh.n_elems * 2 * steps / secs
    return {"value": rate, "unit": "elem-stage/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps} steps of the same {wl.mesh.n_elems}-element workload after 1 untimed step, "
                      f"{secs:.1f} s, OpenMP threads={threads}"}


def measure(wl, precision, steps, warmup, stream, profile):
    """Create the solver on `stream`, warm up, time `steps` steps with the
    stream synchronised on both sides; returns (elapsed s, solver info,
    per-kernel HIP-event times, diagnostics)."""
    import torch
    from paper_2508_21208_amd.dgswe import DGSWE_FP64, DGSWE_MIXED, Solver, dgswe_profile, dgswe_profile_read
    prm = dict(wl.params, precision=DGSWE_MIXED if precision == "mixed" else DGSWE_FP64)
    s = Solver(wl.mesh, prm, wl.forcing, hip_stream=stream.cuda_stream)
    info = s.info()
    s.set_state(wl.w0, 0.0, wl.postprocess_initial)
    log(f"{precision}: solver ready: {info['n_elems']} elements, {info['n_edges']} edges")
    s.step(warmup)
    s.diagnostics()
    torch.cuda.synchronize()
    if profile:
        dgswe_profile(s.h, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = dgswe_profile_read(s.h) if profile else {}
    if profile:
        dgswe_profile(s.h, 0)
    d = s.diagnostics()
    s.close()
    log(f"{precision}: timed {steps} steps in {elapsed:.4f} s; t={d['t']:.2f} s, dt={d['dt_last']:.4f}, "
        f"wet={d['n_wet']} dry={d['n_dry']}")
    kernels = {}
    for k, (ms, n) in prof.items():
        if n:
            kernels[k] = {"avg_us": 1e3 * ms / n, "launches": n, "total_ms": ms}
    return elapsed, info, kernels, d


def roofline(kernels, ne, ned, nn, precision):
    if not kernels:
        return None
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    avg_s = kernels[dom]["avg_us"] * 1e-6
    b = algorithmic_bytes(dom, ne, ned, nn, precision)
    ach = b / avg_s / 1e9
    for k in kernels:
        kb = algorithmic_bytes(k, ne, ned, nn, precision)
        kernels[k]["alg_GBs"] = round(kb / (kernels[k]["avg_us"] * 1e-6) / 1e9, 1)
    return {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_launch": int(b), "avg_launch_us": round(kernels[dom]["avg_us"], 2)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--elems", type=int, default=4_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision variant")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="precision of the headline run (fp64 is the metric's)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of 2 GiB (3 times) to calibrate HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; a multi-GPU run (domain "
                                   "decomposition with a per-stage halo exchange) is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2508_21208_amd import workloads as W

    t0 = time.perf_counter()
    wl = W.cfg_hurricane(n_target=args.elems)
    log(f"mesh {wl.mesh.n_elems} elements, {wl.mesh.n_nodes} nodes in {time.perf_counter() - t0:.1f} s")
    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    profile = not args.no_profile
    elapsed, info, kernels, d = measure(wl, args.precision, args.steps, args.warmup, stream, profile)
    ne, ned, nn = info["n_elems"], info["n_edges"], info["n_nodes"]
    rate = ne * 2 * args.steps / elapsed
    roof = roofline(kernels, ne, ned, nn, args.precision)
    if kernels:
        log(f"{args.precision} kernels: " + json.dumps(kernels))
    variants = {}
    other = "mixed" if args.precision == "fp64" else "fp64"
    if not args.no_mixed:
        el2, _, k2, d2 = measure(wl, other, args.steps, args.warmup, stream, profile)
        variants[other] = {"value": ne * 2 * args.steps / el2, "unit": "elem-stage/s",
                           "ms_per_step": 1e3 * el2 / args.steps, "roofline": roofline(k2, ne, ned, nn, other),
                           "kernels": k2, "t_end": d2["t"]}
        if k2:
            log(f"{other} kernels: " + json.dumps(k2))

    if args.copy_probe:
        n = 2 * 1024 ** 3 // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 3 x (read 2 GiB + write 2 GiB)")
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle) ...")
        cpu = cpu_baseline(wl)

    out = {
        "metric": METRIC, "value": rate, "unit": "elem-stage/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"hurricane graded coastal mesh, {ne} triangles, p=1, Holland 60 hPa/Rmax 40 km "
                               f"at 5 m/s, M2 tide, Manning 0.025, wet/dry, SSP-RK2",
                   "n_elems": ne, "n_edges": ned, "n_nodes": nn, "p": 1, "precision": args.precision},
        "roofline": roof, "kernels": kernels, "variants": variants, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
