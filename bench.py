"""Throughput of the gfx950 DG shallow-water step on one MI355X.

Workload: graded unstructured coastal mesh of ~4M triangles (p = 1) with a
Holland hurricane (60 hPa, Rmax 40 km, 5 m/s across the shelf), M2 tide on
the open boundary, Manning n = 0.025 and wetting/drying, FP64 - synthetic
inputs shaped like the paper's Harvey/TX2008 case.

A step is one SSP-RK(2,2) time step (two stages) over the whole mesh;
metric = element-stage updates per second = n_elems x 2 x steps / time.

Prints one JSON line with the metric (FP64), the roofline of the dominant
kernel (algorithmic bytes / HIP-event duration on the solver's stream,
against 8 TB/s), under "variants" the same workload in mixed precision
(FP32 momentum and flux arithmetic, FP64 elevation and wet/dry) and a
batched storm-surge ensemble (64 coastal meshes of 50k-500k triangles,
19.5M in total, each with its own hurricane track and Manning n, mixed
precision, one launch per stage for all members), the same 4M workload at
p = 2 (six modes per variable) in FP64 and mixed precision, a serving run
(Poisson arrivals of solve requests of 10k-1M triangles and 100-5,000
steps at ~80 % of the pool's throughput, continuous batching in a
device-resident pool in mixed precision, p50/p99 latency against the same
requests served one at a time in FP64), and the FP64 CPU oracle timed on a
bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "elem-stage updates/s @4M tri p=1, FP64 vs mixed/batched; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_hurricane_4M.json")
KERNEL_SOURCES = ("paper_2508_21208_amd/csrc/dgswe_kernels.hip", "paper_2508_21208_amd/csrc/dgswe_p2.hip",
                  "paper_2508_21208_amd/csrc/dgswe_p1.h", "paper_2508_21208_amd/csrc/dgswe_p2.h",
                  "paper_2508_21208_amd/csrc/dgswe_ens.hip", "paper_2508_21208_amd/csrc/dgswe_device.h",
                  "paper_2508_21208_amd/csrc/dgswe_internal.h", "paper_2508_21208_amd/csrc/mesh_prep.cpp",
                  "paper_2508_21208_amd/csrc/dgswe_api.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Algorithmic bytes of one element-stage of the whole path (FP64), every
# array loaded once: state in 72 + RK base (second stage only) 36 + state out
# 72 + vertex bathymetry 24 + inverse Jacobian and area 40 + neighbour ids and
# orientation 13 + edge normal and length 36 (1.5 edges per element) +
# Manning n 8 + nodal forcing 12 (0.5 nodes per element) + wet/dry status 2.
B_ALG_FP64 = 315.0
# Mixed precision: momentum modes in FP32 (state in 24 + 24, RK base 12 + 12,
# state out 24 + 24), inverse Jacobian and area in FP32 20, edge normal and
# length in FP32 18, Manning n 4, nodal forcing in FP32 6; bathymetry,
# neighbour data and wet/dry status as in FP64.  This is the count the
# roofline fraction uses.
B_ALG_MIXED = 207.0
# The mixed path as built keeps the element area (8 B instead of 4) and the
# nodal forcing (12 B instead of 6) in FP64: 217 B per element-stage,
# reported beside the 207-B figure.
B_ALG_MIXED_AS_BUILT = 217.0
# Context only (not a target, other hardware and precision): the paper's
# AREA + EDGE + GATHER kernels on one H100 (GH200, 4 TB/s HBM3) in FP32 on
# its 6,675,517-triangle mesh: per-launch FLOP counts over the achieved
# FLOP rates give 2.15 + 6.12 + 1.00 = 9.27 ms per stage, i.e. about
# 7.2e8 element-stage updates/s for those three kernels alone (no wet/dry,
# limiter, wind or RK update).
PAPER_CONTEXT = {"value": 7.2e8, "unit": "elem-stage/s", "precision": "fp32",
                 "hardware": "NVIDIA H100 96 GB HBM3, 4 TB/s (GH200 node), one GPU",
                 "workload": "Hurricane Harvey on the 6,675,517-triangle TX2008 mesh, p=1",
                 "covers": "AREA + EDGE + GATHER kernels only, derived from the paper's per-kernel FLOP counts and "
                           "measured FLOP rates (Sec. 6.2); context, not a target"}


# p = 2, per element and launch (averaged over the two stages), every array
# loaded once.  k_pp2: raw state in 144 (mixed 96) + vertex bathymetry 24 +
# neighbour ids 12 + post-processed record out 144 (96).  k_rhs2: record in
# 144 (96) + RK base (second stage only) 72 (48) + vertex bathymetry 24 +
# area and inradius 16 + basis gradients 32 (16) + node ids 16 + edge ids 12
# + neighbour ids 12 + edge normal, length and orientation 48 (1.5 edges per
# element) + mean bathymetry 8 + Manning n 8 (4) + nodal forcing 12 (0.5
# nodes per element) + state out 144 (96).
B_ALG_P2 = {("k_pp2", "fp64"): 324.0, ("k_rhs2", "fp64"): 548.0,
            ("k_pp2", "mixed"): 228.0, ("k_rhs2", "mixed"): 408.0}


def algorithmic_bytes(kernel: str, ne, ned: int, nn: int, precision: str = "fp64") -> float:
    """Algorithmic bytes of one launch: k_stage carries the whole p = 1
    stage (B_ALG_FP64 or B_ALG_MIXED per element), k_pp2 and k_rhs2 the
    p = 2 stage (B_ALG_P2); k_forcing reads node coordinates and writes the
    nodal wind stress and pressure (40 B per node); k_vbounds forms the
    vertex-based limiter's node ranges.  For an ensemble of both orders ne
    is {1: p = 1 elements, 2: p = 2 elements}: k_stage12 carries the p = 1
    stage of the first and the p = 2 right-hand side of the second,
    k_stage1pp2 the p = 1 stage and the p = 2 post-processing."""
    if isinstance(ne, dict):
        n1, n2 = ne.get(1, 0), ne.get(2, 0)
        b1 = B_ALG_MIXED if precision == "mixed" else B_ALG_FP64
        if kernel == "k_stage12":
            return b1 * n1 + B_ALG_P2[("k_rhs2", precision)] * n2
        if kernel == "k_stage1pp2":
            return b1 * n1 + B_ALG_P2[("k_pp2", precision)] * n2
        if kernel == "k_stage":
            return b1 * n1
        if (kernel, precision) in B_ALG_P2:
            return B_ALG_P2[(kernel, precision)] * n2
        ne = n1 + n2
    if kernel == "k_stage":
        return (B_ALG_MIXED if precision == "mixed" else B_ALG_FP64) * ne
    if (kernel, precision) in B_ALG_P2:
        return B_ALG_P2[(kernel, precision)] * ne
    if kernel == "k_forcing":
        return 40.0 * nn
    if kernel == "k_vbounds":
        # per node: incidence range 8 + six bounds out 48; per element: its
        # three incidence entries 12 and its three means, each read once
        # (24 FP64, 16 mixed)
        return 56.0 * nn + (12.0 + (16.0 if precision == "mixed" else 24.0)) * ne
    raise KeyError(kernel)


def source_hash() -> str:
    """sha256 over the kernel, data-layout and launch sources: measured
    traffic belongs to exactly this code."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(kernel: str, precision: str, section: str = "kernels"):
    """HBM bytes per launch of `kernel` measured with rocprofv3 counters for
    the current sources, or None (no record, or the kernels changed since).
    section "kernels": the 4M-triangle runs; "ensemble": the 64-member
    ensemble's launches."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_hash():
        return None
    k = rec.get(section, {}).get(kernel, {}).get(precision)
    return None if k is None else k["bytes_per_launch"]


PROFILED = ("k_stage", "k_pp2", "k_rhs2", "k_stage12", "k_stage1pp2")


def kernel_key(name: str):
    """(kernel, 'fp64' | 'mixed') for a k_stage<NT, WPE, T, STAGE, VL, P>,
    k_pp2<T, STAGE, P>, k_rhs2<T, WPE, P> or k_stage12<T, STAGE, WPE, P>
    kernel name, else None."""
    for k in PROFILED:
        tag = k + "<"
        if tag in name:
            args = [a.strip() for a in name.split(tag, 1)[1].split(">", 1)[0].split(",")]
            t = args[2] if k == "k_stage" else args[0]
            return k, ("mixed" if t == "float" else "fp64")
    return None


CMD_TRACE = ("rocprofv3 --kernel-trace --stats -d $OUT/prof -o bench --output-format csv -- "
             "python3 $REPO/bench.py --steps 50 --warmup 5 --no-cpu-baseline --no-profile --no-batched --no-serving "
             "--no-rk --no-graphs")
CMD_PMC = ("rocprofv3 --pmc {c} -d $OUT/pmc/{c} -o run --output-format csv -- python3 $REPO/bench.py --steps 3 "
           "--warmup 1 --no-cpu-baseline --no-profile --copy-probe --no-batched --no-serving --no-rk --no-graphs")
CMD_SUMMARIZE = ("cd $REPO && python3 bench.py --summarize-pmc $OUT/pmc --kernel-trace $OUT/prof/bench_kernel_trace.csv "
                 "--ensemble-kernel-trace $OUT/prof_ens/bench_kernel_trace.csv --summary-md "
                 "profiles/k_stage_hurricane_4M.md")
# the ensemble's launch parameters in its benched line and profiles: the
# library's defaults (chunk 0: chosen per mesh; p = 2 register budget 0)
ENSEMBLE_DEFAULTS = {1: {"chunk": 0, "waves": 0}, 2: {"chunk": 0, "waves": 0}}
CMD_TRACE_ENS = ("rocprofv3 --kernel-trace --stats -d $OUT/prof_ens -o bench --output-format csv -- "
                 "python3 $REPO/bench.py --only-batched --no-ensemble-autotune --steps 50 --warmup 5 --no-profile")
CMD_PMC_ENS = ("rocprofv3 --pmc {c} -d $OUT/pmc/ensemble/{c} -o run --output-format csv -- python3 $REPO/bench.py "
               "--only-batched --no-ensemble-autotune --steps 3 --warmup 1 --no-profile --copy-probe")


def _pmc_rows(pmc_dir, tag):
    with open(os.path.join(pmc_dir, tag, "run_counter_collection.csv")) as fh:
        return list(csv.DictReader(fh))


def _pmc_traffic(pmc_dir, largest_grid):
    """(calibration, {(kernel, precision): record}) from the FETCH_SIZE and
    WRITE_SIZE runs under pmc_dir.  largest_grid: per kernel and precision
    keep only the dispatches of the largest grid (the 4M runs also hold the
    small mixed-precision error check; the ensemble run the autotuner's
    single-member launches and the persistent workgroups' smaller grids)."""
    copy_bytes = 2 * 1024 ** 3
    calib, vals = {}, {}
    for tag in ("FETCH_SIZE", "WRITE_SIZE"):
        rows = _pmc_rows(pmc_dir, tag)
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        big = max(copies)
        scale = copy_bytes / (big * 1024.0)
        calib[tag] = {"copy_KiB": big, "bytes_per_KiB": round(scale * 1024.0, 1), "factor": round(scale, 3)}
        for r in rows:
            kk = kernel_key(r["Kernel_Name"])
            if kk:
                grid = int(float(r.get("Grid_Size") or 0))
                vals.setdefault(kk, {}).setdefault(tag, []).append((grid, float(r["Counter_Value"])))
    out = {}
    for kk, d in vals.items():
        if len(d) < 2:
            continue
        if largest_grid:
            common = {x[0] for x in d["FETCH_SIZE"]} & {x[0] for x in d["WRITE_SIZE"]}
            if not common:
                continue
            g = max(common)
            d = {t: [x for x in v if x[0] == g] for t, v in d.items()}
            if not d["FETCH_SIZE"] or not d["WRITE_SIZE"]:
                continue
        fk = sum(x[1] for x in d["FETCH_SIZE"]) / len(d["FETCH_SIZE"])
        wk = sum(x[1] for x in d["WRITE_SIZE"]) / len(d["WRITE_SIZE"])
        b = fk * 1024.0 * calib["FETCH_SIZE"]["factor"] + wk * 1024.0 * calib["WRITE_SIZE"]["factor"]
        rec = {"fetch_KiB": round(fk, 1), "write_KiB": round(wk, 1),
               "dispatches": [len(d["FETCH_SIZE"]), len(d["WRITE_SIZE"])], "bytes_per_launch": round(b)}
        if largest_grid:
            rec["grid_size"] = g
        out[kk] = rec
    return calib, out


def _trace_groups(trace_csv):
    """{kernel name: {grid work-items: [durations in us]}} of the stage
    kernels and k_forcing in a rocprofv3 kernel_trace.csv"""
    groups = {}
    with open(trace_csv) as fh:
        for r in csv.DictReader(fh):
            if not (kernel_key(r["Kernel_Name"]) or "k_forcing" in r["Kernel_Name"]):
                continue
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            groups.setdefault(r["Kernel_Name"], {}).setdefault(grid, []).append(dur)
    return groups


CMD_COUNTERS = ('ARGS="--steps 3 --warmup 1 --no-cpu-baseline --no-profile --no-batched --no-serving --no-rk '
                '--no-graphs"',
                "timeout -s KILL 240 rocprofv3 --pmc SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_ANY "
                "SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_LDS SQ_INSTS_VALU SQ_INSTS_VMEM_RD GRBM_GUI_ACTIVE -d $OUT/c1 -o run "
                "--output-format csv -- python3 $REPO/bench.py $ARGS",
                "timeout -s KILL 240 rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum SQ_LDS_BANK_CONFLICT SQ_INSTS_LDS "
                "SQ_WAIT_ANY SQ_ACTIVE_INST_ANY GRBM_GUI_ACTIVE -d $OUT/c2 -o run --output-format csv -- "
                "python3 $REPO/bench.py $ARGS")


def summarize_counters(cdir: str, kernels: tuple, title: str, out_md: str):
    """Issue, wait and cache counters per kernel instance (the 4M-mesh
    launches: largest grid) from the two rocprofv3 --pmc runs c1 and c2 of
    CMD_COUNTERS under cdir, as a markdown table."""
    per = {}
    for tag in ("c1", "c2"):
        for r in _pmc_rows(cdir, tag):
            kk = kernel_key(r["Kernel_Name"])
            if not kk or kk[0] not in kernels:
                continue
            grid = int(float(r.get("Grid_Size") or 0))
            d = per.setdefault(r["Kernel_Name"], {}).setdefault(grid, {})
            d.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    rows = []
    for name, by in sorted(per.items()):
        c = {k: sum(v) / len(v) for k, v in by[max(by)].items()}
        n = {k: len(v) for k, v in by[max(by)].items()}
        wv, cyc = c.get("SQ_WAVES", 0.0), c.get("SQ_WAVE_CYCLES", 0.0)
        if not wv or not cyc:
            continue
        hit, miss = c.get("TCC_HIT_sum", 0.0), c.get("TCC_MISS_sum", 0.0)
        pct = lambda k: f"{100.0 * c.get(k, 0.0) / cyc:.1f}"
        nm = name.split("(")[0].replace("dgswe::", "").replace("void ", "")
        lds_act = c.get("SQ_ACTIVE_INST_LDS", 0.0)
        rows.append(f"| `{nm}` | {n.get('SQ_WAVES', 0)} | {wv:.0f} | {c.get('SQ_INSTS_VALU', 0.0) / wv:.0f} | "
                    f"{c.get('SQ_INSTS_LDS', 0.0) / wv:.0f} | {c.get('SQ_INSTS_VMEM_RD', 0.0) / wv:.0f} | "
                    f"{pct('SQ_ACTIVE_INST_ANY')} | {pct('SQ_ACTIVE_INST_VALU')} | {pct('SQ_ACTIVE_INST_LDS')} | "
                    f"{pct('SQ_WAIT_INST_ANY')} | {pct('SQ_WAIT_ANY')} | "
                    f"{100.0 * c.get('SQ_LDS_BANK_CONFLICT', 0.0) / lds_act if lds_act else 0.0:.0f} | "
                    f"{100.0 * hit / (hit + miss) if hit + miss else 0.0:.1f} | {miss * 128 / 1e9:.3f} GB |")
    out = [f"# {title}", "", "Commands, on one MI355X, with REPO = the repository root and OUT = an output folder:",
           "", "```", "cd /tmp && export TMPDIR=/tmp", *CMD_COUNTERS,
           f"cd $REPO && python3 bench.py --summarize-counters $OUT --counter-kernels {','.join(kernels)} "
           f"--summary-md {out_md if out_md.startswith('profiles/') else 'profiles/' + os.path.basename(out_md)}",
           "```", "", f"Kernel sources sha256: `{source_hash()}`", "",
           "Averages per launch over the 4M-mesh dispatches of each kernel instance (largest grid). Per-wave "
           "counts divide by SQ_WAVES; time shares divide by SQ_WAVE_CYCLES, the cycles the waves were resident: "
           "issuing = SQ_ACTIVE_INST_ANY, VALU = SQ_ACTIVE_INST_VALU, LDS = SQ_ACTIVE_INST_LDS, waiting on "
           "dependencies = SQ_WAIT_INST_ANY, waiting (any) = SQ_WAIT_ANY; bank conflicts as a share of the LDS "
           "cycles; L2 bytes missed = TCC_MISS_sum x 128 B.", "",
           "| kernel | dispatches | waves | VALU / wave | LDS / wave | VMEM reads / wave | issuing % | VALU % | "
           "LDS % | waiting on dependencies % | waiting (any) % | LDS bank-conflict share % | L2 hit rate % | "
           "L2 misses x 128 B |", "|---|---|---|---|---|---|---|---|---|---|---|---|---|---|", *rows, ""]
    with open(out_md, "w") as fh:
        fh.write("\n".join(out))
    print("\n".join(rows))


def summarize_pmc(pmc_dir: str, trace_csv: str | None, out_md: str | None, ens_trace_csv: str | None = None):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE, KiB per
    dispatch) of `bench.py --copy-probe` into HBM bytes per launch of each
    stage kernel and precision.  Each counter is scaled by what it reads for
    the 2 GiB device copy in the same run (bytes moved / counter reading).
    The same two runs of `bench.py --only-batched` under pmc_dir/ensemble,
    if present, give the ensemble's launches.  out_md: the p = 1 summary;
    the p = 2 and ensemble ones go beside it."""
    res = {"source_sha256": source_hash(), "kernels": {}, "calibration": {}}
    res["calibration"], per = _pmc_traffic(pmc_dir, True)
    for (k, prec), r in per.items():
        res["kernels"].setdefault(k, {})[prec] = r
    ens_dir = os.path.join(pmc_dir, "ensemble")
    if os.path.isdir(ens_dir):
        res["ensemble_calibration"], per = _pmc_traffic(ens_dir, True)
        res["ensemble_launch"] = "library defaults (chunk 0, waves 0)"
        res["ensemble"] = {}
        for (k, prec), r in per.items():
            res["ensemble"].setdefault(k, {})[prec] = r
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res, indent=1))
    if not out_md:
        return
    groups = _trace_groups(trace_csv) if trace_csv else {}
    c = res["calibration"]
    head = ["Commands, on one MI355X, with REPO = the repository root and OUT = an output folder:", "", "```",
            "cd /tmp && export TMPDIR=/tmp", CMD_TRACE, CMD_PMC.format(c="FETCH_SIZE"), CMD_PMC.format(c="WRITE_SIZE"),
            CMD_SUMMARIZE, "```", "",
            "One bench process runs the p = 1 FP64 headline, the p = 1 mixed variant, then p = 2 in FP64 and "
            "mixed, on the same 4M-triangle mesh.", "",
            f"Kernel sources sha256 (bench.py reports this traffic only for these sources): `{res['source_sha256']}`",
            ""]
    calib = ["", "Calibration: a 2 GiB device copy in the same runs reads "
             f"{c['FETCH_SIZE']['copy_KiB']:.0f} KiB FETCH_SIZE and {c['WRITE_SIZE']['copy_KiB']:.0f} KiB "
             f"WRITE_SIZE, so fetched bytes = FETCH_SIZE x {c['FETCH_SIZE']['bytes_per_KiB']} B and written "
             f"bytes = WRITE_SIZE x {c['WRITE_SIZE']['bytes_per_KiB']} B.", ""]

    def section(title, kernels):
        out = [f"# {title}", ""] + head
        sel = {n: by for n, by in groups.items() if (kernel_key(n) or ("",))[0] in kernels}
        if sel:
            out += ["## Kernel trace (`--kernel-trace`; the 4M-mesh launches, i.e. the largest grid of each kernel)",
                    "", "| kernel | launches | avg us | min us | max us |", "|---|---|---|---|---|"]
            big = {n: by[max(by)] for n, by in sel.items()}
            for n, d in sorted(big.items()):
                nm = n.split("(")[0].replace("dgswe::", "")
                out.append(f"| `{nm}` | {len(d)} | {sum(d) / len(d):.1f} | {min(d):.1f} | {max(d):.1f} |")
            out.append("")
            for k in kernels:
                for prec in ("fp64", "mixed"):
                    ds = [x for n, d in big.items() if kernel_key(n) == (k, prec) for x in d]
                    if ds:
                        out.append(f"{k} {prec}, both RK stages: {len(ds)} launches, average "
                                   f"{sum(ds) / len(ds):.1f} us (bench.py reports the HIP-event average over the "
                                   f"same kernels).")
            out.append("")
        out += ["## HBM traffic per launch (mean over both RK stages, 4M-mesh launches)", "",
                "| kernel | precision | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes per launch (calibrated) |",
                "|---|---|---|---|---|"]
        for k in kernels:
            for prec, d in res["kernels"].get(k, {}).items():
                out.append(f"| {k} | {prec} | {d['fetch_KiB']:.0f} | {d['write_KiB']:.0f} | "
                           f"{d['bytes_per_launch'] / 1e9:.3f} GB |")
        return out + calib

    with open(out_md, "w") as fh:
        fh.write("\n".join(section("k_stage (p = 1) on the 4M-triangle hurricane workload: kernel times and HBM "
                                   "traffic", ("k_stage",))))
    p2_md = os.path.join(os.path.dirname(out_md), "k_rhs2_k_pp2_hurricane_4M_p2.md")
    with open(p2_md, "w") as fh:
        fh.write("\n".join(section("k_pp2 and k_rhs2 (p = 2) on the 4M-triangle hurricane workload: kernel times "
                                   "and HBM traffic", ("k_pp2", "k_rhs2"))))
    if "ensemble" not in res:
        return
    ce = res["ensemble_calibration"]
    out = ["# The 64-member storm-surge ensemble (27 members at p = 1, 37 at p = 2, mixed precision): kernel "
           "times and HBM traffic", "",
           "Commands, on one MI355X, with REPO = the repository root and OUT = an output folder:", "", "```",
           "cd /tmp && export TMPDIR=/tmp", CMD_TRACE_ENS, CMD_PMC_ENS.format(c="FETCH_SIZE"),
           CMD_PMC_ENS.format(c="WRITE_SIZE"),
           CMD_SUMMARIZE,
           "```", "",
           "One bench process (the library's default launch parameters: chunk sizes chosen per mesh) "
           "advances the ensemble in each arrangement (two streams; the pair with the p = 1 stage and the p = 2 "
           "post-processing in one launch, then the p = 2 right-hand side; both orders' stage work in one "
           "launch; persistent workgroups), then all 64 members at p = 1.", "",
           f"Kernel sources sha256: `{res['source_sha256']}`", ""]
    if ens_trace_csv:
        # per kernel instance, the launches of its largest grid (the
        # ensemble-sized ones; the autotuner runs on single member meshes)
        groups = _trace_groups(ens_trace_csv)
        out += ["## Kernel trace (`--kernel-trace`): the ensemble-sized launches (largest grid) of each kernel", "",
                "| kernel | grid (work-items) | launches | avg us | min us | max us |", "|---|---|---|---|---|---|"]
        rows = []
        for name, by in groups.items():
            g = max(by)
            d = by[g]
            rows.append((sum(d), name.split("(")[0].replace("dgswe::", ""), g, d))
        for tot, nm, g, d in sorted(rows, reverse=True):
            out.append(f"| `{nm}` | {g} | {len(d)} | {tot / len(d):.1f} | {min(d):.1f} | {max(d):.1f} |")
        out += ["", "Launch counts: 55 per arrangement and stage (5 warm-up + 50 timed steps), more for a kernel "
                "that several arrangements launch.", ""]
    out += ["## HBM traffic per launch (the ensemble-sized launches: the largest grid of each kernel)", "",
            "| kernel | precision | grid (work-items) | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes per launch "
            "(calibrated) |", "|---|---|---|---|---|---|---|"]
    for k in PROFILED:
        for prec, d in res["ensemble"].get(k, {}).items():
            out.append(f"| {k} | {prec} | {d['grid_size']} | {d['dispatches'][0]} | {d['fetch_KiB']:.0f} | "
                       f"{d['write_KiB']:.0f} | {d['bytes_per_launch'] / 1e9:.3f} GB |")
    out += ["", "Calibration: a 2 GiB device copy in the same runs reads "
            f"{ce['FETCH_SIZE']['copy_KiB']:.0f} KiB FETCH_SIZE and {ce['WRITE_SIZE']['copy_KiB']:.0f} KiB "
            f"WRITE_SIZE.", ""]
    with open(os.path.join(os.path.dirname(out_md), "ensemble_64_members_mixed.md"), "w") as fh:
        fh.write("\n".join(out))


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo, as lscpu shows it)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n):
    """Set the OpenMP thread count of this process (the oracle's runtime)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except (OSError, AttributeError):
        return False


def cpu_baseline(wl, steps=50, single_s=12.0):
    """The FP64 oracle as it stands on the same mesh and forcing: `steps`
    steps on all the host threads OpenMP is given, then a bounded sample on
    one thread."""
    from oracle.oracle import Oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    o = Oracle(wl.mesh, wl.params, wl.forcing)
    o.set_state(wl.w0, 0.0, wl.postprocess_initial)
    o.step(1)
    t0 = time.perf_counter()
    o.step(steps)
    secs = time.perf_counter() - t0
    rate = wl.mesh.n_elems * 2 * steps / secs
    out = {"value": rate, "unit": "elem-stage/s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
           "logical_cpus": os.cpu_count(),
           "sample": f"{steps} steps of the same {wl.mesh.n_elems}-element workload after 1 untimed step, "
                     f"{secs:.1f} s, OpenMP threads={threads}"}
    if _omp_threads(1):
        t0 = time.perf_counter()
        o.step(1)
        t1 = time.perf_counter() - t0
        n1 = max(2, int(single_s / max(t1, 1e-3)) - 1)
        t0 = time.perf_counter()
        if n1:
            o.step(n1)
        t2 = time.perf_counter() - t0
        n_1, s_1 = (n1, t2) if n1 else (1, t1)
        _omp_threads(threads)
        out["single_thread"] = {"value": wl.mesh.n_elems * 2 * n_1 / s_1, "unit": "elem-stage/s",
                                "sample": f"{n_1} steps after 1 untimed step on one thread, {s_1:.1f} s"}
    return out


def measure(wl, precision, steps, warmup, stream, profile, order=1, extra=None, forcing=None, keep=None, repeats=1):
    """Create the solver on `stream`, warm up, then `repeats` times time
    `steps` steps with the stream synchronised on both sides; returns (median
    elapsed s, solver info, per-kernel HIP-event times over all repeats,
    diagnostics, every elapsed s).  order 2: p = 2 with CFL 0.1, starting
    from the p = 1 initial state with zero quadratic modes."""
    import torch
    from paper_2508_21208_amd.dgswe import DGSWE_FP64, DGSWE_MIXED, Solver, dgswe_profile, dgswe_profile_read
    prm = dict(wl.params, precision=DGSWE_MIXED if precision == "mixed" else DGSWE_FP64)
    w0 = wl.w0
    if order == 2:
        prm.update(p=2, cfl=0.1)
        w0 = np.zeros((3, 6, wl.w0.shape[2]))
        w0[:, :3] = wl.w0
    prm.update(extra or {})
    s = Solver(wl.mesh, prm, dict(wl.forcing, **(forcing or {})), hip_stream=stream.cuda_stream)
    info = s.info()
    s.set_state(w0, 0.0, wl.postprocess_initial)
    log(f"{precision}: solver ready: {info['n_elems']} elements, {info['n_edges']} edges")
    s.step(warmup)
    s.diagnostics()
    torch.cuda.synchronize()
    if profile:
        dgswe_profile(s.h, 1)
    runs = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
    elapsed = float(np.median(runs))
    prof = dgswe_profile_read(s.h) if profile else {}
    if profile:
        dgswe_profile(s.h, 0)
    d = s.diagnostics()
    if keep is not None:
        keep["state"] = s.state()  # after the timed region
        keep["steps"] = warmup + repeats * steps
    s.close()
    log(f"{precision}: timed {repeats} x {steps} steps, median {elapsed:.4f} s "
        f"({', '.join(f'{r:.4f}' for r in runs)}); t={d['t']:.2f} s, dt={d['dt_last']:.4f}, "
        f"wet={d['n_wet']} dry={d['n_dry']}")
    kernels = {}
    for k, (ms, n) in prof.items():
        if n:
            kernels[k] = {"avg_us": 1e3 * ms / n, "launches": n, "total_ms": ms}
    return elapsed, info, kernels, d, runs


def measure_host_roundtrip(wl, steps, stream):
    """The same FP64 solve with the state handed over through host memory
    (the boundary's dgswe_set_state / dgswe_read_state, i.e. PCIe and the
    host-side reordering into the caller's element order): elapsed seconds
    of upload, steps and read-back."""
    import torch
    from paper_2508_21208_amd.dgswe import Solver
    s = Solver(wl.mesh, dict(wl.params), wl.forcing, hip_stream=stream.cuda_stream)
    s.set_state(wl.w0, 0.0, wl.postprocess_initial)  # warm-up of every path
    s.step(2)
    s.state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_state(wl.w0, 0.0, wl.postprocess_initial)
    t1 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    w = s.state()
    t3 = time.perf_counter()
    s.close()
    del w
    return {"upload_s": t1 - t0, "steps_s": t2 - t1, "readback_s": t3 - t2, "total_s": t3 - t0}


def mixed_error(wm, wf):
    """The mixed-precision state against the FP64 one after the same steps
    (the FP64 path equals the FP64 oracle to 1e-12, tested at this size):
    largest vertex elevation difference, largest element-mean depth and
    momentum differences, relative L2 per variable."""
    V = np.array([[1.0, -1.0, -1.0], [1.0, 1.0, -1.0], [1.0, 0.0, 2.0]])
    dz = np.abs(V @ (wm[0] - wf[0])).max()
    rel = [float(np.linalg.norm(wm[v] - wf[v]) / max(np.linalg.norm(wf[v]), 1e-300)) for v in range(3)]
    return {"zeta_vertex_max_m": float(dz), "zeta_mean_max_m": float(np.abs(wm[0, 0] - wf[0, 0]).max()),
            "q_mean_max_m2s": float(np.abs(wm[1:, 0] - wf[1:, 0]).max()), "rel_l2": rel}


MIXED_ERROR_FILE = os.path.join(ROOT, "profiles", "mixed_error_vs_oracle.json")


def mixed_error_vs_oracle(stream):
    """Largest elevation error at element vertices and velocity error at
    element means of the mixed path against the FP64 oracle at the
    configured horizons.  The 1,600-element Gaussian hump (200 steps) is
    measured here; the two full-size coastal workloads (600k triangles at
    2,000 steps, 4M at 1,000) take the oracle minutes, so their figures come
    from the full-horizon parity tests' report (profiles/, with the kernel
    sources' hash they were measured on)."""
    import torch
    from oracle.oracle import Oracle
    from paper_2508_21208_amd import workloads as W
    from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Solver
    wl = W.cfg_gaussian_1600()
    s = Solver(wl.mesh, dict(wl.params, precision=DGSWE_MIXED), wl.forcing, hip_stream=stream.cuda_stream)
    s.set_state(wl.w0, 0.0, wl.postprocess_initial)
    s.step(wl.steps)
    wg = s.state()
    dg = s.diagnostics()
    s.close()
    torch.cuda.synchronize()
    o = Oracle(wl.mesh, wl.params, wl.forcing)
    o.set_state(wl.w0, 0.0, wl.postprocess_initial)
    o.step(wl.steps)
    wo = o.state()
    V = np.array([[1.0, -1.0, -1.0], [1.0, 1.0, -1.0], [1.0, 0.0, 2.0]])
    H = wo[0, 0] + wl.mesh.hb[wl.mesh.tri].mean(axis=1)
    Hg = wg[0, 0] + wl.mesh.hb[wl.mesh.tri].mean(axis=1)
    ok = H >= 0.5
    ev = max(float(np.abs(wg[v, 0][ok] / Hg[ok] - wo[v, 0][ok] / H[ok]).max()) for v in (1, 2))
    out = {"gaussian_1600/mixed": {"steps": wl.steps, "zeta_vertex_max_m": float(np.abs(V @ (wg[0] - wo[0])).max()),
                                   "velocity_mean_max_ms": ev, "t_end": dg["t"], "t_oracle": o.t,
                                   "source": "measured by this run"}}
    try:
        with open(MIXED_ERROR_FILE) as fh:
            rec = json.load(fh)
        same = rec.get("source_sha256") == source_hash()
        for k, v in rec.get("results", {}).items():
            if k.endswith("/mixed"):
                out[k] = dict(v, source="tests/test_full_horizon_gpu.py report in profiles/",
                              sources_match_this_build=same)
    except (OSError, ValueError):
        pass
    return out


def tune_ensemble_orders(ens, orders, stream):
    """Chunk size (and at p = 2 the register budget) per order from the
    autotuner, timed on the median-size member mesh of that order in mixed
    precision; returns ({order: params}, {order: table})."""
    from paper_2508_21208_amd import workloads as W
    from paper_2508_21208_amd.autotune import tune
    from paper_2508_21208_amd.dgswe import DGSWE_MIXED
    out, tables = {}, {}
    for p in (1, 2):
        idx = sorted((i for i, o in enumerate(orders) if o == p), key=lambda i: ens[i].mesh.n_elems)
        if not idx:
            continue
        w = ens[idx[len(idx) // 2]]
        prm = dict(w.params, precision=DGSWE_MIXED, p=p, **({"cfl": 0.1} if p == 2 else {}))
        w0 = w.w0 if p == 1 else np.concatenate([w.w0, np.zeros((3, 3, w.w0.shape[2]))], axis=1)
        best, table = tune(w.mesh, prm, w.forcing, w0, w.postprocess_initial, steps=20, hip_stream=stream.cuda_stream,
                           use_cache=False)
        out[p] = {k: best[k] for k in ("chunk", "waves")}
        tables[p] = {"mesh_elems": w.mesh.n_elems,
                     "us_per_step": {f"chunk {r[0]}, waves {r[1]}": round(r[2], 1) for r in table}}
        log(f"ensemble tuning p = {p} on {w.mesh.n_elems} triangles: {out[p]}")
    return out, tables


def measure_ensemble(ens, steps, warmup, stream, profile, tuned=None, fused=True, graphs=6, persistent=0,
                     orders=None):
    """The storm-surge ensemble (NEXT-2 configuration): seeded orders p in
    {1, 2}, mixed precision, the p = 2 members at CFL 0.1, chunk sizes from
    the autotuner, step graphs; fused: both orders advanced by
    dgswe_step_pair (one stage launch for every member), else batch by
    batch.  Returns the variant record; with profile the
    kernels' HIP-event averages come from a second, plain (graph-free) run."""
    import torch
    from paper_2508_21208_amd import workloads as W
    from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Ensemble, dgswe_mesh_info, dgswe_profile, dgswe_profile_read
    orders = orders if orders is not None else W.ensemble_orders(len(ens))
    ne = {p: sum(w.mesh.n_elems for w, o in zip(ens, orders) if o == p) for p in (1, 2)}
    op = {1: dict(persistent=persistent, **(tuned or {}).get(1, {})),
          2: dict(cfl=0.1, persistent=persistent, **(tuned or {}).get(2, {}))}
    t0 = time.perf_counter()
    e = Ensemble([w.mesh for w in ens], orders, dict(ens[0].params, precision=DGSWE_MIXED),
                 [w.forcing for w in ens], hip_stream=stream.cuda_stream, order_params=op, fused=fused)
    e.use_graphs(graphs)
    for i, w in enumerate(ens):
        e.set_state(i, w.w0, 0.0, w.postprocess_initial)
    info = {p: dgswe_mesh_info(b.h) for p, b in e.batches.items()}
    tag = f"ensemble fused={fused} graphs={graphs} persistent={persistent}"
    log(f"{tag}: {orders.count(1)} p=1 members ({ne[1]} el), {orders.count(2)} p=2 members ({ne[2]} el), "
        f"ready in {time.perf_counter() - t0:.1f} s")
    e.step(warmup)
    e.diagnostics(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ts = [e.diagnostics(i)["t"] for i in range(len(ens))]
    kernels = {}
    if profile:
        for b in e.batches.values():
            dgswe_profile(b.h, 1)
        e.step(20)
        torch.cuda.synchronize()
        for b in e.batches.values():
            for k, (ms, n) in dgswe_profile_read(b.h).items():
                if n:
                    r = kernels.setdefault(k, {"total_ms": 0.0, "launches": 0})
                    r["total_ms"] += ms
                    r["launches"] += n
            dgswe_profile(b.h, 0)
        for r in kernels.values():
            r["avg_us"] = 1e3 * r["total_ms"] / r["launches"]
    e.close()
    log(f"{tag}: timed {steps} steps in {elapsed:.4f} s; member times {min(ts):.1f}-{max(ts):.1f} s")
    nn = sum(int(v["n_nodes"]) for v in info.values())
    ned = sum(int(v["n_edges"]) for v in info.values())
    rec = {"value": 2 * (ne[1] + ne[2]) * steps / elapsed, "unit": "elem-stage/s", "precision": "mixed",
           "members": len(ens), "members_p1": orders.count(1), "members_p2": orders.count(2),
           "n_elems_p1": ne[1], "n_elems_p2": ne[2], "n_nodes": nn, "n_edges": ned,
           "ms_per_step": 1e3 * elapsed / steps, "graphs": graphs, "fused_one_launch": fused,
           "persistent": persistent, "chunk_params": op, "kernels": kernels,
           "note": "element-stages of both orders counted alike; a p = 2 element-stage does about 2.6x the work"}
    if kernels:
        # the ensemble's measured traffic belongs to its profiled launch
        # parameters (the library's defaults)
        same = persistent == 0 and all(op[o].get(k, 0) == v for o in (1, 2) for k, v in ENSEMBLE_DEFAULTS[o].items())
        rec["roofline"] = roofline(kernels, {1: ne[1], 2: ne[2]}, ned, nn, "mixed", with_traffic=same,
                                   section="ensemble")
    return rec


def measure_serving(n_requests, pool_rate_hint, stream):
    """Serving: the pool (mixed, continuous batching) and the one-at-a-time
    FP64 baseline on the same Poisson arrivals; the arrival rate offers 80 %
    of pool_rate_hint (elem-stage/s)."""
    from paper_2508_21208_amd import workloads as W
    from paper_2508_21208_amd.serving import serve_one_at_a_time, serve_pool, summarize
    t0 = time.perf_counter()
    meshes = W.serving_meshes()
    reqs = W.cfg_serving(n_requests, meshes=meshes)
    work = float(np.mean([r.mesh.n_elems * r.horizon * 2 for r in reqs]))
    lam = 0.8 * pool_rate_hint / work
    log(f"serving: {len(reqs)} requests on {len(meshes)} meshes ({min(m.n_elems for m in meshes)}-"
        f"{max(m.n_elems for m in meshes)} triangles) in {time.perf_counter() - t0:.1f} s; "
        f"{lam:.2f} requests/s")
    # chunk sizes from the autotuner's measurements: 128 below 50k triangles
    out, el = serve_pool(reqs, W.default_params(precision=1, dt_max=0.3), lam, max_elems=16_000_000,
                         max_members=256, round_cap=100, hip_stream=stream.cuda_stream,
                         chunk_rule=lambda n: 128 if n < 50_000 else 256)
    pool = summarize(out, el)
    log("serving pool: " + json.dumps(pool))
    out2, el2 = serve_one_at_a_time(reqs, W.default_params(precision=0, dt_max=0.3), lam, deadline_s=3 * el,
                                    hip_stream=stream.cuda_stream)
    alone = summarize(out2, el2) if out2 else None
    if alone:
        alone["completed_of"] = len(reqs)
    log("serving one at a time: " + json.dumps(alone))
    return {"requests": len(reqs), "arrival_rate_per_s": lam, "offered_load": 0.8,
            "mean_request_elem_stages": work, "pool_mixed": pool, "one_at_a_time_fp64": alone,
            "p50_speedup": alone["p50_s"] / pool["p50_s"] if alone else None,
            "p99_speedup": alone["p99_s"] / pool["p99_s"] if alone else None}


def measure_graphs(stream, steps=600):
    """Launch cost on a small mesh: the 1,600-element Gaussian hump (FP64),
    steps launched one by one against replays of captured 60-step graphs."""
    import torch
    from paper_2508_21208_amd.dgswe import Solver
    from paper_2508_21208_amd import workloads as W
    wl = W.cfg_gaussian_1600()
    out = {"workload": "Gaussian hump, 1,600 triangles, FP64", "steps": steps}
    for name, g in (("plain", 0), ("graphs", 60)):
        s = Solver(wl.mesh, wl.params, wl.forcing, hip_stream=stream.cuda_stream)
        s.set_state(wl.w0)
        s.use_graphs(g)
        s.step(120)
        s.diagnostics()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        s.diagnostics()
        el = time.perf_counter() - t0
        s.close()
        out[name] = {"steps_per_s": steps / el, "us_per_step": 1e6 * el / steps}
    out["speedup"] = out["graphs"]["steps_per_s"] / out["plain"]["steps_per_s"]
    log("graphs: " + json.dumps(out))
    return out


def measure_autotune(stream):
    """The launch autotuner on two coastal meshes (10k and 130k triangles,
    FP64, tide): microseconds per step for each chunk size ("auto": the
    library's per-mesh default)."""
    from paper_2508_21208_amd import workloads as W
    from paper_2508_21208_amd.autotune import tune
    out = {}
    for n, seed in ((10_000, W.BASE_SEED + 5001), (130_000, W.BASE_SEED + 5006)):
        m = W.coastal_mesh(n, seed, hmin=1000.0 if n < 30_000 else 200.0, hmax=15000.0 if n < 30_000 else 5000.0)
        best, table = tune(m, W.default_params(dt_max=0.3), W.default_forcing(manning_n=0.025, **W.m2_tide(1.0)),
                           W.coastal_initial_state(m), steps=40, hip_stream=stream.cuda_stream, use_cache=False)
        default = [r[2] for r in table if r[0] == 0][0]
        out[str(m.n_elems)] = {"us_per_step": {("auto" if r[0] == 0 else str(r[0])): round(r[2], 1) for r in table},
                               "best_chunk": best["chunk"] or "auto",
                               "speedup_vs_default": default / min(r[2] for r in table)}
    log("autotune: " + json.dumps(out))
    return out


def roofline(kernels, ne, ned, nn, precision, with_traffic=True, section="kernels"):
    if not kernels:
        return None
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    avg_s = kernels[dom]["avg_us"] * 1e-6
    b = algorithmic_bytes(dom, ne, ned, nn, precision)
    ach = b / avg_s / 1e9
    for k in kernels:
        kb = algorithmic_bytes(k, ne, ned, nn, precision)
        kernels[k]["alg_GBs"] = round(kb / (kernels[k]["avg_us"] * 1e-6) / 1e9, 1)
    traffic = stored_traffic(dom, precision, section) if with_traffic else None
    out = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
           "bytes_per_launch": int(b), "avg_launch_us": round(kernels[dom]["avg_us"], 2)}
    if dom == "k_stage" and precision == "mixed":
        b2 = B_ALG_MIXED_AS_BUILT * (ne.get(1, 0) if isinstance(ne, dict) else ne)
        out["as_built"] = {"bytes_per_element_stage": B_ALG_MIXED_AS_BUILT, "bytes_per_launch": int(b2),
                           "frac": round(b2 / avg_s / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def measure_batched(args, stream, profile):
    """The batched ensemble variants: the library's default arrangement
    (dgswe_step_pair, "pair") at the library's default launch parameters as
    "batched" (what its profiles measure), the other arrangements and the
    autotuner's launch parameters under "batched_modes", and all 64 members
    at p = 1."""
    from paper_2508_21208_amd import workloads as W
    variants = {}
    t0 = time.perf_counter()
    ens = W.cfg_ensemble()
    orders = W.ensemble_orders(len(ens))
    log(f"ensemble: {len(ens)} members, {sum(w.mesh.n_elems for w in ens)} elements, generated in "
        f"{time.perf_counter() - t0:.1f} s")
    defaults = {o: dict(v) for o, v in ENSEMBLE_DEFAULTS.items()}
    tuned, tables = (None, None) if args.no_ensemble_autotune else tune_ensemble_orders(ens, orders, stream)
    # how the two orders' batches are advanced: each batch on its own
    # stream (they overlap on the GPU), or together by dgswe_step_pair
    # on one stream (per stage the p = 1 stage with the p = 2
    # post-processing in one launch, then the p = 2 right-hand side; or
    # the p = 2 post-processing, then one launch of both orders' stage
    # work), with one workgroup per chunk or persistent workgroups
    modes = {}
    for name, kw, env in (("two_streams", dict(fused=False), None),
                          ("pair", dict(fused=True), None),
                          ("pair_both_stages_one_launch", dict(fused=True), "DGSWE_PAIR_SPLIT"),
                          ("pair_persistent", dict(fused=True, persistent=2), None)):
        if env:
            os.environ[env] = "0"
        try:
            modes[name] = measure_ensemble(ens, args.steps, args.warmup, stream, profile, tuned=defaults,
                                           orders=orders, **kw)
        finally:
            if env:
                del os.environ[env]
        log(f"ensemble {name}: {modes[name]['ms_per_step']:.3f} ms per step")
    if tuned is not None:
        modes["pair_autotuned"] = measure_ensemble(ens, args.steps, args.warmup, stream, profile, tuned=tuned,
                                                   orders=orders, fused=True)
        log(f"ensemble pair_autotuned: {modes['pair_autotuned']['ms_per_step']:.3f} ms per step")
    variants["batched"] = dict(modes["pair"], mode="pair", autotune=tables,
                               modes_ms_per_step={k: v["ms_per_step"] for k, v in modes.items()})
    variants["batched_modes"] = {k: v for k, v in modes.items() if k != "pair"}
    variants["batched_p1_only"] = measure_ensemble(ens, args.steps, args.warmup, stream, profile, tuned=defaults,
                                                   orders=[1] * len(ens))
    del ens
    return variants


def copy_probe(dev):
    """a plain device copy of 2 GiB, three times: the reference for the HBM
    counters"""
    import torch
    n = 2 * 1024 ** 3 // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copy probe: 3 x (read 2 GiB + write 2 GiB)")
    del src, dst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of --steps steps each for the headline and mixed lines (the median is reported)")
    ap.add_argument("--elems", type=int, default=4_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision variant")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched ensemble variant")
    ap.add_argument("--no-p2", action="store_true", help="skip the p = 2 variants")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--no-graphs", action="store_true", help="skip the step-graph launch-cost run")
    ap.add_argument("--no-rk", action="store_true", help="skip the time-stepper and Roe-flux variants")
    ap.add_argument("--serving-requests", type=int, default=60)
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64",
                    help="precision of the headline run (fp64 is the metric's)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of 2 GiB (3 times) to calibrate HBM counters")
    ap.add_argument("--summarize-pmc", metavar="DIR",
                    help="no GPU run: turn rocprofv3 FETCH_SIZE/WRITE_SIZE runs under DIR into the traffic record")
    ap.add_argument("--kernel-trace", help="with --summarize-pmc: rocprofv3 kernel_trace.csv of the 4M run")
    ap.add_argument("--summary-md", help="with --summarize-pmc: write a markdown summary here")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="no GPU run: tabulate the issue/wait/cache counter runs c1, c2 under DIR")
    ap.add_argument("--counter-kernels", default="k_stage", help="with --summarize-counters: kernels to tabulate")
    ap.add_argument("--ensemble-kernel-trace", help="with --summarize-pmc: kernel_trace.csv of an --only-batched run")
    ap.add_argument("--no-ensemble-autotune", action="store_true",
                    help="skip the ensemble's autotuned mode (the profiles measure the default launch parameters)")
    ap.add_argument("--only-batched", action="store_true",
                    help="run only the batched ensemble variants (for the ensemble's profiles); prints them")
    args = ap.parse_args()
    if args.summarize_counters:
        ks = tuple(args.counter_kernels.split(","))
        title = ("k_stage (p = 1)" if ks == ("k_stage",) else " and ".join(ks) + " (p = 2)") + \
            " on the 4M-triangle hurricane workload: issue, wait and cache counters"
        summarize_counters(args.summarize_counters, ks, title, args.summary_md)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc, args.kernel_trace, args.summary_md, args.ensemble_kernel_trace)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; a multi-GPU run (domain "
                                   "decomposition with a per-stage halo exchange) is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2508_21208_amd import workloads as W

    if args.only_batched:
        torch.cuda.init()
        dev = torch.device("cuda:0")
        out = {"variants": measure_batched(args, torch.cuda.current_stream(dev), not args.no_profile),
               "steps": args.steps, "warmup": args.warmup}
        if args.copy_probe:
            copy_probe(dev)
        print(json.dumps(out), flush=True)
        return
    t0 = time.perf_counter()
    wl = W.cfg_hurricane(n_target=args.elems)
    log(f"mesh {wl.mesh.n_elems} elements, {wl.mesh.n_nodes} nodes in {time.perf_counter() - t0:.1f} s")
    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    profile = not args.no_profile
    kept = {}
    elapsed, info, kernels, d, runs = measure(wl, args.precision, args.steps, args.warmup, stream, profile,
                                              keep=None if args.no_mixed else kept, repeats=args.repeats)
    ne, ned, nn = info["n_elems"], info["n_edges"], info["n_nodes"]
    rate = ne * 2 * args.steps / elapsed
    roof = roofline(kernels, ne, ned, nn, args.precision)
    if kernels:
        log(f"{args.precision} kernels: " + json.dumps(kernels))
    variants = {}
    other = "mixed" if args.precision == "fp64" else "fp64"
    if not args.no_mixed:
        kept2 = {}
        el2, _, k2, d2, runs2 = measure(wl, other, args.steps, args.warmup, stream, profile, keep=kept2,
                                        repeats=args.repeats)
        err = mixed_error(kept2["state"], kept["state"]) if other == "mixed" else \
            mixed_error(kept["state"], kept2["state"])
        kept.clear()
        kept2.clear()
        n_cmp = kept2.get("steps")
        log(f"mixed vs fp64 GPU after {n_cmp} steps: " + json.dumps(err))
        variants[other] = {"value": ne * 2 * args.steps / el2, "unit": "elem-stage/s",
                           "ms_per_step": 1e3 * el2 / args.steps, "runs_ms_per_step": [1e3 * r / args.steps for r in runs2],
                           "roofline": roofline(k2, ne, ned, nn, other),
                           "kernels": k2, "t_end": d2["t"], "t_end_" + args.precision: d["t"],
                           "error_vs_fp64_gpu": dict(err, steps=n_cmp),
                           "error_vs_oracle": mixed_error_vs_oracle(stream)}
        if k2:
            log(f"{other} kernels: " + json.dumps(k2))
    rt = measure_host_roundtrip(wl, args.steps, stream)
    variants["host_roundtrip"] = {
        "value": ne * 2 * args.steps / rt["total_s"], "unit": "elem-stage/s", "precision": "fp64",
        "note": "state uploaded from and read back to host memory through the C ABI, inside the timed region",
        **{k: round(v, 4) for k, v in rt.items()}}
    log("host round trip: " + json.dumps(variants["host_roundtrip"]))
    if not args.no_p2:
        for prec in ("fp64", "mixed"):
            el4, _, k4, d4, _ = measure(wl, prec, args.steps, args.warmup, stream, profile, order=2)
            variants["p2_" + prec] = {"value": ne * 2 * args.steps / el4, "unit": "elem-stage/s", "p": 2,
                                      "precision": prec, "ms_per_step": 1e3 * el4 / args.steps,
                                      "roofline": roofline(k4, ne, ned, nn, prec),
                                      "kernels": k4, "t_end": d4["t"]}
            if k4:
                log(f"p2 {prec} kernels: " + json.dumps(k4))
    if not args.no_rk:
        # time steppers at their SSP limits: model seconds per wall second
        # is what a larger stable step buys
        from paper_2508_21208_amd.dgswe import DgsweError
        # "sources": Coriolis (f at 30 N) and heavy rain (50 mm/h) added
        for name, extra, ns, fx in (("ssprk33", dict(rk=33, cfl=0.2), 3, {}), ("ssprk52", dict(rk=52, cfl=0.8), 5, {}),
                                    ("roe", dict(flux=1), 2, {}), ("vertex_limiter", dict(limiter=2), 2, {}),
                                    ("sources", {}, 2, dict(coriolis=7.29e-5, rain=50e-3 / 3600))):
            try:
                el5, _, k5, d5, _ = measure(wl, "fp64", args.steps, args.warmup, stream, profile, extra=extra,
                                            forcing=fx)
                variants[name] = {
                    "value": ne * ns * args.steps / el5, "unit": "elem-stage/s", **extra, **fx, "stages": ns,
                    "ms_per_step": 1e3 * el5 / args.steps, "dt_last": d5["dt_last"],
                    "model_s_per_wall_s": d5["dt_last"] / (el5 / args.steps),
                    "model_s_per_wall_s_default": d["dt_last"] / (elapsed / args.steps),
                    "roofline": roofline(k5, ne, ned, nn, "fp64")}
                if k5:
                    log(f"{name} kernels: " + json.dumps(k5))
            except DgsweError as ex:
                variants[name] = {"error": str(ex), **extra}
    if not args.no_batched:
        variants.update(measure_batched(args, stream, profile))

    if not args.no_graphs:
        variants["graphs_small_mesh"] = measure_graphs(stream)
        variants["autotune"] = measure_autotune(stream)
    if not args.no_serving:
        hint = variants.get("mixed", {}).get("value") or 1.2e10
        variants["serving"] = measure_serving(args.serving_requests, hint, stream)

    if args.copy_probe:
        copy_probe(dev)

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
        "timing": {"repeats": args.repeats, "statistic": "median",
                   "runs_ms_per_step": [1e3 * r / args.steps for r in runs]},
        "paper_context": PAPER_CONTEXT,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
