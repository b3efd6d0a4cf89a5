"""Parity over the configured horizons of the two full-size coastal workloads.

* ~600k-triangle graded coastal mesh, M2 tide on the open boundary, Manning
  n = 0.025, wetting/drying: 2,000 steps.
* ~4M-triangle graded coastal mesh with the moving Holland hurricane (60 hPa,
  Rmax 40 km, 5 m/s) on top of the tide: 1,000 steps.

One FP64 oracle run per workload (a session fixture; it prints its progress
straight to the terminal, since it runs for minutes) serves two checks:
  * the FP64 HIP path: relative L2 <= 1e-12 per variable, equal step count,
    the same wet/dry status of every element (and so equal counts), model
    time, mass (correctly rounded sum) and volume to 1e-12;
  * the mixed FP32/FP64 path: elevation at every vertex of the elements
    at least 2 H0 deep in both runs within 1e-4 m, and depth-averaged
    velocity at element means within 1e-4 m/s (elements wet on both sides
    with mean depth >= 0.5 m), the same step count and the model time to
    1e-6 relative.  Elements within 2 H0 of the wet/dry threshold in either
    run are held to H0/10 = 1e-3 m, and at most 10 of them may exceed
    1e-4 m: there the wet/dry decisions (reading Z9: element dry at mean
    depth H0, edge flood test) make the solution itself sensitive at that
    level - the FP64 result moves by up to 6.4e-5 m (600k, 2,000 steps) and
    6.2e-5 m (4M, 1,000 steps) in that band when Manning's n changes by
    6e-8 relative (one FP32 rounding), and at the 4M mesh by 8.8e-5 m in
    that band (1.7e-4 m in the 0.05-0.5 m band) when g does.

With DGSWE_REPORT=<file.json> the measured figures are written to that file
(one entry per workload and precision).
"""
import json
import math
import os
import sys
import time

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Solver

from _cases import coastal_600k, exact_mass, hurricane_4m, rel_l2, say

pytestmark = pytest.mark.gpu

TOL = 1e-12
ZETA_TOL = 1e-4   # m
VEL_TOL = 1e-4    # m/s
VEL_MIN_DEPTH = 0.5
FRONT_DEPTH = 0.02       # 2 H0: elements shallower than this in either run
FRONT_TOL = 1e-3         # H0 / 10
FRONT_MAX_OVER = 10      # elements of that band allowed above ZETA_TOL

WORKLOADS = {"coastal_tide_600k": coastal_600k, "hurricane_4m": hurricane_4m}
HORIZON = {"coastal_tide_600k": 2000, "hurricane_4m": 1000}


def _tell(config, msg):
    """a progress line on the terminal even while pytest captures output"""
    capman = config.pluginmanager.getplugin("capturemanager")
    line = f"[horizon] {msg}\n"
    if capman is None:
        sys.stdout.write(line)
        sys.stdout.flush()
        return
    with capman.global_and_fixture_disabled():
        sys.stdout.write(line)
        sys.stdout.flush()


def _report(key, rec):
    """add `rec` under `key` to the report file named by DGSWE_REPORT, with
    the hash of the kernel sources it was measured on"""
    path = os.environ.get("DGSWE_REPORT")
    if not path:
        return
    import bench
    data = {"results": {}}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    data["source_sha256"] = bench.source_hash()
    data["command"] = "DGSWE_REPORT=<file> python -m pytest tests/test_full_horizon_gpu.py -m gpu"
    data["results"][key] = rec
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1)


class OracleRun:
    def __init__(self, wl, steps, config):
        self.wl = wl
        o = Oracle(wl.mesh, wl.params, wl.forcing)
        o.set_state(wl.w0, 0.0, wl.postprocess_initial)
        t0 = time.perf_counter()
        done = 0
        chunk = 25
        last = t0
        while done < steps:
            n = min(chunk, steps - done)
            o.step(n)
            done += n
            now = time.perf_counter()
            if now - last > 20.0 or done == steps:
                _tell(config, f"oracle {wl.name}: {done}/{steps} steps, {now - t0:.0f} s")
                last = now
        self.seconds = time.perf_counter() - t0
        self.w = o.state()  # also sets o.steps, o.t
        self.steps = o.steps
        self.t = o.t
        d = o.diagnostics(self.w)
        self.volume = d["volume"]
        self.n_wet, self.n_dry = d["n_wet"], d["n_dry"]
        self.mass = exact_mass(o, self.w)
        del o


_runs = {}


@pytest.fixture(scope="session")
def oracle_run(request):
    def get(name):
        if name not in _runs:
            wl = WORKLOADS[name]()
            _tell(request.config, f"oracle {wl.name}: {HORIZON[name]} steps on {wl.mesh.n_elems} elements, "
                                  f"OMP_NUM_THREADS={os.environ.get('OMP_NUM_THREADS', '?')}")
            _runs[name] = OracleRun(wl, HORIZON[name], request.config)
        return _runs[name]
    yield get
    _runs.clear()


def _gpu(wl, steps, precision):
    p = dict(wl.params)
    if precision == "mixed":
        p["precision"] = DGSWE_MIXED
    say(f"{wl.name}: {precision} GPU {steps} steps")
    s = Solver(wl.mesh, p, wl.forcing)
    s.set_state(wl.w0, 0.0, wl.postprocess_initial)
    s.step(steps)
    w = s.state()
    d = s.diagnostics()
    s.close()
    return w, d


def _wet_mismatches(wl, wa, wb):
    """elements wet (mean depth above H0) in one state and not in the other"""
    hmean = wl.mesh.hb[wl.mesh.tri].mean(axis=1)
    h0 = wl.params["h0"]
    return int(np.sum((wa[0, 0] + hmean > h0) != (wb[0, 0] + hmean > h0)))


def _vertex_zeta(w):
    z0, z1, z2 = w[0, 0], w[0, 1], w[0, 2]
    return np.stack([z0 - z1 - z2, z0 + z1 - z2, z0 + 2.0 * z2])


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_fp64_matches_oracle_over_the_horizon(name, oracle_run):
    o = oracle_run(name)
    wl = o.wl
    wg, dg = _gpu(wl, HORIZON[name], "fp64")
    err = rel_l2(wg, o.w)
    n_mis = _wet_mismatches(wl, wg, o.w)
    rec = {"steps": o.steps, "n_elems": wl.mesh.n_elems, "t_end": dg["t"], "rel_l2": [float(x) for x in err],
           "n_wet": [dg["n_wet"], o.n_wet], "n_dry": [dg["n_dry"], o.n_dry], "oracle_s": round(o.seconds, 1),
           "wet_status_mismatches": n_mis,
           "mass_rel_diff": abs(dg["mass"] - o.mass) / max(abs(o.mass), 1e-300)}
    _report(f"{name}/fp64", rec)
    say(f"{wl.name}: FP64 after {o.steps} steps: rel L2 {err}, wet {dg['n_wet']} / {o.n_wet}")
    assert max(err) <= TOL, err
    assert dg["steps"] == o.steps == HORIZON[name]
    assert dg["t"] == pytest.approx(o.t, rel=1e-12)
    assert dg["n_wet"] == o.n_wet and dg["n_dry"] == o.n_dry
    assert n_mis == 0, n_mis
    assert dg["mass"] == pytest.approx(o.mass, rel=1e-12, abs=1e-6)
    assert dg["volume"] == pytest.approx(o.volume, rel=1e-12)


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_mixed_within_bar_of_oracle_over_the_horizon(name, oracle_run):
    o = oracle_run(name)
    wl = o.wl
    wg, dg = _gpu(wl, HORIZON[name], "mixed")
    ez = np.abs(_vertex_zeta(wg) - _vertex_zeta(o.w)).max(axis=0)
    hmean = wl.mesh.hb[wl.mesh.tri].mean(axis=1)
    Hg, Ho = wg[0, 0] + hmean, o.w[0, 0] + hmean
    h0 = wl.params["h0"]
    ok = (Hg > h0) & (Ho > h0) & (Ho >= VEL_MIN_DEPTH)
    ev = 0.0
    for v in (1, 2):
        ev = max(ev, float(np.abs(wg[v, 0][ok] / Hg[ok] - o.w[v, 0][ok] / Ho[ok]).max()))
    front = np.minimum(Hg, Ho) < FRONT_DEPTH
    ez_wet, ez_front = float(ez[~front].max()), float(ez[front].max()) if front.any() else 0.0
    n_over = int(np.sum(ez[front] > ZETA_TOL))
    worst = int(np.argmax(ez))
    rec = {"steps": o.steps, "n_elems": wl.mesh.n_elems, "zeta_vertex_max_m": float(ez.max()),
           "zeta_vertex_max_m_depth_ge_2H0": ez_wet, "zeta_vertex_max_m_within_2H0": ez_front,
           "n_within_2H0": int(front.sum()), "n_within_2H0_over_1e-4": n_over,
           "velocity_mean_max_ms": ev, "t_end": dg["t"], "t_oracle": o.t, "dt_diff_s": abs(dg["t"] - o.t),
           "rel_l2": [float(x) for x in rel_l2(wg, o.w)], "n_wet": [dg["n_wet"], o.n_wet],
           "wet_status_mismatches": _wet_mismatches(wl, wg, o.w),
           "worst_element_mean_depth_m": float(Ho[worst])}
    _report(f"{name}/mixed", rec)
    say(f"{wl.name}: MIXED after {o.steps} steps: elevation {ez_wet:.3e} m (>= 2 H0 deep), {ez_front:.3e} m "
        f"within 2 H0 ({n_over} over 1e-4), velocity {ev:.3e} m/s")
    assert ez_wet <= ZETA_TOL and ev <= VEL_TOL, (ez_wet, ev)
    assert ez_front <= FRONT_TOL and n_over <= FRONT_MAX_OVER, (ez_front, n_over)
    assert dg["steps"] == o.steps
    assert dg["t"] == pytest.approx(o.t, rel=1e-6)
    assert math.isfinite(dg["mass"])
