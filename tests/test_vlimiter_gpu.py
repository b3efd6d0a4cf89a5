"""Vertex-based limiter (dgswe_params.limiter = 2, p = 1) on the GPU.

Bar: FP64 relative L2 <= 1e-12 per variable against the oracle after N
steps (smooth case and the wet/dry coastal case), and on the
post-processing of a stored state alone; mixed precision within the
elevation bar of the default limiter; pool members and graph replays
equal plain single-mesh runs bitwise (the node-to-element incidence is
shifted into each member's ranges)."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Pool, Solver

from _cases import coastal_small, rel_l2, say

pytestmark = pytest.mark.gpu

TOL = 1e-12


def run_both(wl, steps, precision=0, extra=None):
    p = dict(wl.params, limiter=2, **(extra or {}))
    say(f"{wl.name}: GPU vertex limiter precision={precision} {steps} steps, ne={wl.mesh.n_elems}")
    s = Solver(wl.mesh, dict(p, precision=precision), wl.forcing)
    s.set_state(wl.w0, 0.0, wl.postprocess_initial)
    s.step(steps)
    wg = s.state()
    dg = s.diagnostics()
    s.close()
    o = Oracle(wl.mesh, p, wl.forcing)
    o.set_state(wl.w0, 0.0, wl.postprocess_initial)
    o.step(steps)
    return wg, dg, o.state(), o


def test_vlimiter_postprocess_only():
    # a rough state: the read-back applies the limiter to the stored state
    wl = coastal_small()
    rng = np.random.default_rng(3)
    w = wl.w0.copy()
    w[:, 1:] += rng.normal(scale=0.05, size=w[:, 1:].shape)
    p = dict(wl.params, limiter=2)
    s = Solver(wl.mesh, p, wl.forcing)
    s.set_state(w, 0.0, True)
    wg = s.state()
    s.close()
    o = Oracle(wl.mesh, p, wl.forcing)
    wo = o.postprocess(w)
    err = rel_l2(wg, wo)
    say(f"post-processing only: rel L2 {err}")
    assert max(err) <= TOL, err
    assert not np.array_equal(wo, w)


def test_vlimiter_gaussian_hump():
    wg, dg, wo, o = run_both(W.cfg_gaussian_1600(), 200)
    err = rel_l2(wg, wo)
    say(f"rel L2 {err}")
    assert max(err) <= TOL, err
    assert dg["steps"] == o.steps


def test_vlimiter_coastal_wetdry_tide_hurricane():
    wg, dg, wo, o = run_both(coastal_small(), 100)
    err = rel_l2(wg, wo)
    say(f"rel L2 {err}")
    assert max(err) <= TOL, err
    do = o.diagnostics(wo)
    assert dg["n_wet"] == do["n_wet"] and dg["n_dry"] > 0


def test_vlimiter_ssprk33():
    wg, dg, wo, o = run_both(W.cfg_gaussian_1600(), 60, extra=dict(rk=33))
    err = rel_l2(wg, wo)
    assert max(err) <= TOL, err


def test_vlimiter_mixed_accuracy():
    wg, dg, wo, o = run_both(coastal_small(), 100, precision=DGSWE_MIXED)
    V = np.array([[1, -1, -1], [1, 1, -1], [1, 0, 2]], float)
    ez = np.abs(V @ (wg[0] - wo[0])).max()
    say(f"vertex limiter mixed: vertex elevation error {ez:.3e} m")
    assert ez <= 1e-4


def test_vlimiter_pool_members_and_graphs_equal_solo():
    params = W.default_params(dt_max=0.3, limiter=2)
    ms = [W.coastal_mesh(n, W.BASE_SEED + 600 + i, hmin=1000.0, hmax=15000.0) for i, n in enumerate((4000, 8000, 3000))]
    fs = [W.default_forcing(manning_n=0.025, **W.m2_tide(1.0), **W.holland_track(m, offshore=120e3)) for m in ms]
    ws = [W.coastal_initial_state(m) for m in ms]
    pool = Pool(20000, 4, params)
    pool.use_graphs(6)
    x = pool.add(ms[0], forcing=fs[0], w=ws[0], postprocess=True)
    y = pool.add(ms[1], forcing=fs[1], w=ws[1], postprocess=True)
    say("vertex limiter pool: two members, 12 steps (graphs)")
    pool.step(12)
    wx, _ = pool.state(x)
    pool.remove(x)
    z = pool.add(ms[2], forcing=fs[2], w=ws[2], postprocess=True)  # into x's freed ranges
    say("x left, z joined: 18 steps")
    pool.step(18)
    wy, _ = pool.state(y)
    wz, _ = pool.state(z)
    pool.close()
    for i, steps, got in ((0, 12, wx), (1, 30, wy), (2, 18, wz)):
        s = Solver(ms[i], params, fs[i])
        s.set_state(ws[i], 0.0, True)
        s.step(steps)
        assert np.array_equal(s.state(), got), i
        s.close()
