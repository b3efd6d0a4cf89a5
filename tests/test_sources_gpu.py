"""Coriolis and rain sources (dgswe_forcing.coriolis, .rain) on the GPU
against the oracle: FP64 relative L2 <= 1e-12 per variable for p = 1 and
p = 2, equal wet/dry counts; mixed precision within the elevation bar of
the default configuration."""

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Solver

from _cases import coastal_small, rel_l2, say

pytestmark = pytest.mark.gpu

TOL = 1e-12


def run_both(wl, steps, sources, order=1, precision=0, extra=None):
    p = dict(wl.params, **(extra or {}))
    forcing = dict(wl.forcing, **sources)
    w0 = wl.w0
    if order == 2:
        w0 = np.zeros((3, 6, wl.w0.shape[2]))
        w0[:, :3] = wl.w0
        p.update(p=2)
    say(f"{wl.name}: GPU sources {sources} p={order} precision={precision} {steps} steps")
    s = Solver(wl.mesh, dict(p, precision=precision), forcing)
    s.set_state(w0, 0.0, wl.postprocess_initial)
    s.step(steps)
    wg = s.state()
    dg = s.diagnostics()
    s.close()
    o = Oracle(wl.mesh, p, forcing, order=order)
    o.set_state(w0, 0.0, wl.postprocess_initial)
    o.step(steps)
    return wg, dg, o.state(), o


@pytest.mark.parametrize("order", [1, 2])
def test_coriolis_gaussian_hump(order):
    wg, dg, wo, o = run_both(W.cfg_gaussian_1600(), 150 if order == 1 else 60, dict(coriolis=1.0e-3), order,
                             extra=None if order == 1 else dict(cfl=0.1))
    err = rel_l2(wg, wo)
    say(f"rel L2 {err}")
    assert max(err) <= TOL, err
    assert dg["steps"] == o.steps


@pytest.mark.parametrize("order", [1, 2])
def test_coriolis_and_rain_coastal_wetdry(order):
    # heavy rain (0.1 mm/s) on the coastal case: dry cells take water and
    # cross the wet threshold during the run
    wg, dg, wo, o = run_both(coastal_small(), 100 if order == 1 else 40, dict(coriolis=7.0e-5, rain=1.0e-4),
                             order, extra=None if order == 1 else dict(cfl=0.1))
    err = rel_l2(wg, wo)
    say(f"rel L2 {err}")
    assert max(err) <= TOL, err
    do = o.diagnostics(wo)
    assert dg["n_wet"] == do["n_wet"] and dg["n_dry"] == do["n_dry"]


def test_rain_mass_budget_closed_basin():
    # a closed basin at rest gains exactly R * t * area of water
    m = W.rect_mesh(40, 30, 8000.0, 6000.0, hb=5.0)
    R, dt, n = 2.0e-5, 4.0, 50
    s = Solver(m, W.default_params(dt_fixed=dt), W.default_forcing(rain=R))
    s.set_state(np.zeros((3, 3, m.n_elems)), 0.0, False)
    s.step(n)
    w = s.state()
    s.close()
    say(f"rain: mean elevation {w[0, 0].mean()} vs {R * dt * n}")
    assert np.allclose(w[0, 0], R * dt * n, rtol=1e-12)
    assert np.abs(w[1:]).max() < 1e-12


def test_sources_mixed_accuracy():
    wg, dg, wo, o = run_both(coastal_small(), 100, dict(coriolis=7.0e-5, rain=1.0e-4), precision=DGSWE_MIXED)
    V = np.array([[1, -1, -1], [1, 1, -1], [1, 0, 2]], float)
    ez = np.abs(V @ (wg[0] - wo[0])).max()
    say(f"sources mixed: vertex elevation error {ez:.3e} m")
    assert ez <= 1e-4
