"""SSP Runge-Kutta variants (dgswe_params.rk) on the GPU against the oracle.

Bar as for the default scheme: FP64 relative L2 <= 1e-12 per variable after
N steps, same step counts and model time; mixed precision within the
accuracy bar of the default scheme.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Solver

from _cases import coastal_small, rel_l2, say

pytestmark = pytest.mark.gpu

TOL = 1e-12


def run_both(wl, steps, params, order=1):
    p = dict(wl.params, **params)
    w0 = wl.w0
    if order == 2:
        w0 = np.zeros((3, 6, wl.w0.shape[2]))
        w0[:, :3] = wl.w0
        p.update(p=2)
    say(f"{wl.name}: GPU rk={p['rk']} p={order} {steps} steps")
    s = Solver(wl.mesh, p, wl.forcing)
    s.set_state(w0, 0.0, wl.postprocess_initial)
    s.step(steps)
    wg = s.state()
    dg = s.diagnostics()
    s.close()
    o = Oracle(wl.mesh, p, wl.forcing, order=order)
    o.set_state(w0, 0.0, wl.postprocess_initial)
    o.step(steps)
    wo = o.state()
    return wg, dg, wo, o


@pytest.mark.parametrize("rk,cfl", [(33, 0.2), (32, 0.4), (42, 0.6), (52, 0.8)])
def test_schemes_gaussian_hump(rk, cfl):
    wg, dg, wo, o = run_both(W.cfg_gaussian_1600(), 100, dict(rk=rk, cfl=cfl))
    err = rel_l2(wg, wo)
    say(f"rel L2 {err}")
    assert max(err) <= TOL, err
    assert dg["steps"] == o.steps and dg["t"] == pytest.approx(o.t, rel=1e-12)


@pytest.mark.parametrize("rk", [33, 52])
def test_schemes_coastal_wetdry_tide_hurricane(rk):
    wl = coastal_small()
    wg, dg, wo, o = run_both(wl, 60, dict(rk=rk, dt_max=0.3))
    err = rel_l2(wg, wo)
    say(f"rel L2 {err}")
    assert max(err) <= TOL, err
    do = o.diagnostics(wo)
    assert dg["n_wet"] == do["n_wet"] and dg["steps"] == o.steps


def test_ssprk33_p2():
    wg, dg, wo, o = run_both(W.cfg_gaussian_1600(), 60, dict(rk=33, cfl=0.1), order=2)
    err = rel_l2(wg, wo)
    say(f"rel L2 {err}")
    assert max(err) <= TOL, err


def test_ssprk52_mixed_accuracy():
    wl = coastal_small()
    p = dict(wl.params, rk=52, dt_max=0.3)
    s = Solver(wl.mesh, dict(p, precision=DGSWE_MIXED), wl.forcing)
    s.set_state(wl.w0, 0.0, True)
    s.step(60)
    wg = s.state()
    s.close()
    o = Oracle(wl.mesh, p, wl.forcing)
    o.set_state(wl.w0, 0.0, True)
    o.step(60)
    wo = o.state()
    V = np.array([[1, -1, -1], [1, 1, -1], [1, 0, 2]], float)
    ez = np.abs(V @ (wg[0] - wo[0])).max()
    say(f"SSPRK(5,2) mixed: vertex elevation error {ez:.3e} m")
    assert ez <= 1e-4
