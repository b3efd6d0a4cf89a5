"""Roe flux (dgswe_params.flux = 1) on the GPU against the oracle: FP64
relative L2 <= 1e-12 per variable, equal step counts and wet/dry counts;
mixed precision within the accuracy bar of the default flux."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Solver

from _cases import coastal_small, rel_l2, say

pytestmark = pytest.mark.gpu

TOL = 1e-12


def run_both(wl, steps, params, order=1, precision=0):
    p = dict(wl.params, flux=1, **params)
    w0 = wl.w0
    if order == 2:
        w0 = np.zeros((3, 6, wl.w0.shape[2]))
        w0[:, :3] = wl.w0
        p.update(p=2)
    say(f"{wl.name}: GPU Roe p={order} precision={precision} {steps} steps")
    s = Solver(wl.mesh, dict(p, precision=precision), wl.forcing)
    s.set_state(w0, 0.0, wl.postprocess_initial)
    s.step(steps)
    wg = s.state()
    dg = s.diagnostics()
    s.close()
    o = Oracle(wl.mesh, p, wl.forcing, order=order)
    o.set_state(w0, 0.0, wl.postprocess_initial)
    o.step(steps)
    return wg, dg, o.state(), o


def test_roe_gaussian_hump():
    wg, dg, wo, o = run_both(W.cfg_gaussian_1600(), 200, {})
    err = rel_l2(wg, wo)
    say(f"rel L2 {err}")
    assert max(err) <= TOL, err
    assert dg["steps"] == o.steps


def test_roe_coastal_wetdry_tide_hurricane():
    wg, dg, wo, o = run_both(coastal_small(), 100, {})
    err = rel_l2(wg, wo)
    say(f"rel L2 {err}")
    assert max(err) <= TOL, err
    do = o.diagnostics(wo)
    assert dg["n_wet"] == do["n_wet"] and dg["n_dry"] > 0


def test_roe_p2_and_ssprk33():
    wg, dg, wo, o = run_both(W.cfg_gaussian_1600(), 60, dict(cfl=0.1, rk=33), order=2)
    err = rel_l2(wg, wo)
    say(f"rel L2 {err}")
    assert max(err) <= TOL, err


def test_roe_mixed_accuracy():
    wg, dg, wo, o = run_both(coastal_small(), 100, {}, precision=DGSWE_MIXED)
    V = np.array([[1, -1, -1], [1, 1, -1], [1, 0, 2]], float)
    ez = np.abs(V @ (wg[0] - wo[0])).max()
    say(f"Roe mixed: vertex elevation error {ez:.3e} m")
    assert ez <= 1e-4
