"""The numerical variants at the 600k-triangle coastal size (graded mesh,
M2 tide, wet/dry), 20 steps, FP64 against the oracle: relative L2 <= 1e-12
per variable and equal wet counts: Roe flux, vertex-based limiter,
SSPRK(3,3), SSPRK(5,2) and Coriolis + rain; at p = 2 (10 steps) Roe and
SSPRK(3,3) with Coriolis + rain."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_21208_amd.dgswe import Solver

from _cases import coastal_600k, rel_l2, say

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.mark.parametrize("params,sources", [(dict(flux=1), {}), (dict(limiter=2), {}), (dict(rk=33), {}),
                                            (dict(rk=52, cfl=0.5), {}), ({}, dict(coriolis=6.0e-5, rain=2.0e-5))],
                         ids=["roe", "vertex_limiter", "ssprk33", "ssprk52", "coriolis_rain"])
def test_variant_600k(params, sources):
    wl = coastal_600k()
    p = dict(wl.params, **params)
    f = dict(wl.forcing, **sources)
    say(f"600k variant {params} {sources}: GPU 20 steps")
    s = Solver(wl.mesh, p, f)
    s.set_state(wl.w0, 0.0, wl.postprocess_initial)
    s.step(20)
    wg = s.state()
    dg = s.diagnostics()
    s.close()
    say("oracle 20 steps")
    o = Oracle(wl.mesh, p, f)
    o.set_state(wl.w0, 0.0, wl.postprocess_initial)
    o.step(20)
    wo = o.state()
    err = rel_l2(wg, wo)
    say(f"rel L2 {err}")
    assert max(err) <= TOL, err
    assert dg["n_wet"] == o.diagnostics(wo)["n_wet"]


@pytest.mark.parametrize("params,sources", [(dict(flux=1), {}), (dict(rk=33), dict(coriolis=6.0e-5, rain=2.0e-5))],
                         ids=["p2_roe", "p2_ssprk33_coriolis_rain"])
def test_p2_variant_600k(params, sources):
    wl = coastal_600k()
    p = dict(wl.params, p=2, cfl=0.1, **params)
    f = dict(wl.forcing, **sources)
    w0 = np.concatenate([wl.w0, np.zeros_like(wl.w0)], axis=1)
    say(f"600k p=2 variant {params} {sources}: GPU 10 steps")
    s = Solver(wl.mesh, p, f)
    s.set_state(w0, 0.0, wl.postprocess_initial)
    s.step(10)
    wg = s.state()
    dg = s.diagnostics()
    s.close()
    say("p=2 oracle 10 steps")
    o = Oracle(wl.mesh, p, f, order=2)
    o.set_state(w0, 0.0, wl.postprocess_initial)
    o.step(10)
    wo = o.state()
    err = rel_l2(wg, wo)
    say(f"rel L2 {err}")
    assert max(err) <= TOL, err
    assert dg["n_wet"] == o.diagnostics(wo)["n_wet"]
