"""Schemes whose last stage runs at t + dt reuse that stage's nodal forcing
for the next step's first stage (the same time, bit for bit): results equal
the path that evaluates the forcing at every stage
(DGSWE_FORCING_EVERY_STAGE=1) bitwise, also across a forcing change
between step calls and under step graphs."""
import os

import numpy as np
import pytest

from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Solver

from _cases import coastal_small, say

pytestmark = pytest.mark.gpu


def run(wl, params, every, graphs=0):
    if every:
        os.environ["DGSWE_FORCING_EVERY_STAGE"] = "1"
    try:
        s = Solver(wl.mesh, params, wl.forcing)
    finally:
        os.environ.pop("DGSWE_FORCING_EVERY_STAGE", None)
    if graphs:
        s.use_graphs(graphs)
    w0 = wl.w0
    if params.get("p", 1) == 2:
        w0 = np.concatenate([wl.w0, np.zeros_like(wl.w0)], axis=1)
    s.set_state(w0, 0.0, True)
    s.step(7)
    s.step(6)
    w1 = s.state()
    # a different storm from here on: the reused forcing must be dropped
    f2 = dict(wl.forcing, **W.holland_track(wl.mesh, speed=8.0, heading=0.3))
    s.set_forcing(f2)
    s.step(9)
    w2 = s.state()
    s.close()
    return w1, w2


@pytest.mark.parametrize("extra", [dict(), dict(precision=DGSWE_MIXED), dict(p=2, cfl=0.1), dict(rk=52, cfl=0.5),
                                   dict(rk=33)])
def test_reused_forcing_equals_every_stage(extra):
    wl = coastal_small()
    params = dict(wl.params, **extra)
    say(f"forcing reuse {extra}")
    a = run(wl, params, False)
    b = run(wl, params, True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_reused_forcing_under_graphs():
    wl = coastal_small()
    a = run(wl, wl.params, False, graphs=6)
    b = run(wl, wl.params, True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
