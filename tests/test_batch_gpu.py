"""A batch of independent meshes advanced by one stage launch per stage.

Every member follows exactly the arithmetic of its mesh alone: its state,
time, dt, step count and diagnostics after N steps equal its solo run bit
for bit, in FP64 and in mixed precision; an error in one member (a NaN)
stops that member only; re-setting one member's state mid-run leaves the
others untouched.
"""
import math

import numpy as np
import pytest

from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Batch, DgsweError, Solver, dgswe_read_state

from _cases import coastal_small, say

pytestmark = pytest.mark.gpu


def members():
    """mixed sizes and forcings: tiny walled boxes, the Gaussian hump, two
    coastal meshes with tide / hurricane / static wind and per-element
    Manning n"""
    out = []
    wl = W.cfg_gaussian_1600()
    out.append((wl.mesh, wl.w0, wl.params, wl.forcing, wl.postprocess_initial))
    for nx, ny in ((1, 1), (17, 3)):
        m = W.rect_mesh(nx, ny, 100.0 * nx, 100.0 * ny, hb=lambda x, y: 5.0 + 0.001 * x)
        zn = 0.05 * np.sin(m.xy[:, 0] / 150.0) + 0.02 * np.cos(m.xy[:, 1] / 90.0)
        out.append((m, W.state_from_nodal(m.tri, zn), W.default_params(), W.default_forcing(manning_n=0.02), False))
    wl = coastal_small()
    out.append((wl.mesh, wl.w0, wl.params, wl.forcing, True))
    m = W.coastal_mesh(12000, W.BASE_SEED + 1001, hmin=500.0)
    rng = np.random.default_rng(5)
    tau = np.zeros((m.n_nodes, 2)); tau[:, 0] = 0.3
    f = W.default_forcing(manning_n=0.0, manning_n_elem=rng.uniform(0.015, 0.035, m.n_elems), wind_tau=tau,
                          patm=101300.0 + 2e-3 * m.xy[:, 1], **W.m2_tide(0.5))
    out.append((m, W.coastal_initial_state(m), W.default_params(), f, True))
    return out


def solo(mesh, w0, params, forcing, pp, steps):
    s = Solver(mesh, params, forcing)
    s.set_state(w0, 0.0, pp)
    s.step(steps)
    w = s.state()
    d = s.diagnostics()
    s.close()
    return w, d


@pytest.mark.parametrize("precision", [0, DGSWE_MIXED])
def test_every_member_equals_its_solo_run(precision):
    ms = members()
    prm = dict(W.default_params(), precision=precision)
    steps = 60
    say(f"batch of {len(ms)} meshes, precision {precision}, {steps} steps")
    b = Batch([x[0] for x in ms], prm, [x[3] for x in ms])
    for i, x in enumerate(ms):
        b.set_state(i, x[1], 0.0, x[4])
    b.step(steps)
    got = [(b.state(i), b.diagnostics(i)) for i in range(len(ms))]
    b.close()
    dts = set()
    for i, x in enumerate(ms):
        say(f"solo run of member {i} ({x[0].n_elems} elements)")
        w, d = solo(x[0], x[1], prm, x[3], x[4], steps)
        assert np.array_equal(got[i][0], w), i
        assert got[i][1] == d, i
        dts.add(d["dt_last"])
    assert len(dts) > 1  # the members really step with their own dt


def test_error_in_one_member_stops_only_that_member():
    ms = members()[:3]
    prm = W.default_params()
    b = Batch([x[0] for x in ms], prm, [x[3] for x in ms])
    for i, x in enumerate(ms):
        w = x[1].copy()
        if i == 1:
            w[1, 0, 0] = math.nan
        b.set_state(i, w, 0.0, x[4])
    say("batch with a NaN in member 1")
    b.step(20)
    with pytest.raises(DgsweError) as ei:
        b.state(1)
    assert ei.value.status == 5
    for i in (0, 2):
        w, d = solo(ms[i][0], ms[i][1], prm, ms[i][3], ms[i][4], 20)
        assert np.array_equal(b.state(i), w)
    b.close()


def test_resetting_one_member_leaves_the_others():
    ms = members()[:4]
    prm = W.default_params()
    b = Batch([x[0] for x in ms], prm, [x[3] for x in ms])
    for i, x in enumerate(ms):
        b.set_state(i, x[1], 0.0, x[4])
    b.step(15)
    say("reset member 2 at t = 5 after 15 steps, 25 more steps")
    b.set_state(2, ms[2][1], 5.0, ms[2][4])
    b.step(25)
    for i, x in enumerate(ms):
        if i == 2:
            s = Solver(x[0], prm, x[3])
            s.set_state(x[1], 5.0, x[4])
            s.step(25)
            w, d = s.state(), s.diagnostics()
            s.close()
        else:
            w, d = solo(x[0], x[1], prm, x[3], x[4], 40)
        assert np.array_equal(b.state(i), w), i
        assert b.diagnostics(i) == d, i
    b.close()


def test_single_mesh_calls_refuse_a_batch():
    ms = members()[1:3]
    b = Batch([x[0] for x in ms], W.default_params())
    with pytest.raises(DgsweError) as ei:
        dgswe_read_state(b.h, None, True)
    assert ei.value.status == 1
    with pytest.raises(DgsweError) as ei:
        dgswe_read_state(b.h, None, True, member=2)
    assert ei.value.status == 1
    b.close()
