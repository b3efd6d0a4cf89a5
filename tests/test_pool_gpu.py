"""Serving pool (dgswe_create_pool): members join and leave between steps.

Bar: every member's state after its steps equals, bitwise, the same mesh
run alone by a single-mesh solver for the same number of steps (the
per-member arithmetic does not depend on what else is in the pool, nor on
where in the device stores the member landed).  Admission is by memory:
a mesh that does not fit is refused with DGSWE_E_NOMEM and the pool keeps
working.
"""
import numpy as np
import pytest

from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, DgsweError, Pool, Solver

from _cases import say

pytestmark = pytest.mark.gpu


def pad(w, nm):
    if nm == 3:
        return w
    out = np.zeros((3, 6, w.shape[2]))
    out[:, :3] = w
    return out


def request(i, n):
    m = W.coastal_mesh(n, W.BASE_SEED + 300 + i, hmin=1000.0, hmax=15000.0)
    f = W.default_forcing(manning_n=0.02 + 0.002 * i, **W.m2_tide(0.5 + 0.1 * i),
                          **W.holland_track(m, speed=3.0 + i, offshore=120e3))
    return m, f, W.coastal_initial_state(m)


def solo(m, f, w0, params, steps):
    s = Solver(m, params, f)
    s.set_state(w0, 0.0, True)
    s.step(steps)
    w = s.state()
    d = s.diagnostics()
    s.close()
    return w, d


@pytest.mark.parametrize("prec,order", [(0, 1), (DGSWE_MIXED, 1), (0, 2)])
def test_members_joining_and_leaving_equal_solo_runs(prec, order):
    # dt capped at 0.3 s: explicit Manning friction on the shallow coastal
    # cells of these coarse meshes is unstable at their CFL step
    params = W.default_params(precision=prec, p=order, cfl=0.2 if order == 1 else 0.1, dt_max=0.3)
    nm = 6 if order == 2 else 3
    reqs = [request(i, n) for i, n in enumerate((4000, 12000, 3000, 7000))]
    pool = Pool(30000, 6, params)
    say(f"pool precision={prec} p={order}: A joins, 12 steps")
    a = pool.add(reqs[0][0], forcing=reqs[0][1], w=pad(reqs[0][2], nm), postprocess=True)
    pool.step(12)
    say("B joins, 20 steps")
    b = pool.add(reqs[1][0], forcing=reqs[1][1], w=pad(reqs[1][2], nm), postprocess=True)
    pool.step(20)
    wa, da = pool.state(a)
    pool.remove(a)
    say("A left; C joins (into A's freed store), D joins, 15 steps")
    c = pool.add(reqs[2][0], forcing=reqs[2][1], w=pad(reqs[2][2], nm), postprocess=True)
    d = pool.add(reqs[3][0], forcing=reqs[3][1], w=pad(reqs[3][2], nm), postprocess=True)
    pool.step(15)
    wb, _ = pool.state(b)
    wc, _ = pool.state(c)
    wd, _ = pool.state(d)
    u = pool.usage()
    assert u["members"] == 3 and u["elems_used"] == sum(r[0].n_elems for r in reqs[1:])
    pool.close()
    for (m, f, w0), steps, wp, name in ((reqs[0], 32, wa, "A"), (reqs[1], 35, wb, "B"), (reqs[2], 15, wc, "C"),
                                        (reqs[3], 15, wd, "D")):
        say(f"solo run of {name}, {steps} steps")
        ws, ds = solo(m, f, pad(w0, nm), params, steps)
        assert np.array_equal(ws, wp), name
        assert np.abs(ws[1:, 0]).max() < 1e3  # a sane flow, not a diverged one
    assert da.steps == 32


def test_admission_by_memory_and_reuse():
    params = W.default_params(precision=DGSWE_MIXED, dt_max=0.3)
    reqs = [request(i, n) for i, n in enumerate((6000, 6000, 9000))]
    assert reqs[0][0].n_elems + reqs[1][0].n_elems + reqs[2][0].n_elems > 16000
    pool = Pool(16000, 4, params)
    a = pool.add(reqs[0][0], forcing=reqs[0][1], w=reqs[0][2], postprocess=True)
    b = pool.add(reqs[1][0], forcing=reqs[1][1], w=reqs[1][2], postprocess=True)
    prep = pool.prepare(reqs[2][0])
    with pytest.raises(DgsweError) as ei:
        pool.add(prepared=prep)
    assert ei.value.status == 3
    pool.step(10)
    wa, _ = pool.state(a)
    # b's store joins the free tail: room for the third mesh
    pool.remove(b)
    c = pool.add(prepared=prep, forcing=reqs[2][1], w=reqs[2][2], postprocess=True)
    pool.step(10)
    wc, _ = pool.state(c)
    wa2, _ = pool.state(a)
    pool.close()
    ws, _ = solo(*reqs[2], params, 10)
    assert np.array_equal(ws, wc)
    ws, _ = solo(*reqs[0], params, 20)
    assert np.array_equal(ws, wa2)
    assert not np.array_equal(wa, wa2)


def test_empty_pool_steps_and_slot_errors():
    pool = Pool(1000, 2, W.default_params())
    pool.step(3)  # nothing to do
    with pytest.raises(DgsweError):
        pool.remove(0)
    m = W.rect_mesh(4, 3, 400.0, 300.0, hb=5.0)
    s0 = pool.add(m, forcing=W.default_forcing(), w=W.state_from_nodal(m.tri, np.full(m.n_nodes, 0.1)))
    s1 = pool.add(m, forcing=W.default_forcing(), w=W.state_from_nodal(m.tri, np.full(m.n_nodes, 0.1)))
    with pytest.raises(DgsweError) as ei:
        pool.add(m)
    assert ei.value.status == 3  # no free slot
    pool.step(5)
    w0, d0 = pool.state(s0)
    w1, d1 = pool.state(s1)
    assert np.array_equal(w0, w1) and d0.steps == 5
    pool.close()
