"""Step graphs (dgswe_use_graphs): replays of captured steps equal the
launch-by-launch steps bitwise, replay after replay, with the program's
own eager work (read-backs, diagnostics) between the replays."""
import numpy as np
import pytest

from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Pool, Solver

from _cases import coastal_small, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("params", [dict(), dict(precision=DGSWE_MIXED), dict(p=2, cfl=0.1), dict(rk=33)])
def test_graph_replays_equal_eager_steps(params):
    wl = coastal_small()
    p = dict(wl.params, **params)
    nm = 6 if p.get("p", 1) == 2 else 3
    w0 = wl.w0 if nm == 3 else np.concatenate([wl.w0, np.zeros((3, 3, wl.w0.shape[2]))], axis=1)
    a = Solver(wl.mesh, p, wl.forcing)
    b = Solver(wl.mesh, p, wl.forcing)
    for s in (a, b):
        s.set_state(w0, 0.0, True)
    b.use_graphs(6)
    say(f"graphs {params}: replays of 6 steps against plain steps")
    for chunk in (6, 6, 5, 12, 7):
        a.step(chunk)
        b.step(chunk)
        wa, wb = a.state(), b.state()
        assert np.array_equal(wa, wb), chunk
        assert a.diagnostics()["t"] == b.diagnostics()["t"]
    a.close()
    b.close()


def test_graphs_in_a_pool_follow_joins():
    params = W.default_params(dt_max=0.3)
    ms = [W.coastal_mesh(n, W.BASE_SEED + 500 + i, hmin=1000.0, hmax=15000.0) for i, n in enumerate((4000, 8000))]
    fs = [W.default_forcing(manning_n=0.025, **W.m2_tide(1.0), **W.holland_track(m, offshore=120e3)) for m in ms]
    ws = [W.coastal_initial_state(m) for m in ms]
    pool = Pool(20000, 4, params)
    pool.use_graphs(6)
    x = pool.add(ms[0], forcing=fs[0], w=ws[0], postprocess=True)
    pool.step(12)
    y = pool.add(ms[1], forcing=fs[1], w=ws[1], postprocess=True)  # the graphs are recaptured
    pool.step(18)
    wx, _ = pool.state(x)
    wy, _ = pool.state(y)
    pool.close()
    for m, f, w, steps, got in ((ms[0], fs[0], ws[0], 30, wx), (ms[1], fs[1], ws[1], 18, wy)):
        s = Solver(m, params, f)
        s.set_state(w, 0.0, True)
        s.step(steps)
        assert np.array_equal(s.state(), got)
        s.close()
