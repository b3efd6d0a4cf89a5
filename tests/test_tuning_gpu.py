"""Launch tuning (dgswe_params.chunk, .waves) and the autotuner: the chunk
size and the register budget change how the work is split over workgroups,
never the results (bitwise)."""
import numpy as np
import pytest

from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.autotune import tune
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Pool, Solver

from _cases import coastal_small, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("params", [dict(), dict(precision=DGSWE_MIXED), dict(p=2, cfl=0.1)])
def test_results_do_not_depend_on_the_launch_configuration(params):
    wl = coastal_small()
    p = dict(wl.params, **params)
    w0 = wl.w0
    if p.get("p", 1) == 2:
        w0 = np.concatenate([wl.w0, np.zeros_like(wl.w0)], axis=1)
    ref = None
    configs = [(0, 0), (64, 0), (128, 0), (192, 0)] + ([(0, 1), (96, 3)] if p.get("p", 1) == 2 else [])
    for c, wv in configs:
        say(f"{params}: chunk {c}, waves {wv}")
        s = Solver(wl.mesh, dict(p, chunk=c, waves=wv), wl.forcing)
        s.set_state(w0, 0.0, True)
        s.step(25)
        w = s.state()
        s.close()
        if ref is None:
            ref = w
        assert np.array_equal(w, ref), (c, wv)


def test_pool_members_with_different_chunks():
    params = W.default_params(dt_max=0.3)
    ms = [W.coastal_mesh(n, W.BASE_SEED + 600 + i, hmin=1000.0, hmax=15000.0) for i, n in enumerate((4000, 9000))]
    f = W.default_forcing(manning_n=0.025, **W.m2_tide(1.0))
    pool = Pool(20000, 4, params)
    a = pool.add(prepared=Pool.prepare_with(pool, ms[0], dict(params, chunk=64)), forcing=f,
                 w=W.coastal_initial_state(ms[0]), postprocess=True)
    b = pool.add(ms[1], forcing=f, w=W.coastal_initial_state(ms[1]), postprocess=True)
    pool.step(20)
    wa, _ = pool.state(a)
    wb, _ = pool.state(b)
    pool.close()
    for m, got in ((ms[0], wa), (ms[1], wb)):
        s = Solver(m, params, f)
        s.set_state(W.coastal_initial_state(m), 0.0, True)
        s.step(20)
        assert np.array_equal(s.state(), got)
        s.close()


def test_autotuner_picks_a_candidate():
    m = W.coastal_mesh(10000, W.BASE_SEED + 610, hmin=1000.0, hmax=15000.0)
    p = W.default_params(dt_max=0.3)
    best, table = tune(m, p, W.default_forcing(manning_n=0.025), W.coastal_initial_state(m), steps=10,
                       use_cache=False)
    say(f"autotune 10k: {table} -> chunk {best['chunk']}")
    assert best["chunk"] in (0, 64, 128, 192, 256) and len(table) == 5
