"""Serving loop with continuous batching (paper_2508_21208_amd.serving).

Bar: every request completes, and its result from the pool, where it
shared every step with whatever else was admitted, equals bitwise the
result of the same request run alone on its own solver (same precision).
"""
import numpy as np
import pytest

from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.serving import serve_one_at_a_time, serve_pool, summarize

from _cases import say

pytestmark = pytest.mark.gpu


def small_requests(n=10):
    meshes = [W.coastal_mesh(k, W.BASE_SEED + 400 + i, hmin=1000.0, hmax=15000.0)
              for i, k in enumerate((3000, 6000, 12000))]
    return W.cfg_serving(n, meshes=meshes, min_steps=20, max_steps=120, seed=W.BASE_SEED + 401)


@pytest.mark.parametrize("prec", [0, 1])
def test_pool_results_equal_alone_results(prec):
    reqs = small_requests()
    params = W.default_params(precision=prec, dt_max=0.3)
    say(f"serving {len(reqs)} requests through a pool (precision {prec})")
    # a small pool and short rounds: requests wait for room and join mid-run
    pool_out, el = serve_pool(reqs, params, rate=200.0, max_elems=30000, max_members=8, round_cap=16,
                              prep_workers=4, keep_states=True)
    st = summarize(pool_out, el)
    say(f"pool: {st}")
    assert len(pool_out) == len(reqs)
    say("the same requests one at a time")
    alone, _ = serve_one_at_a_time(reqs, params, rate=200.0, keep_states=True)
    by = {o.rid: o for o in alone}
    for o in pool_out:
        a = by[o.rid]
        assert o.t_model == a.t_model
        assert np.array_equal(o.state, a.state), o.rid
    # some requests had to wait for room or shared rounds with others
    assert max(o.admitted - o.arrival for o in pool_out) > 0
