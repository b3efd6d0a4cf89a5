"""An ensemble with members of both orders (dgswe.Ensemble: one batch per
order on one stream, step graphs on): every member's state, time and step
count equal its solo run at its order, bitwise."""
import numpy as np
import pytest

from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Ensemble, Solver

from _cases import say

pytestmark = pytest.mark.gpu


def members():
    out = []
    for i, n in enumerate((3000, 5000, 4000, 2500, 6000)):
        m = W.coastal_mesh(n, W.BASE_SEED + 700 + i, hmin=1000.0, hmax=15000.0)
        f = W.default_forcing(manning_n=0.02 + 0.003 * i, **W.m2_tide(1.0),
                              **W.holland_track(m, speed=3.0 + i, offshore=120e3))
        out.append((m, f, W.coastal_initial_state(m)))
    return out


@pytest.mark.parametrize("prec", [0, DGSWE_MIXED])
def test_mixed_order_ensemble_equals_solo_runs(prec):
    mem = members()
    orders = [1, 2, 2, 1, 2]
    params = W.default_params(precision=prec, dt_max=0.3)
    op = {2: dict(cfl=0.1)}
    ens = Ensemble([m for m, _, _ in mem], orders, params, [f for _, f, _ in mem], order_params=op)
    ens.use_graphs(6)
    for i, (_, _, w0) in enumerate(mem):
        ens.set_state(i, w0, 0.0, True)
    say(f"ensemble precision={prec}: orders {orders}, 13 steps")
    ens.step(13)
    got = [ens.state(i) for i in range(len(mem))]
    dg = [ens.diagnostics(i) for i in range(len(mem))]
    ens.close()
    for i, ((m, f, w0), p) in enumerate(zip(mem, orders)):
        prm = dict(params, p=p, **op.get(p, {}))
        s = Solver(m, prm, f)
        w = w0 if p == 1 else np.concatenate([w0, np.zeros((3, 3, w0.shape[2]))], axis=1)
        s.set_state(w, 0.0, True)
        s.step(13)
        ws = s.state()
        d = s.diagnostics()
        s.close()
        assert ws.shape == got[i].shape and np.array_equal(ws, got[i]), i
        assert d["t"] == dg[i]["t"] and d["steps"] == dg[i]["steps"] == 13
