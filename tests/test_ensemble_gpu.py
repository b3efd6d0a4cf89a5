"""An ensemble with members of both orders (dgswe.Ensemble: one batch per
order; on a shared stream both advance through dgswe_step_pair, one stage
launch for every member): every member's state, time and step count equal
its solo run at its order, bitwise, with and without step graphs and
persistent workgroups."""
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


CASES = [(0, False, 6, 0, 1), (DGSWE_MIXED, False, 6, 0, 1), (0, True, 0, 0, 1), (DGSWE_MIXED, True, 6, 0, 1),
         (0, True, 0, 2, 1), (DGSWE_MIXED, True, 6, 3, 1), (0, True, 6, 0, 0), (DGSWE_MIXED, True, 0, 2, 0)]


@pytest.mark.parametrize("prec,fused,graphs,persistent,split", CASES)
def test_mixed_order_ensemble_equals_solo_runs(prec, fused, graphs, persistent, split, monkeypatch):
    import torch
    # split = 0: the other arrangement of a pair stage (the p = 2
    # post-processing, then one launch of both orders' stage work)
    monkeypatch.setenv("DGSWE_PAIR_SPLIT", str(split))
    mem = members()
    orders = [1, 2, 2, 1, 2]
    params = W.default_params(precision=prec, dt_max=0.3, persistent=persistent)
    op = {2: dict(cfl=0.1)}
    stream = torch.cuda.current_stream().cuda_stream if fused else None
    ens = Ensemble([m for m, _, _ in mem], orders, params, [f for _, f, _ in mem], order_params=op,
                   hip_stream=stream, fused=fused)
    assert ens.fused == fused
    ens.use_graphs(graphs)
    for i, (_, _, w0) in enumerate(mem):
        ens.set_state(i, w0, 0.0, True)
    say(f"ensemble precision={prec} fused={fused} graphs={graphs} persistent={persistent} split={split}: "
        f"orders {orders}, 13 steps")
    ens.step(13)
    got = [ens.state(i) for i in range(len(mem))]
    dg = [ens.diagnostics(i) for i in range(len(mem))]
    ens.close()
    for i, ((m, f, w0), p) in enumerate(zip(mem, orders)):
        prm = dict(params, p=p, persistent=0, **op.get(p, {}))
        s = Solver(m, prm, f)
        w = w0 if p == 1 else np.concatenate([w0, np.zeros((3, 3, w0.shape[2]))], axis=1)
        s.set_state(w, 0.0, True)
        s.step(13)
        ws = s.state()
        d = s.diagnostics()
        s.close()
        assert ws.shape == got[i].shape and np.array_equal(ws, got[i]), i
        assert d["t"] == dg[i]["t"] and d["steps"] == dg[i]["steps"] == 13
