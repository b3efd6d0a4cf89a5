"""The storm-surge ensemble at its full size (64 members, 19.5M triangles,
mixed precision), as one p = 1 batch and with seeded orders p in {1, 2}
advanced together (the bench's configurations): members equal their solo
runs bitwise and agree with the FP64 oracle within the mixed-precision bar
(vertex elevation 1e-4 m)."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Batch, Solver

from _cases import say

pytestmark = pytest.mark.gpu

STEPS = 5


def test_full_ensemble_members():
    ens = W.cfg_ensemble()
    ne = sum(w.mesh.n_elems for w in ens)
    assert len(ens) == 64 and ne > 15_000_000
    params = dict(ens[0].params, precision=DGSWE_MIXED)
    say(f"full ensemble: 64 members, {ne} triangles, {STEPS} steps")
    b = Batch([w.mesh for w in ens], params, [w.forcing for w in ens])
    for i, w in enumerate(ens):
        b.set_state(i, w.w0, 0.0, w.postprocess_initial)
    b.step(STEPS)
    picks = (0, 37, 63)
    got = {i: b.state(i) for i in picks}
    steps = [b.diagnostics(i)["steps"] for i in picks]
    b.close()
    assert steps == [STEPS] * 3
    for i in picks:
        w = ens[i]
        say(f"solo member {i} ({w.mesh.n_elems} triangles)")
        s = Solver(w.mesh, params, w.forcing)
        s.set_state(w.w0, 0.0, w.postprocess_initial)
        s.step(STEPS)
        assert np.array_equal(s.state(), got[i]), i
        s.close()
    w = ens[0]
    say("oracle, member 0")
    o = Oracle(w.mesh, w.params, w.forcing)
    o.set_state(w.w0, 0.0, w.postprocess_initial)
    o.step(STEPS)
    wo = o.state()
    V = np.array([[1, -1, -1], [1, 1, -1], [1, 0, 2]], float)
    ez = np.abs(V @ (got[0][0] - wo[0])).max()
    say(f"member 0: vertex elevation error {ez:.3e} m")
    assert ez <= 1e-4


def test_full_ensemble_both_orders_one_launch():
    """The same 64 members with seeded orders p in {1, 2} (27 at p = 1, 37 at
    p = 2), both orders advanced by dgswe_step_pair with 6-step graphs: one
    member of each order equals its solo run bitwise and agrees with the
    FP64 oracle of its order within the mixed-precision bar."""
    import torch
    from paper_2508_21208_amd.dgswe import Ensemble
    ens = W.cfg_ensemble()
    orders = W.ensemble_orders(len(ens))
    params = dict(ens[0].params, precision=DGSWE_MIXED)
    op = {2: dict(cfl=0.1)}
    e = Ensemble([w.mesh for w in ens], orders, params, [w.forcing for w in ens],
                 hip_stream=torch.cuda.current_stream().cuda_stream, order_params=op)
    assert e.fused
    e.use_graphs(6)
    for i, w in enumerate(ens):
        e.set_state(i, w.w0, 0.0, w.postprocess_initial)
    say(f"full ensemble, both orders ({orders.count(1)} p=1, {orders.count(2)} p=2), 6 steps")
    e.step(6)
    picks = (orders.index(1), orders.index(2))
    got = {i: e.state(i) for i in picks}
    e.close()
    V = np.array([[1, -1, -1, 1, 1, 1], [1, 1, -1, 1, -1, 1], [1, 0, 2, 0, 0, 3]], float)
    for i in picks:
        w, p = ens[i], orders[i]
        prm = dict(params, p=p, **op.get(p, {}))
        w0 = w.w0 if p == 1 else np.concatenate([w.w0, np.zeros((3, 3, w.w0.shape[2]))], axis=1)
        say(f"solo member {i} at p = {p} ({w.mesh.n_elems} triangles)")
        s = Solver(w.mesh, prm, w.forcing)
        s.set_state(w0, 0.0, w.postprocess_initial)
        s.step(6)
        assert np.array_equal(s.state(), got[i]), i
        s.close()
        say(f"oracle, member {i} at p = {p}")
        o = Oracle(w.mesh, dict(w.params, p=p, **op.get(p, {})), w.forcing, order=p)
        o.set_state(w0, 0.0, w.postprocess_initial)
        o.step(6)
        wo = o.state()
        nm = 3 if p == 1 else 6
        ez = np.abs(V[:, :nm] @ (got[i][0] - wo[0])).max()
        say(f"member {i}: vertex elevation error {ez:.3e} m")
        assert ez <= 1e-4
