"""The storm-surge ensemble at its full size (64 members, 19.5M triangles,
mixed precision, one batch: the bench's configuration), 5 steps: three
members equal their solo runs bitwise, and member 0 agrees with the FP64
oracle within the mixed-precision bar (vertex elevation 1e-4 m)."""
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
