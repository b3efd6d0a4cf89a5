"""The serving loop's scheduling, on the host with a stand-in pool (no GPU):
every request completes; admission is in arrival order and waits for room
when the pool is full (a request larger than the empty pool is an error);
each request runs exactly its horizon; latencies are measured from arrival;
the summary's percentiles match the outcomes."""
import types

import numpy as np
import pytest

from paper_2508_21208_amd import serving as SV
from paper_2508_21208_amd.dgswe import DgsweError


class FakePool:
    """Capacity in elements and slots; step(k) advances every member by k
    steps; state() returns the member's step count as its 'state'."""
    log = []

    def __init__(self, max_elems, max_members, params, hip_stream=None):
        self.cap, self.slots = max_elems, max_members
        self.members = {}
        FakePool.log = []

    def prepare(self, mesh):
        return types.SimpleNamespace(n=mesh.n_elems, rid=mesh.rid)

    def prepare_with(self, mesh, params):
        return self.prepare(mesh)

    def add(self, mesh=None, forcing=None, w=None, t=0.0, postprocess=False, prepared=None):
        p = prepared
        used = sum(m["n"] for m in self.members.values())
        if p.n > self.cap or used + p.n > self.cap or len(self.members) >= self.slots:
            raise DgsweError(3, "no room")
        slot = min(set(range(self.slots)) - set(self.members))
        self.members[slot] = {"n": p.n, "steps": 0, "rid": p.rid}
        FakePool.log.append(("add", p.rid))
        return slot

    def step(self, k):
        for m in self.members.values():
            m["steps"] += k

    def usage(self):
        return {}

    def state(self, slot):
        m = self.members[slot]
        return np.array([m["steps"]]), types.SimpleNamespace(t=float(m["steps"]))

    def remove(self, slot):
        FakePool.log.append(("remove", self.members[slot]["rid"]))
        del self.members[slot]

    def close(self):
        pass


def _requests(sizes, horizons):
    reqs = []
    for i, (n, h) in enumerate(zip(sizes, horizons)):
        mesh = types.SimpleNamespace(n_elems=n, rid=i)
        reqs.append(types.SimpleNamespace(rid=i, mesh=mesh, forcing={}, w0=None, horizon=h, arrival=0.01 * i))
    return reqs


@pytest.fixture(autouse=True)
def fake_pool(monkeypatch):
    monkeypatch.setattr(SV, "Pool", FakePool)
    monkeypatch.setattr(SV, "dgswe_prepared_free", lambda p: None)


def test_all_requests_complete_with_their_horizons_in_arrival_order():
    sizes = [400, 300, 500, 200, 600, 100, 350]
    horizons = [30, 5, 12, 40, 7, 3, 20]
    reqs = _requests(sizes, horizons)
    out, elapsed = SV.serve_pool(reqs, {}, rate=100.0, max_elems=1000, max_members=3, round_cap=4,
                                 keep_states=True)
    assert sorted(o.rid for o in out) == list(range(len(reqs)))
    for o in out:
        assert o.state[0] == o.horizon == horizons[o.rid]  # exactly its horizon
        assert o.finished >= o.admitted >= o.arrival - 1e-9 and o.latency >= 0
    adds = [rid for kind, rid in FakePool.log if kind == "add"]
    assert adds == sorted(adds)  # admission in arrival order
    s = SV.summarize(out, elapsed)
    lat = np.array([o.latency for o in out])
    assert s["requests"] == len(reqs) and s["p50_s"] == float(np.percentile(lat, 50))
    assert s["max_s"] == float(lat.max())


def test_waits_for_room_and_refuses_what_never_fits():
    reqs = _requests([900, 900, 900], [5, 5, 5])  # one at a time in a pool of 1000
    out, _ = SV.serve_pool(reqs, {}, rate=1000.0, max_elems=1000, max_members=4)
    assert len(out) == 3
    kinds = [k for k, _ in FakePool.log]
    assert kinds == ["add", "remove", "add", "remove", "add", "remove"]
    with pytest.raises(DgsweError):
        SV.serve_pool(_requests([2000], [5]), {}, rate=1000.0, max_elems=1000, max_members=4)


class ConsumingFailPool(FakePool):
    """add() takes the prepared handle and then fails while configuring the
    member (as a bad forcing or state would), after removing the member."""
    freed = []

    def add(self, mesh=None, forcing=None, w=None, t=0.0, postprocess=False, prepared=None):
        slot = super().add(mesh, forcing, w, t, postprocess, prepared)
        if prepared.rid == 1:
            self.remove(slot)
            e = ValueError("bad forcing array")
            e.prepared_consumed = True
            raise e
        return slot


def test_a_handle_taken_by_the_pool_is_never_freed_again(monkeypatch):
    ConsumingFailPool.freed = []
    monkeypatch.setattr(SV, "Pool", ConsumingFailPool)
    monkeypatch.setattr(SV, "dgswe_prepared_free", lambda p: ConsumingFailPool.freed.append(p.rid))
    reqs = _requests([100, 200, 300], [5, 5, 5])
    with pytest.raises(ValueError):
        SV.serve_pool(reqs, {}, rate=1e6, max_elems=10_000, max_members=4)
    # request 1's handle went to the pool: neither the failure path nor the
    # final clean-up frees it; request 2 (prepared, never admitted) is freed
    assert 1 not in ConsumingFailPool.freed
    assert ConsumingFailPool.freed.count(2) <= 1
    assert ("remove", 1) in FakePool.log


def test_a_handle_refused_before_admission_is_freed_once(monkeypatch):
    class RefusingPool(FakePool):
        def add(self, mesh=None, forcing=None, w=None, t=0.0, postprocess=False, prepared=None):
            e = DgsweError(1, "invalid forcing")
            e.prepared_consumed = False
            raise e
    freed = []
    monkeypatch.setattr(SV, "Pool", RefusingPool)
    monkeypatch.setattr(SV, "dgswe_prepared_free", lambda p: freed.append(p.rid))
    with pytest.raises(DgsweError):
        SV.serve_pool(_requests([100], [5]), {}, rate=1e6, max_elems=10_000, max_members=4)
    assert freed == [0]
