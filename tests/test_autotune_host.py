"""The autotuner's logic on the host with a stand-in solver and clock (no
GPU): the candidate sets (chunk sizes; register budgets at p = 2 only), the
choice of the fastest measured candidate, and the cache per (order,
precision, mesh-size decade)."""
import types

import pytest
import torch

from paper_2508_21208_amd import autotune as AT


class Clock:
    t = 0.0

    @classmethod
    def perf_counter(cls):
        return cls.t


COST = {}  # (chunk, waves) -> seconds per step
RUNS = []


class FakeSolver:
    def __init__(self, mesh, params, forcing, hip_stream=None):
        self.key = (params["chunk"], params["waves"])
        RUNS.append(self.key)

    def set_state(self, w, t, pp):
        pass

    def step(self, n):
        Clock.t += n * COST.get(self.key, 1e-3)

    def diagnostics(self):
        return {}

    def close(self):
        pass


@pytest.fixture(autouse=True)
def fakes(monkeypatch):
    monkeypatch.setattr(AT, "Solver", FakeSolver)
    monkeypatch.setattr(AT, "time", types.SimpleNamespace(perf_counter=Clock.perf_counter))
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    AT._cache.clear()
    RUNS.clear()
    COST.clear()


def test_median_of_repeats():
    """each candidate is timed `repeats` times and its median kept"""
    mesh = types.SimpleNamespace(n_elems=12_000)
    COST.update({(0, 0): 2.2e-5, (64, 0): 3e-5, (128, 0): 2e-5, (192, 0): 2.5e-5, (256, 0): 2.8e-5})
    best, table = AT.tune(mesh, {"p": 1, "precision": 0}, {}, None, steps=10, repeats=5)
    assert best["chunk"] == 128 and len(table) == 5


def test_candidates():
    assert AT.candidates({"p": 1}) == [(0, 0), (64, 0), (128, 0), (192, 0), (256, 0)]
    assert AT.candidates({"p": 1}, auto=False) == [(64, 0), (128, 0), (192, 0), (256, 0)]
    c2 = AT.candidates({"p": 2})
    assert len(c2) == 8 and {w for _, w in c2} == {2, 3} and {c for c, _ in c2} == {64, 128, 192, 256}


def test_picks_the_fastest_and_caches_per_size_decade():
    mesh = types.SimpleNamespace(n_elems=12_000)
    COST.update({(64, 0): 3e-5, (128, 0): 2e-5, (192, 0): 2.5e-5, (256, 0): 2.8e-5})
    best, table = AT.tune(mesh, {"p": 1, "precision": 0}, {}, None, steps=10)
    assert best["chunk"] == 128 and best["waves"] == 0
    assert [r[:2] for r in table] == AT.candidates({"p": 1})
    assert abs(dict(((c, w), us) for c, w, us in table)[(128, 0)] - 20.0) < 1e-9  # us per step
    n = len(RUNS)
    again, t2 = AT.tune(types.SimpleNamespace(n_elems=30_000), {"p": 1, "precision": 0}, {}, None)
    assert t2 is None and again["chunk"] == 128 and len(RUNS) == n  # same decade: cached
    COST[(256, 0)] = 1e-5
    other, t3 = AT.tune(types.SimpleNamespace(n_elems=300_000), {"p": 1, "precision": 0}, {}, None)
    assert t3 is not None and other["chunk"] == 256  # another decade: measured again


def test_p2_tunes_the_register_budget():
    mesh = types.SimpleNamespace(n_elems=5_000)
    COST.update({(192, 3): 1e-5})
    best, table = AT.tune(mesh, {"p": 2, "precision": 0}, {}, None, steps=5)
    assert (best["chunk"], best["waves"]) == (192, 3) and len(table) == 8
