"""Serving loop with continuous batching over a device-resident pool.

Requests (mesh, forcing, initial state, horizon in steps) arrive over time.
Each arriving mesh is prepared on a host worker thread (validation, element
ordering, halo and edge tables: `dgswe_prepare_mesh`, no device work) while
the device steps the requests already admitted.  At every round boundary the
loop retires the requests that reached their horizon (their state is read
back), then admits waiting prepared requests in arrival order as long as the
pool has room (admission by device memory: `dgswe_member_add_prepared`
refuses a mesh that does not fit), and enqueues the next round: one
`dgswe_step` of K steps for all members, K = the smallest remaining horizon,
capped so that new arrivals wait at most one round.  Every member advances
with its own dt, forcing and time; its result does not depend on the other
members (bitwise).

`serve_one_at_a_time` is the baseline: the same requests in arrival order,
each alone on a fresh single-mesh solver.
"""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from .dgswe import DgsweError, Pool, Solver, dgswe_prepared_free


@dataclass
class Outcome:
    rid: int
    n_elems: int
    horizon: int
    arrival: float      # s after the start of the run
    admitted: float     # s, when the request joined the pool (or started alone)
    finished: float     # s, when its result was back on the host
    t_model: float      # model time reached
    state: np.ndarray | None = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def summarize(outcomes: list, elapsed: float) -> dict:
    lat = np.array([o.latency for o in outcomes])
    work = sum(o.n_elems * o.horizon * 2 for o in outcomes)
    return {"requests": len(outcomes), "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()), "max_s": float(lat.max()),
            "makespan_s": elapsed, "elem_stage_per_s": work / elapsed if elapsed > 0 else 0.0}


def serve_pool(requests, params: dict, rate: float, max_elems: int, max_members: int = 256,
               round_cap: int = 100, prep_workers: int = 8, keep_states: bool = False, hip_stream=None,
               log=None, chunk_rule=None):
    """Run `requests` (workloads.Request, arrival in mean gaps) arriving at
    `rate` per second through a pool; returns (outcomes, elapsed s).
    chunk_rule(n_elems) -> chunk size used to prepare each mesh (e.g. from
    the autotuner: smaller chunks for small meshes); default: the pool's."""
    pool = Pool(max_elems, max_members, params, hip_stream=hip_stream)
    reqs = sorted(requests, key=lambda r: r.arrival)
    arrive = [r.arrival / rate for r in reqs]
    ex = ThreadPoolExecutor(max_workers=prep_workers)
    futures = {}
    waiting = []        # indices into reqs, arrival order, not yet admitted
    active = {}         # slot -> [index, remaining steps, admitted time]
    outcomes = []
    nxt = 0
    t0 = time.perf_counter()

    def now():
        return time.perf_counter() - t0

    try:
        while len(outcomes) < len(reqs):
            # arrivals: start their host preparation
            while nxt < len(reqs) and arrive[nxt] <= now():
                if chunk_rule is None:
                    futures[nxt] = ex.submit(pool.prepare, reqs[nxt].mesh)
                else:
                    futures[nxt] = ex.submit(pool.prepare_with, reqs[nxt].mesh,
                                             dict(params, chunk=chunk_rule(reqs[nxt].mesh.n_elems)))
                waiting.append(nxt)
                nxt += 1
            # admission, in arrival order, while the pool has room
            while waiting and futures[waiting[0]].done():
                i = waiting[0]
                r = reqs[i]
                prep = futures[i].result()
                try:
                    slot = pool.add(prepared=prep, forcing=r.forcing, w=r.w0, t=0.0, postprocess=True)
                except Exception as e:
                    if getattr(e, "prepared_consumed", False):
                        # the pool took the handle (and let the member go again)
                        del futures[i]
                        raise
                    if not isinstance(e, DgsweError) or e.status != 3 or not active:
                        # not a matter of waiting: invalid, or larger than the empty pool
                        del futures[i]
                        dgswe_prepared_free(prep)
                        raise
                    futures[i] = _Done(prep)  # keep it prepared; retry after the next retirement
                    break
                waiting.pop(0)
                del futures[i]
                active[slot] = [i, r.horizon, now()]
            if not active:
                # idle: wait for the next preparation or arrival
                if waiting:
                    f = futures[waiting[0]]
                    if hasattr(f, "result") and not isinstance(f, _Done):
                        f.result()
                    continue
                if nxt < len(reqs):
                    time.sleep(max(0.0, arrive[nxt] - now()))
                continue
            k = min(rem for _, rem, _ in active.values())
            k = max(1, min(k, round_cap))
            pool.step(k)
            done = []
            for slot, a in active.items():
                a[1] -= k
                if a[1] == 0:
                    done.append(slot)
            # the reads wait for the round; a round without a retirement
            # still synchronises (usage) before admitting new members
            if not done:
                pool.usage()
            for slot in done:
                i, _, adm = active.pop(slot)
                w, d = pool.state(slot)
                pool.remove(slot)
                r = reqs[i]
                outcomes.append(Outcome(r.rid, r.mesh.n_elems, r.horizon, arrive[i], adm, now(), d.t,
                                        w if keep_states else None))
                if log:
                    log(f"serve: request {r.rid} ({r.mesh.n_elems} el, {r.horizon} steps) done, "
                        f"latency {outcomes[-1].latency:.3f} s, {len(active)} active")
    finally:
        ex.shutdown(wait=True)
        for f in futures.values():
            prep = f.result() if not isinstance(f, _Done) else f.value
            dgswe_prepared_free(prep)
        pool.close()
    return outcomes, now()


class _Done:
    """a preparation that finished earlier (kept while the pool is full)"""

    def __init__(self, value):
        self.value = value

    def done(self):
        return True

    def result(self):
        return self.value


def serve_one_at_a_time(requests, params: dict, rate: float, keep_states: bool = False, hip_stream=None,
                        log=None, deadline_s: float | None = None):
    """The baseline: requests in arrival order, each alone on a new
    single-mesh solver (created, forced, stepped to its horizon, read back,
    destroyed).  With deadline_s, stops starting requests after that many
    seconds (the unfinished ones are left out of the outcomes)."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    outcomes = []
    t0 = time.perf_counter()
    for r in reqs:
        arr = r.arrival / rate
        wait = arr - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        if deadline_s is not None and time.perf_counter() - t0 > deadline_s:
            break
        start = time.perf_counter() - t0
        s = Solver(r.mesh, params, r.forcing, hip_stream=hip_stream)
        s.set_state(r.w0, 0.0, True)
        s.step(r.horizon)
        w = s.state()
        t_model = s.diag.t
        s.close()
        outcomes.append(Outcome(r.rid, r.mesh.n_elems, r.horizon, arr, start, time.perf_counter() - t0, t_model,
                                w if keep_states else None))
        if log:
            log(f"alone: request {r.rid} ({r.mesh.n_elems} el, {r.horizon} steps), "
                f"latency {outcomes[-1].latency:.3f} s")
    return outcomes, time.perf_counter() - t0
