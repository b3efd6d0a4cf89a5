"""Launch-configuration autotuner: times candidate chunk sizes (elements
per workgroup chunk of the stage kernels) and, at p = 2, the register
budget of the stage kernel (waves per SIMD) on the mesh at hand, with its
own forcing and state, and returns the fastest.  The configurations change
only how the work is split over workgroups, never the results (bitwise).

Small meshes favour small chunks (more workgroups for a short grid, less
time per chunk), large ones large chunks (less halo recomputation); at
p = 1 chunk 0 is also a candidate: the library's own per-mesh choice, the
largest chunk whose LDS lets the most workgroups share a compute unit.
Results are cached per (order, precision, mesh-size decade).
"""
from __future__ import annotations

import math
import time

from .dgswe import Solver

_cache: dict = {}


def candidates(params: dict, auto: bool = True):
    p2 = int(params.get("p", 1)) == 2
    chunks = (64, 128, 192, 256) if p2 or not auto else (0, 64, 128, 192, 256)
    waves = (2, 3) if p2 else (0,)
    return [(c, w) for c in chunks for w in waves]


def tune(mesh, params: dict, forcing: dict, w0, postprocess=True, steps=20, hip_stream=None, use_cache=True,
         repeats=3, auto=True):
    """Returns (best params dict, table of (chunk, waves, us per step)); each
    candidate's time is the median of `repeats` runs of `steps` steps.
    auto=False leaves out chunk 0 (the library's per-mesh choice), so that
    the result names an explicit chunk size."""
    key = (int(params.get("p", 1)), int(params.get("precision", 0)), int(math.log10(max(1, mesh.n_elems))), auto)
    if use_cache and key in _cache:
        best = _cache[key]
        return dict(params, chunk=best[0], waves=best[1]), None
    import torch
    table = []
    for c, w in candidates(params, auto):
        s = Solver(mesh, dict(params, chunk=c, waves=w), forcing, hip_stream=hip_stream)
        s.set_state(w0, 0.0, postprocess)
        s.step(3)
        s.diagnostics()
        torch.cuda.synchronize()
        runs = []
        for _ in range(max(1, repeats)):
            t0 = time.perf_counter()
            s.step(steps)
            s.diagnostics()
            runs.append(1e6 * (time.perf_counter() - t0) / steps)
        table.append((c, w, sorted(runs)[len(runs) // 2]))
        s.close()
    best = min(table, key=lambda r: r[2])
    _cache[key] = best[:2]
    return dict(params, chunk=best[0], waves=best[1]), table
