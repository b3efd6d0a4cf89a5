"""Shared seeded workloads and comparison helpers for the parity tests."""
import functools
import math
import sys

import numpy as np

from paper_2508_21208_amd import workloads as W


def say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def coastal_small(n=30000, seed=W.BASE_SEED + 21, hmin=300.0):
    m = W.coastal_mesh(n, seed, hmin=hmin)
    f = W.default_forcing(manning_n=0.025, **W.m2_tide(1.0), **W.holland_track(m))
    return W.Workload(f"coastal_small_{m.n_elems}", m, W.coastal_initial_state(m), W.default_params(), f,
                      200, True)


@functools.lru_cache(maxsize=None)
def coastal_600k():
    return W.cfg_coastal_tide()


@functools.lru_cache(maxsize=None)
def hurricane_4m():
    return W.cfg_hurricane()


def rel_l2(a, b):
    """Relative L2 difference per variable (zeta, Qx, Qy) over all modes."""
    out = []
    for v in range(3):
        den = np.linalg.norm(b[v])
        num = np.linalg.norm(a[v] - b[v])
        out.append(num / den if den > 0 else num)
    return out


def exact_mass(o, w):
    """sum of A_e zeta_0 over the oracle's elements, correctly rounded (the
    oracle's own diagnostic adds in element order, whose rounding error on a
    4M-element sum of mixed-sign terms reaches ~1e-11 relative)"""
    return math.fsum((o.geometry()["area"] * w[0, 0]).tolist())


@functools.lru_cache(maxsize=None)
def shallow_open_boundary():
    """A 6 km x 2 km box open to the sea on its west side, whose bed rises
    to h_e = -0.015 m (dry land) along that side and deepens eastward; a
    tide zeta_b = 0.02 + 0.05 cos(2 pi t / 400 s) makes the ocean ghost
    (wet iff zeta_b + the edge's mean bathymetry > H0) wet and dry in turn,
    and the boundary elements flood and drain through it."""
    m = W.rect_mesh(30, 10, 6000.0, 2000.0, hb=lambda x, y: -0.015 + 3.0e-3 * x + 1e-4 * y,
                    types=(W.BC_LAND, W.BC_LAND, W.BC_LAND, W.BC_OCEAN))
    w0 = W.state_from_nodal(m.tri, np.zeros(m.n_nodes))
    f = W.default_forcing(manning_n=0.02, tide_amp=[0.05], tide_omega=[2 * math.pi / 400.0], tide_phase=[0.0],
                          tide_offset=0.02)
    return W.Workload("shallow_open_boundary", m, w0, W.default_params(), f, 300, True)


def isolated_triangles(n, size=100.0, gap=50.0, hb=10.0):
    """n triangles that share no edge (each one a closed basin, every edge a
    wall), laid out on a grid: any 256 consecutive ones have 768 edges, more
    than the stage kernel takes per chunk, so the library must chunk such a
    mesh more finely."""
    k = int(math.ceil(math.sqrt(n)))
    xy, tri = [], []
    for i in range(n):
        x0, y0 = (i % k) * (size + gap), (i // k) * (size + gap)
        b = len(xy)
        xy += [(x0, y0), (x0 + size, y0), (x0, y0 + size)]
        tri.append((b, b + 1, b + 2))
    tri = np.asarray(tri, np.int32)
    bnd = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]]).astype(np.int32)
    xy = np.asarray(xy, np.float64)
    return W.Mesh(xy, np.full(len(xy), hb), tri, bnd, np.full(len(bnd), W.BC_LAND, np.int32),
                  {"kind": "isolated", "n": n})
