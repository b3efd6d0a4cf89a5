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
