"""The oracle's OpenMP loops only split independent work (edge slots,
elements, nodes) and its one reduction is an exact minimum, so its result
must be bitwise independent of the thread count."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, {root!r})
from oracle.oracle import Oracle
from paper_2508_21208_amd import workloads as W
m = W.coastal_mesh(20000, W.BASE_SEED + 31, hmin=500.0)
f = W.default_forcing(manning_n=0.025, **W.m2_tide(1.0), **W.holland_track(m))
o = Oracle(m, W.default_params(), f)
o.set_state(W.coastal_initial_state(m), 0.0, True)
o.step(30)
np.save(sys.argv[1], o.state())
"""


def run(threads, path):
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    subprocess.run([sys.executable, "-c", SCRIPT.format(root=ROOT), path], check=True, env=env)
    return np.load(path)


def test_oracle_bitwise_independent_of_threads(tmp_path):
    a = run(1, str(tmp_path / "a.npy"))
    b = run(4, str(tmp_path / "b.npy"))
    assert np.isfinite(a).all()
    assert np.array_equal(a, b)
