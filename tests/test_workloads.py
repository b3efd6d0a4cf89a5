"""The seeded input generators (paper_2508_21208_amd.workloads) produce the
workloads their recipe states: sizes, grading, bathymetry, boundary types,
forcing parameters and seeded determinism.  CPU only; no method arithmetic
is involved."""
import math

import numpy as np
import pytest

from paper_2508_21208_amd import workloads as W


def _angles(m):
    P = m.xy[m.tri]

    def ang(a, b, c):
        u, v = b - a, c - a
        cos = np.sum(u * v, -1) / np.linalg.norm(u, axis=-1) / np.linalg.norm(v, axis=-1)
        return np.degrees(np.arccos(np.clip(cos, -1.0, 1.0)))
    return np.stack([ang(P[:, 0], P[:, 1], P[:, 2]), ang(P[:, 1], P[:, 2], P[:, 0]), ang(P[:, 2], P[:, 0], P[:, 1])], 1)


def _areas(m):
    P = m.xy[m.tri]
    return 0.5 * ((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1]) - (P[:, 2, 0] - P[:, 0, 0]) * (P[:, 1, 1] - P[:, 0, 1]))


def _edges(tri):
    e = np.sort(np.concatenate([tri[:, [1, 2]], tri[:, [2, 0]], tri[:, [0, 1]]]), axis=1)
    return np.unique(e, axis=0)


def test_gaussian_hump():
    wl = W.cfg_gaussian_1600()
    m = wl.mesh
    assert (m.n_elems, m.n_nodes, len(_edges(m.tri))) == (1600, 861, 2460)
    assert np.all(m.hb == 10.0) and np.all(m.bnd_type == W.BC_LAND)
    assert np.allclose(_areas(m), 500.0 * 500.0 / 2)
    vz = wl.w0[0, 0] + np.array([[-1, -1], [1, -1], [0, 2]]) @ wl.w0[0, 1:]  # vertex values
    assert math.isclose(vz.max(), 0.1, rel_tol=1e-12)  # the hump's peak sits on the centre node
    assert np.all(wl.w0[1:] == 0.0) and wl.params["cfl"] == 0.2


@pytest.fixture(scope="module")
def coastal600():
    return W.cfg_coastal_tide()


def test_coastal_600k_recipe(coastal600):
    wl = coastal600
    m = wl.mesh
    assert abs(m.n_elems - 600_000) <= 0.02 * 600_000
    assert np.all(_areas(m) > 0.0)
    assert _angles(m).min() > 19.0
    assert m.hb.min() == -2.0 and 2800.0 < m.hb.max() < 3300.0
    # open ocean on x = 0 only, land on the other sides
    ocean = m.bnd[m.bnd_type == W.BC_OCEAN].reshape(-1)
    assert np.all(m.xy[ocean, 0] == 0.0) and np.any(m.bnd_type == W.BC_LAND)
    # grading: fine near the coastline, coarse offshore
    xc = m.meta["xc"]
    cen = m.xy[m.tri].mean(axis=1)
    d = xc(cen[:, 1]) - cen[:, 0]
    size = np.sqrt(2.0 * _areas(m))
    assert np.median(size[np.abs(d) < 2e3]) < 300.0 and np.median(size[cen[:, 0] < 30e3]) > 2000.0
    # forcing: M2 tide of 1 m and Manning 0.025
    f = wl.forcing
    assert f["tide_amp"] == [1.0] and math.isclose(2 * math.pi / f["tide_omega"][0], 44714.0, rel_tol=1e-5)
    assert f["manning_n"] == 0.025 and not f.get("holland")


def test_coastal_mesh_is_seeded():
    a = W.coastal_mesh(8000, W.BASE_SEED + 77, hmin=1000.0, hmax=15000.0)
    b = W.coastal_mesh(8000, W.BASE_SEED + 77, hmin=1000.0, hmax=15000.0)
    c = W.coastal_mesh(8000, W.BASE_SEED + 78, hmin=1000.0, hmax=15000.0)
    assert np.array_equal(a.xy, b.xy) and np.array_equal(a.tri, b.tri) and np.array_equal(a.hb, b.hb)
    assert a.xy.shape != c.xy.shape or not np.array_equal(a.xy, c.xy)


def test_hurricane_track_defaults(coastal600):
    m = coastal600.mesh
    h = W.holland_track(m)
    assert h["holland"] and (h["dp"], h["rmax"], h["pn"]) == (6000.0, 40000.0, 101300.0)
    assert (h["y0"], h["vx"], h["vy"]) == (300e3, 5.0, 0.0)
    assert math.isclose(h["x0"], m.meta["xc"](300e3) - 100e3, rel_tol=1e-12)


def test_serving_requests():
    meshes = [W.coastal_mesh(n, W.BASE_SEED + 900 + i, hmin=1000.0, hmax=15000.0) for i, n in enumerate((3000, 6000))]
    reqs = W.cfg_serving(40, meshes=meshes)
    assert len(reqs) == 40
    arr = [r.arrival for r in reqs]
    assert all(b > a for a, b in zip(arr, arr[1:]))
    assert all(100 <= r.horizon <= 5000 for r in reqs)
    assert {id(r.mesh) for r in reqs} <= {id(m) for m in meshes}
    storms = sum(1 for r in reqs if r.forcing.get("holland"))
    assert 0 < storms < 40
    assert all(0.015 <= r.forcing["manning_n"] <= 0.035 for r in reqs)
    again = W.cfg_serving(40, meshes=meshes)
    assert [(r.arrival, r.horizon) for r in again] == [(r.arrival, r.horizon) for r in reqs]
