"""Pins of the oracle's Coriolis and rain sources (Sec. 2.1 source list;
readings: Coriolis f (Qy, -Qx) in wet elements, uniform rain R on zeta)."""
import math

import numpy as np

from oracle import oracle as O
from paper_2508_21208_amd import workloads as W
from test_oracle_pins import _interior_far


def test_coriolis_closed_form():
    # uniform flow on a flat bed: away from walls the flux divergence
    # vanishes and dQ/dt = f (Qy, -Qx) exactly
    m = W.rect_mesh(12, 12, 12000.0, 12000.0, hb=10.0)
    f = 1.0e-4
    o = O.Oracle(m, W.default_params(limiter=0), W.default_forcing(coriolis=f))
    qx, qy = 1.5, -0.7
    w = np.zeros((3, 3, o.ne)); w[0, 0] = 0.2; w[1, 0] = qx; w[2, 0] = qy
    dw = o.rhs(w)
    inner = _interior_far(o, m, 1500.0)
    assert np.allclose(dw[1, 0, inner], f * qy, rtol=1e-12)
    assert np.allclose(dw[2, 0, inner], -f * qx, rtol=1e-12)
    assert np.abs(dw[0, :, inner]).max() < 1e-15
    # the same with p = 2
    o2 = O.Oracle(m, W.default_params(limiter=0), W.default_forcing(coriolis=f), order=2)
    w2 = np.zeros((3, 6, o2.ne)); w2[:, :3] = w
    dw2 = o2.rhs(w2)
    assert np.allclose(dw2[1, 0, inner], f * qy, rtol=1e-12)
    assert np.abs(dw2[1:, 3:, inner]).max() < 1e-14


def test_rain_fills_a_closed_basin_uniformly():
    m = W.rect_mesh(8, 6, 8000.0, 6000.0, hb=5.0)
    R, dt, n = 2.0e-5, 4.0, 50
    o = O.Oracle(m, W.default_params(dt_fixed=dt), W.default_forcing(rain=R))
    o.set_state(np.zeros((3, 3, o.ne)))
    m0 = o.diagnostics()["mass"]
    o.step(n)
    w = o.state()
    assert np.allclose(w[0, 0], R * dt * n, rtol=1e-12)
    assert np.abs(w[0, 1:]).max() < 1e-15 and np.abs(w[1:]).max() < 1e-12
    assert o.diagnostics()["mass"] - m0 == np.float64(o.diagnostics()["mass"] - m0)
    assert math.isclose(o.diagnostics()["mass"] - m0, R * dt * n * 8000.0 * 6000.0, rel_tol=1e-12)


def test_rain_wets_dry_land():
    # bare land 0.5 m above the geoid: rain raises the depth until the
    # elements pass H0 and become wet
    m = W.rect_mesh(4, 4, 400.0, 400.0, hb=-0.5)
    R, dt = 1e-3, 1.0
    w0 = W.state_from_nodal(m.tri, np.full(m.n_nodes, 0.5))  # zeta = -h_b: depth 0
    o = O.Oracle(m, W.default_params(dt_fixed=dt), W.default_forcing(rain=R))
    o.set_state(w0, 0.0, True)
    assert o.diagnostics()["n_wet"] == 0
    o.step(20)
    d = o.diagnostics()
    assert d["n_wet"] == m.n_elems
    assert np.allclose(o.state()[0, 0] - 0.5, R * dt * 20, rtol=1e-12)  # depth zeta + h_b
