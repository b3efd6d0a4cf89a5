"""Pins of the oracle's Roe flux (Sec. 2.2 names Roe beside LLF).

* consistency F(w, w, n) = F(w).n;
* the Roe property: with every wave speed of the linearised problem
  positive (negative), the flux is the left (right) physical flux exactly,
  which holds only if the averages and the eigen-decomposition are right;
* antisymmetry and rotation invariance;
* closed form at rest: for zero velocities the dissipation is c dH on the
  mass and c dq_n on the normal momentum (no momentum-jump term in the
  mass flux, unlike LLF);
* lake at rest, mass conservation with wetting and drying, and a Stoker dam
  break that converges under refinement and beats LLF at equal resolution.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_21208_amd import workloads as W
from test_oracle_pins import G, _phys_flux_dot_n, stoker_depth


def rand_state(rng, hb, un_range, ut_range, n):
    ze = rng.uniform(-0.5, 0.5)
    H = ze + hb
    un, ut = rng.uniform(*un_range), rng.uniform(*ut_range)
    u = un * n[0] - ut * n[1]
    v = un * n[1] + ut * n[0]
    return np.array([ze, H * u, H * v])


def test_consistency():
    rng = np.random.default_rng(31)
    for _ in range(50):
        th = rng.uniform(0, 2 * math.pi)
        n = np.array([math.cos(th), math.sin(th)])
        hb = rng.uniform(1.0, 50.0)
        w = rand_state(rng, hb, (-3, 3), (-3, 3), n)
        f = O.roe(G, w, w, hb, n)
        assert np.allclose(f, _phys_flux_dot_n(w, hb, n), rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("sign", [1, -1])
def test_supersonic_is_pure_upwind(sign):
    rng = np.random.default_rng(32 + sign)
    for _ in range(50):
        th = rng.uniform(0, 2 * math.pi)
        n = np.array([math.cos(th), math.sin(th)])
        hb = rng.uniform(0.5, 2.0)
        c = math.sqrt(G * (hb + 0.5))
        lo, hi = sorted((sign * (2 * c + 2), sign * (4 * c + 2)))
        wl = rand_state(rng, hb, (lo, hi), (-3, 3), n)
        wr = rand_state(rng, hb, (lo, hi), (-3, 3), n)
        f = O.roe(G, wl, wr, hb, n)
        up = _phys_flux_dot_n(wl if sign > 0 else wr, hb, n)
        assert np.allclose(f, up, rtol=1e-12, atol=1e-10), (f, up)
        # LLF is not upwind there (a check that the test can fail)
        assert not np.allclose(O.llf(G, wl, wr, hb, n), up, rtol=1e-6)


def test_antisymmetry_and_rotation():
    rng = np.random.default_rng(33)
    for _ in range(50):
        th = rng.uniform(0, 2 * math.pi)
        n = np.array([math.cos(th), math.sin(th)])
        hb = rng.uniform(1.0, 20.0)
        wl = rand_state(rng, hb, (-2, 2), (-2, 2), n)
        wr = rand_state(rng, hb, (-2, 2), (-2, 2), n)
        f = O.roe(G, wl, wr, hb, n)
        g = O.roe(G, wr, wl, hb, -n)
        assert np.allclose(f, -g, rtol=1e-13, atol=1e-12)
        a = rng.uniform(0, 2 * math.pi)
        R = np.array([[math.cos(a), -math.sin(a)], [math.sin(a), math.cos(a)]])
        rot = lambda w: np.array([w[0], *(R @ w[1:])])
        fr = O.roe(G, rot(wl), rot(wr), hb, R @ n)
        assert np.allclose(fr, rot(f), rtol=1e-12, atol=1e-11)


def test_closed_form_at_rest():
    rng = np.random.default_rng(34)
    for _ in range(20):
        n = np.array([0.6, 0.8])
        hb = 10.0
        zl, zr = rng.uniform(-0.3, 0.3, 2)
        qnl, qnr = rng.uniform(-1e-9, 1e-9, 2)  # at rest up to rounding
        wl = np.array([zl, qnl * n[0], qnl * n[1]])
        wr = np.array([zr, qnr * n[0], qnr * n[1]])
        f = O.roe(G, wl, wr, hb, n)
        c = math.sqrt(G * (hb + 0.5 * (zl + zr)))
        fl, fr = _phys_flux_dot_n(wl, hb, n), _phys_flux_dot_n(wr, hb, n)
        assert f[0] == pytest.approx(0.5 * (fl[0] + fr[0]) - 0.5 * c * (zr - zl), rel=1e-9, abs=1e-9)
        pn = 0.5 * (fl[1] * n[0] + fl[2] * n[1] + fr[1] * n[0] + fr[2] * n[1])
        assert f[1] * n[0] + f[2] * n[1] == pytest.approx(pn, rel=1e-9, abs=1e-6)


def test_lake_at_rest_and_mass_with_roe():
    m = W.rect_mesh(20, 10, 20e3, 10e3, hb=lambda x, y: 10 + 5 * np.sin(x / 3e3) * np.cos(y / 2e3))
    w0 = W.state_from_nodal(m.tri, np.full(m.n_nodes, 0.3))
    o = O.Oracle(m, W.default_params(flux=1), W.default_forcing(manning_n=0.025))
    o.set_state(w0)
    o.step(300)
    w = o.state()
    assert np.abs(w[0] - w0[0]).max() < 1e-13 and np.abs(w[1:]).max() < 1e-10
    m = W.rect_mesh(30, 6, 3000.0, 600.0, hb=lambda x, y: 4.0 - x / 500.0)
    zn = np.maximum(np.where(m.hb > 0.01, 0.4 * np.cos(np.pi * m.xy[:, 0] / 3000.0), 0.01 - m.hb), 0.01 - m.hb)
    w0 = W.state_from_nodal(m.tri, zn)
    o = O.Oracle(m, W.default_params(flux=1), W.default_forcing(manning_n=0.02))
    w0 = o.postprocess(w0)
    o.set_state(w0)
    m0 = o.diagnostics(w0)["mass"]
    for _ in range(6):
        o.step(50)
        d = o.diagnostics()
        assert abs(d["mass"] - m0) / abs(m0) < 1e-12


def _dam_break_error(nx, flux):
    hl, hr, x0, T = 10.0, 1.0, 1000.0, 30.0
    m = W.rect_mesh(nx, 2, 2000.0, 2000.0 / nx * 2, hb=0.0)
    c = m.xy[m.tri].mean(axis=1)[:, 0]
    w0 = np.zeros((3, 3, m.n_elems))
    w0[0, 0] = np.where(c < x0, hl, hr)
    o = O.Oracle(m, W.default_params(cfl=0.2, flux=flux), W.default_forcing())
    o.set_state(w0)
    while True:
        w = o.state()
        if o.t >= T - 1e-9:
            break
        dt = 0.2 * o.dt_raw(w)
        if o.t + dt > T:
            o.set_params(W.default_params(dt_fixed=T - o.t, flux=flux))
        o.step(1)
    return np.mean(np.abs(o.state()[0, 0] - stoker_depth(c, T, x0, hl, hr)))


def test_stoker_dam_break_with_roe():
    errs = [_dam_break_error(nx, 1) for nx in (50, 100, 200)]
    assert errs[1] < errs[0] and errs[2] < errs[1], errs
    assert errs[2] < 0.05, errs
    assert errs[2] <= _dam_break_error(200, 0) * 1.02
