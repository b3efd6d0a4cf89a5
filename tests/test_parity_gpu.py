"""Parity of the HIP step (through the C ABI) against the FP64 oracle.

Bar: relative L2 difference <= 1e-12 per variable after N steps (FP64 on
both sides; the two differ only in the rounding of sums that are ordered
differently).  Integer results (step counts, wet/dry counts) must be equal.
"""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.dgswe import DgsweError, Solver

from _cases import (coastal_600k, coastal_small, exact_mass, hurricane_4m, isolated_triangles, rel_l2, say,
                    shallow_open_boundary)

pytestmark = pytest.mark.gpu

TOL = 1e-12


def run_both(wl, steps, params=None, forcing=None):
    p = dict(wl.params, **(params or {}))
    f = dict(wl.forcing, **(forcing or {}))
    say(f"{wl.name}: GPU {steps} steps, ne={wl.mesh.n_elems}")
    s = Solver(wl.mesh, p, f)
    s.set_state(wl.w0, 0.0, wl.postprocess_initial)
    s.step(steps)
    wg = s.state()
    dg = s.diagnostics()
    s.close()
    say(f"{wl.name}: oracle {steps} steps")
    o = Oracle(wl.mesh, p, f)
    o.set_state(wl.w0, 0.0, wl.postprocess_initial)
    o.step(steps)
    wo = o.state()
    return wg, dg, wo, o


def check(wg, dg, wo, o, tol=TOL, qscale=None):
    """qscale: momentum scale for states whose momentum is a near-cancellation
    of much larger pressure terms (the momentum error is then measured
    against max(|Q|, qscale) instead of |Q|)."""
    err = rel_l2(wg, wo)
    if qscale is not None:
        for v in (1, 2):
            err[v] = np.linalg.norm(wg[v] - wo[v]) / max(np.linalg.norm(wo[v]), qscale)
    assert max(err) <= tol, err
    assert dg["steps"] == o.steps
    assert dg["t"] == pytest.approx(o.t, rel=1e-12)
    do = o.diagnostics(wo)
    assert dg["mass"] == pytest.approx(exact_mass(o, wo), rel=1e-12, abs=1e-6)
    assert dg["volume"] == pytest.approx(do["volume"], rel=1e-12)
    assert dg["n_wet"] == do["n_wet"] and dg["n_dry"] == do["n_dry"]
    return err


def test_gaussian_hump_1600_200_steps():
    wl = W.cfg_gaussian_1600()
    wg, dg, wo, o = run_both(wl, 200)
    err = check(wg, dg, wo, o)
    say(f"rel L2 {err}")
    assert dg["t"] == pytest.approx(1179.78, abs=0.5)


def test_coastal_wetdry_tide_hurricane_200_steps():
    wl = coastal_small()
    wg, dg, wo, o = run_both(wl, 200)
    err = check(wg, dg, wo, o)
    assert dg["n_dry"] > 0 and dg["n_wet"] > 0
    say(f"rel L2 {err}")


def test_coastal_tide_600k_full_size():
    wl = coastal_600k()
    assert abs(wl.mesh.n_elems - 600_000) < 0.02 * 600_000
    wg, dg, wo, o = run_both(wl, 20)
    err = check(wg, dg, wo, o)
    say(f"rel L2 {err}")


def test_hurricane_4m_full_size():
    wl = hurricane_4m()
    assert abs(wl.mesh.n_elems - 4_000_000) < 0.02 * 4_000_000
    wg, dg, wo, o = run_both(wl, 4)
    err = check(wg, dg, wo, o)
    say(f"rel L2 {err}")


def test_shallow_open_boundary_ghost_wets_and_dries():
    """the ocean ghost's dry branch: a tide that takes the ghost's depth
    above and below H0 over a bed at -0.015 m along the open boundary"""
    wl = shallow_open_boundary()
    wg, dg, wo, o = run_both(wl, wl.steps)
    err = check(wg, dg, wo, o)
    say(f"rel L2 {err}")


def test_rechunked_mesh_of_isolated_triangles():
    """a mesh the default 256-element chunks cannot take (no two triangles
    share an edge, 768 edges per chunk): prepared with smaller chunks, its
    700 sloshing basins match the oracle"""
    m = isolated_triangles(700)
    zn = 0.2 * np.sin(m.xy[:, 0] / 70.0) * np.cos(m.xy[:, 1] / 90.0)
    wl = W.Workload("isolated_700", m, W.state_from_nodal(m.tri, zn), W.default_params(),
                    W.default_forcing(manning_n=0.02), 100)
    wg, dg, wo, o = run_both(wl, 100)
    # each closed basin's momentum decays tenfold every 10 steps (the wall
    # flux damps it) to ~1e-10 of its size after the first steps, the
    # residue of wall pressure terms of O(10) that cancel: its error is
    # measured against that early momentum scale (L2 norm ~0.1), not
    # against the residue
    check(wg, dg, wo, o, qscale=1e-2)
    # the mixed path (smaller LDS per chunk, chunked on its own) within its bar
    s = Solver(m, dict(wl.params, precision=1), wl.forcing)
    s.set_state(wl.w0)
    s.step(100)
    wm = s.state()
    s.close()
    V = np.array([[1.0, -1.0, -1.0], [1.0, 1.0, -1.0], [1.0, 0.0, 2.0]])
    assert np.abs(V @ (wm[0] - wo[0])).max() <= 1e-4


def test_bitwise_deterministic_and_resumable():
    wl = coastal_small()
    say("determinism: two runs of 60 steps")
    runs = []
    for _ in range(2):
        s = Solver(wl.mesh, wl.params, wl.forcing)
        s.set_state(wl.w0, 0.0, True)
        s.step(60)
        runs.append(s.state())
        s.close()
    assert np.array_equal(runs[0], runs[1])
    say("resume: 25 steps, read, set, 35 steps")
    s = Solver(wl.mesh, wl.params, wl.forcing)
    s.set_state(wl.w0, 0.0, True)
    s.step(25)
    mid = s.state()
    t_mid = s.diag.t
    s.close()
    s = Solver(wl.mesh, wl.params, wl.forcing)
    s.set_state(mid, t_mid, False)
    s.step(35)
    assert np.array_equal(s.state(), runs[0])
    s.close()


def test_element_order_does_not_matter():
    wl = coastal_small()
    rng = np.random.default_rng(3)
    perm = rng.permutation(wl.mesh.n_elems)
    m = wl.mesh
    mp = W.Mesh(m.xy, m.hb, m.tri[perm], m.bnd, m.bnd_type, m.meta)
    say("permuted element order, 50 steps")
    a = Solver(m, wl.params, wl.forcing); a.set_state(wl.w0, 0.0, True); a.step(50); wa = a.state(); a.close()
    b = Solver(mp, wl.params, wl.forcing); b.set_state(wl.w0[:, :, perm], 0.0, True); b.step(50)
    wb = b.state(); b.close()
    assert max(rel_l2(wb, wa[:, :, perm])) <= TOL


@pytest.mark.parametrize("nx,ny", [(1, 1), (3, 1), (16, 8), (17, 15), (129, 2)])
def test_ragged_small_meshes(nx, ny):
    """tiny meshes and element counts that leave ragged final blocks
    (2, 6, 256, 510, 516 elements).  On the smallest meshes the walls hold the
    water almost still and |Q| is ~1e-6 of the pressure-flux scale, so the
    momentum error is measured against sqrt(g H) |zeta|."""
    m = W.rect_mesh(nx, ny, 100.0 * nx, 100.0 * ny, hb=lambda x, y: 5.0 + 0.001 * x)
    zn = 0.05 * np.sin(m.xy[:, 0] / 150.0) + 0.02 * np.cos(m.xy[:, 1] / 90.0)
    w0 = W.state_from_nodal(m.tri, zn)
    wl = W.Workload(f"rect_{nx}x{ny}", m, w0, W.default_params(), W.default_forcing(manning_n=0.02), 30)
    wg, dg, wo, o = run_both(wl, 30)
    qscale = np.sqrt(9.81 * 5.5) * np.linalg.norm(w0[0])
    check(wg, dg, wo, o, qscale=qscale)


def test_switches_fixed_dt_cap_and_static_forcing():
    wl = coastal_small()
    m = wl.mesh
    rng = np.random.default_rng(9)
    tau = np.zeros((m.n_nodes, 2)); tau[:, 0] = 0.5; tau[:, 1] = -0.2
    patm = 101300.0 + 1e-3 * m.xy[:, 0]
    nel = rng.uniform(0.015, 0.035, m.n_elems)
    base = dict(wl.forcing, holland=0, wind_tau=tau, patm=patm, manning_n_elem=nel)
    for params in (dict(dt_fixed=0.5), dict(dt_max=0.4), dict(limiter=0), dict(cfl=0.3, limiter=0)):
        wg, dg, wo, o = run_both(wl, 40, params=params, forcing=base)
        check(wg, dg, wo, o)


def test_wetdry_off_on_deep_water():
    m = W.rect_mesh(20, 10, 2000.0, 1000.0, hb=lambda x, y: 30.0 + 0.01 * x)
    zn = 0.3 * np.exp(-((m.xy[:, 0] - 700.0) ** 2 + (m.xy[:, 1] - 500.0) ** 2) / 2e4)
    wl = W.Workload("deep", m, W.state_from_nodal(m.tri, zn), W.default_params(wetdry=0),
                    W.default_forcing(manning_n=0.03), 50)
    wg, dg, wo, o = run_both(wl, 50)
    check(wg, dg, wo, o)


def test_lake_at_rest_and_mass_on_gpu():
    m = W.rect_mesh(40, 20, 20e3, 10e3, hb=lambda x, y: 10 + 5 * np.sin(x / 3e3) * np.cos(y / 2e3))
    w0 = W.state_from_nodal(m.tri, np.full(m.n_nodes, 0.3))
    say("lake at rest, 500 steps")
    s = Solver(m, W.default_params(), W.default_forcing(manning_n=0.025))
    s.set_state(w0)
    d0 = s.diagnostics()
    s.step(500)
    w = s.state()
    d1 = s.diagnostics()
    s.close()
    assert np.abs(w[1:]).max() < 1e-10
    assert abs(d1["mass"] - d0["mass"]) <= 1e-12 * abs(d0["mass"])


def test_all_dry_domain_reports_error():
    m = W.rect_mesh(4, 4, 400.0, 400.0, hb=-1.0)  # land everywhere, no water
    w0 = W.state_from_nodal(m.tri, np.full(m.n_nodes, 1.0))  # zeta = -h_b: depth 0
    say("all dry")
    s = Solver(m, W.default_params(), W.default_forcing())
    s.set_state(w0, 0.0, True)
    s.step(3)
    with pytest.raises(DgsweError) as ei:
        s.state()
    assert ei.value.status == 6
    s.close()
    # with a dt cap the dry domain just sits still
    s = Solver(m, W.default_params(dt_max=1.0), W.default_forcing())
    s.set_state(w0, 0.0, True)
    s.step(3)
    d = s.diagnostics()
    assert d["steps"] == 3 and d["n_dry"] == m.n_elems and d["t"] == pytest.approx(3.0)
    s.close()


def test_nonfinite_state_reports_error():
    wl = W.cfg_gaussian_1600()
    w = wl.w0.copy()
    w[1, 0, 100] = math.nan
    say("NaN in the state")
    s = Solver(wl.mesh, wl.params, dict(wl.forcing))
    s.set_state(w, 0.0, False)
    s.step(2)
    with pytest.raises(DgsweError) as ei:
        s.state()
    assert ei.value.status == 5
    s.close()
