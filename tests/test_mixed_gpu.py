"""Mixed-precision path (DGSWE_MIXED) through the C ABI against the FP64 oracle.

The mixed path stores the momentum in FP32 and runs the flux, volume and
source arithmetic in FP32 (zeta, bathymetry, every limiter and wet/dry
operation and the zeta update stay FP64), so it is compared with the FP64
oracle by the accuracy it has to deliver, not bit for bit:
  * elevation at the element vertices within 1e-4 m of the oracle;
  * depth-averaged velocity at element means within 1e-4 m/s of the oracle,
    over elements wet on both sides with mean depth >= 0.5 m;
  * step count and model time as the oracle's (the CFL step is formed in
    FP64 from the stored state, so it matches to rounding);
  * mass conserved to FP64 rounding on a closed basin with wetting and
    drying, bitwise determinism and exact resumption.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2508_21208_amd import workloads as W
from paper_2508_21208_amd.dgswe import DGSWE_MIXED, Solver

from _cases import coastal_600k, coastal_small, hurricane_4m, say, shallow_open_boundary

pytestmark = pytest.mark.gpu

ZETA_TOL = 1e-4   # m
VEL_TOL = 1e-4    # m/s
VEL_MIN_DEPTH = 0.5


def mixed(p):
    return dict(p, precision=DGSWE_MIXED)


def vertex_zeta(w):
    z0, z1, z2 = w[0, 0], w[0, 1], w[0, 2]
    return np.stack([z0 - z1 - z2, z0 + z1 - z2, z0 + 2.0 * z2])


def errors(mesh, wg, wo, h0):
    """max elevation error at the vertices and max velocity error at the
    element means (elements wet in both with mean depth >= VEL_MIN_DEPTH)"""
    ez = np.abs(vertex_zeta(wg) - vertex_zeta(wo)).max()
    hmean = mesh.hb[mesh.tri].mean(axis=1)
    Hg, Ho = wg[0, 0] + hmean, wo[0, 0] + hmean
    ok = (Hg > h0) & (Ho > h0) & (Ho >= VEL_MIN_DEPTH)
    ev = 0.0
    if ok.any():
        for v in (1, 2):
            ev = max(ev, np.abs(wg[v, 0][ok] / Hg[ok] - wo[v, 0][ok] / Ho[ok]).max())
    return ez, ev


def run_mixed_vs_oracle(wl, steps):
    p = mixed(wl.params)
    say(f"{wl.name}: MIXED GPU {steps} steps, ne={wl.mesh.n_elems}")
    s = Solver(wl.mesh, p, wl.forcing)
    s.set_state(wl.w0, 0.0, wl.postprocess_initial)
    s.step(steps)
    wg = s.state()
    dg = s.diagnostics()
    s.close()
    say(f"{wl.name}: FP64 oracle {steps} steps")
    o = Oracle(wl.mesh, wl.params, wl.forcing)
    o.set_state(wl.w0, 0.0, wl.postprocess_initial)
    o.step(steps)
    wo = o.state()
    ez, ev = errors(wl.mesh, wg, wo, wl.params["h0"])
    say(f"{wl.name}: max elevation error {ez:.3e} m, max velocity error {ev:.3e} m/s")
    assert ez <= ZETA_TOL and ev <= VEL_TOL, (ez, ev)
    assert dg["steps"] == o.steps
    assert dg["t"] == pytest.approx(o.t, rel=1e-6)
    return wg, dg, wo, o


def test_mixed_gaussian_hump_1600_200_steps():
    run_mixed_vs_oracle(W.cfg_gaussian_1600(), 200)


def test_mixed_coastal_wetdry_tide_hurricane_200_steps():
    wg, dg, wo, o = run_mixed_vs_oracle(coastal_small(), 200)
    do = o.diagnostics(wo)
    assert dg["n_dry"] > 0 and dg["n_wet"] > 0
    assert abs(dg["n_wet"] - do["n_wet"]) <= 1e-3 * dg["n_wet"]


def test_mixed_shallow_open_boundary():
    wl = shallow_open_boundary()
    run_mixed_vs_oracle(wl, wl.steps)


def test_mixed_coastal_tide_600k_full_size():
    run_mixed_vs_oracle(coastal_600k(), 20)


def test_mixed_hurricane_4m_full_size():
    run_mixed_vs_oracle(hurricane_4m(), 4)


def test_mixed_mass_closed_basin_with_wetdry():
    m = W.rect_mesh(60, 20, 6000.0, 2000.0, hb=lambda x, y: 4.0 - 8.0 * x / 6000.0)
    zn = np.maximum(0.5 * np.exp(-((m.xy[:, 0] - 1500) ** 2 + (m.xy[:, 1] - 1000) ** 2) / 2e5), -m.hb)
    w0 = W.state_from_nodal(m.tri, zn)
    say("MIXED closed basin with a beach, 600 steps")
    s = Solver(m, mixed(W.default_params()), W.default_forcing(manning_n=0.025))
    s.set_state(w0, 0.0, True)
    d0 = s.diagnostics()
    s.step(600)
    d1 = s.diagnostics()
    s.close()
    assert d1["n_dry"] > 0 and d1["n_wet"] > 0
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * d0["volume"]


def test_mixed_lake_at_rest():
    m = W.rect_mesh(40, 20, 20e3, 10e3, hb=lambda x, y: 10 + 5 * np.sin(x / 3e3) * np.cos(y / 2e3))
    # zeta = 0: the hydrostatic term vanishes exactly and the lake stays at rest
    w0 = W.state_from_nodal(m.tri, np.zeros(m.n_nodes))
    s = Solver(m, mixed(W.default_params()), W.default_forcing(manning_n=0.025))
    s.set_state(w0)
    s.step(500)
    w = s.state()
    s.close()
    assert np.abs(w[1:]).max() == 0.0 and np.abs(w[0]).max() == 0.0
    # zeta = 0.3: balance up to FP32 rounding of the flux terms
    w0 = W.state_from_nodal(m.tri, np.full(m.n_nodes, 0.3))
    s = Solver(m, mixed(W.default_params()), W.default_forcing(manning_n=0.025))
    s.set_state(w0)
    d0 = s.diagnostics()
    s.step(500)
    w = s.state()
    d1 = s.diagnostics()
    s.close()
    assert np.abs(w[1:]).max() < 1e-4
    assert np.abs(w[0] - w0[0]).max() < 1e-6
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * d0["volume"]


def test_mixed_state_roundtrip_deterministic_and_resumable():
    wl = coastal_small()
    p = mixed(wl.params)
    say("MIXED: state round trip")
    s = Solver(wl.mesh, p, wl.forcing)
    s.set_state(wl.w0, 0.0, False)
    w = s.state()
    s.close()
    assert np.array_equal(w[0], wl.w0[0])
    assert np.array_equal(w[1:], wl.w0[1:].astype(np.float32).astype(np.float64))
    say("MIXED: determinism, two runs of 60 steps")
    runs = []
    for _ in range(2):
        s = Solver(wl.mesh, p, wl.forcing)
        s.set_state(wl.w0, 0.0, True)
        s.step(60)
        runs.append(s.state())
        s.close()
    assert np.array_equal(runs[0], runs[1])
    say("MIXED: resume after 25 steps")
    s = Solver(wl.mesh, p, wl.forcing)
    s.set_state(wl.w0, 0.0, True)
    s.step(25)
    mid = s.state()
    t_mid = s.diag.t
    s.close()
    s = Solver(wl.mesh, p, wl.forcing)
    s.set_state(mid, t_mid, False)
    s.step(35)
    assert np.array_equal(s.state(), runs[0])
    s.close()
