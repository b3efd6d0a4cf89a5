"""Pins of the oracle's SSP Runge-Kutta schemes (Eq. RKSSP; the paper names
optimized SSP schemes without coefficients).

Still water over a flat bed with a spatially uniform, time-dependent mass
source s(t): the state stays uniform, every flux and source but s vanishes,
and one step of a Runge-Kutta scheme applied to zeta' = s(t) is the
scheme's quadrature rule: zeta1 = zeta0 + dt sum_i b_i s(t0 + c_i dt), with
the weights b and nodes c of its Butcher form.  SSPRK(3,3) is third order,
so the rule (Simpson's, b = (1/6, 1/6, 2/3), c = (0, 1, 1/2)) integrates a
cubic exactly; SSPRK(s,2) spends dt/(s-1) per Euler stage and averages with
weight 1/s, so b_i = 1/s at c_i = (i-1)/(s-1): exact for a linear s(t), and
off by a closed form for t^2.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_21208_amd import workloads as W


def one_step(rk, src_t, dt=7.0, t0=3.0, p=1):
    m = W.rect_mesh(4, 4, 4000.0, 4000.0, hb=10.0)
    o = O.Oracle(m, W.default_params(dt_fixed=dt, rk=rk), W.default_forcing(), order=p)
    nm = 6 if p == 2 else 3

    def src(t, xy):
        out = np.zeros((3, xy.shape[0]))
        out[0] = src_t(t)
        return out

    o.set_extra_source(src)
    o.set_state(np.zeros((3, nm, o.ne)), t=t0)
    o.step(1)
    w = o.state()
    assert o.t == t0 + dt
    scale = max(1.0, np.abs(w[0, 0]).max())
    # uniform up to rounding: no slope, no flow
    assert np.abs(w[1:]).max() < 1e-13 * scale
    assert np.abs(w[0, 1:]).max() < 1e-15 * scale
    return w[0, 0]


@pytest.mark.parametrize("p", [1, 2])
def test_ssprk33_is_exact_for_a_cubic_source(p):
    cf = (2e-4, -3e-5, 4e-6, -5e-7)
    dt, t0 = 7.0, 3.0

    def s(t):
        return cf[0] + cf[1] * t + cf[2] * t * t + cf[3] * t ** 3

    def S(t):  # antiderivative
        return cf[0] * t + cf[1] * t ** 2 / 2 + cf[2] * t ** 3 / 3 + cf[3] * t ** 4 / 4

    z = one_step(33, s, dt, t0, p)
    assert np.allclose(z, S(t0 + dt) - S(t0), rtol=1e-13, atol=0)
    # and is not exact at degree 4
    z4 = one_step(33, lambda t: 1e-6 * t ** 4, dt, t0, p)
    assert abs(z4[0] - 1e-6 * ((t0 + dt) ** 5 - t0 ** 5) / 5) > 1e-9


def test_ssprk33_stage_times_and_weights():
    c, om, dt, t0 = 1e-3, 0.05, 7.0, 3.0
    z = one_step(33, lambda t: c * math.cos(om * t), dt, t0)
    expect = dt * (c * math.cos(om * t0) / 6 + c * math.cos(om * (t0 + dt)) / 6 +
                   2 * c * math.cos(om * (t0 + dt / 2)) / 3)
    assert np.allclose(z, expect, rtol=1e-13)


@pytest.mark.parametrize("s", [2, 3, 4, 5])
def test_ssprk_s2_equal_weights_at_equal_spacing(s):
    rk = 10 * s + 2
    dt, t0 = 7.0, 3.0
    # exact for a linear source
    z = one_step(rk, lambda t: 2e-4 - 3e-5 * t, dt, t0)
    exact = 2e-4 * dt - 3e-5 * ((t0 + dt) ** 2 - t0 ** 2) / 2
    assert np.allclose(z, exact, rtol=1e-13)
    # t^2 about t0: the rule gives dt^3 (2s-1)/(6(s-1)) for the quadratic part
    z2 = one_step(rk, lambda t: (t - t0) ** 2, dt, t0)
    assert np.allclose(z2, dt ** 3 * (2 * s - 1) / (6 * (s - 1)), rtol=1e-13)
    # a smooth source: the equal-weight rule
    c, om = 1e-3, 0.05
    zc = one_step(rk, lambda t: c * math.cos(om * t), dt, t0)
    expect = dt / s * sum(c * math.cos(om * (t0 + k * dt / (s - 1))) for k in range(s))
    assert np.allclose(zc, expect, rtol=1e-13)


def test_unknown_scheme_rejected():
    m = W.rect_mesh(2, 2, 200.0, 200.0)
    with pytest.raises(O.OracleError):
        O.Oracle(m, W.default_params(rk=23), W.default_forcing())


def test_ssprk_s2_larger_cfl_stays_stable_where_ssprk22_does_not():
    """The SSP coefficient s - 1 of SSPRK(s,2): on the Gaussian hump, CFL 1.2
    (6x the default) blows up with SSPRK(2,2) but stays bounded with
    SSPRK(5,2) (coefficient 4)."""
    wl = W.cfg_gaussian_1600()
    res = {}
    for rk in (22, 52):
        o = O.Oracle(wl.mesh, dict(wl.params, cfl=1.2, rk=rk), wl.forcing)
        o.set_state(wl.w0)
        try:
            o.step(60)
            res[rk] = np.abs(o.state()[0, 0]).max()
        except O.OracleError:
            res[rk] = math.inf
    assert res[52] < 0.2 and not res[22] < 0.2, res
