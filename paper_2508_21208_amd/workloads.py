"""Seeded synthetic inputs for the DG shallow-water step.

This module produces meshes, bathymetry, initial states and forcing
parameters.  It holds none of the step's arithmetic: no flux, quadrature,
limiter, wet/dry rule or time integration lives here.  The only piece of the
discretisation it knows is the coordinate convention of the state that the
library boundary accepts: p=1 modal coefficients in the orthogonal Dubiner
basis (paper Sec. 2.2, Eq. "dubiner"), ordered [phi_00, phi_10, phi_01].  An
initial field given by its nodal values is expressed in those coordinates by
exact linear interpolation (vertex values -> modes), see `modes_from_vertices`.

Workloads stand in for the paper's Hurricane Harvey / TX2008 case (Sec. 6.1),
which is not available: a graded unstructured coastal mesh (fine near the
shoreline, coarse offshore), a tidal open boundary, a moving Holland-model
hurricane, wet/dry land and Manning friction.

Arrays returned:
    xy        (n_nodes, 2) float64  node coordinates [m]
    hb        (n_nodes,)   float64  bathymetry, positive downward [m]
    tri       (n_elems, 3) int32    counter-clockwise node indices
    bnd       (n_bnd, 2)   int32    boundary edges as node pairs
    bnd_type  (n_bnd,)     int32    1 = land (no normal flow), 2 = ocean (elevation)
    w0        (3, 3, n_elems) float64  state [var (zeta, Qx, Qy)][mode][elem]
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 250821208

BC_LAND = 1
BC_OCEAN = 2

G = 9.81
RHO0 = 1000.0
H0 = 0.01
M2_OMEGA = 1.405189e-4  # rad/s, principal lunar semi-diurnal constituent


# --------------------------------------------------------------------------
# state coordinates at the boundary
# --------------------------------------------------------------------------
def modes_from_vertices(v: np.ndarray) -> np.ndarray:
    """Vertex values (..., 3 vertices) -> p=1 Dubiner modes (..., 3 modes).

    The p=1 modes take the values phi_10 = (-1, 1, 0) and phi_01 = (-1, -1, 2)
    at the three reference vertices, so a linear field with vertex values
    (v1, v2, v3) has coefficients u0 = mean(v), u1 = (v2 - v1)/2,
    u2 = (v3 - u0)/2.
    """
    v = np.asarray(v, dtype=np.float64)
    u0 = (v[..., 0] + v[..., 1] + v[..., 2]) / 3.0
    u1 = 0.5 * (v[..., 1] - v[..., 0])
    u2 = 0.5 * (v[..., 2] - u0)
    return np.stack([u0, u1, u2], axis=-1)


def state_from_nodal(tri: np.ndarray, zeta_n, qx_n=None, qy_n=None) -> np.ndarray:
    """Continuous nodal fields -> state array (3, 3, n_elems)."""
    ne = tri.shape[0]
    w = np.zeros((3, 3, ne), dtype=np.float64)
    for m, f in enumerate((zeta_n, qx_n, qy_n)):
        if f is None:
            continue
        f = np.asarray(f, dtype=np.float64)
        w[m] = modes_from_vertices(f[tri]).T
    return w


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
@dataclass
class Mesh:
    xy: np.ndarray
    hb: np.ndarray
    tri: np.ndarray
    bnd: np.ndarray
    bnd_type: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.tri.shape[0])


def rect_mesh(nx: int, ny: int, lx: float, ly: float, hb=10.0,
              types=(BC_LAND, BC_LAND, BC_LAND, BC_LAND)) -> Mesh:
    """nx x ny quads on [0,lx]x[0,ly], each split along its SW->NE diagonal.

    Nodes are numbered row-major from (0,0).  `types` gives the boundary type
    of the (south, east, north, west) sides.  `hb` is a constant or a
    function hb(x, y) evaluated at the nodes.
    """
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    X, Y = np.meshgrid(xs, ys)  # [j][i]
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    nid = lambda i, j: j * (nx + 1) + i  # noqa: E731
    I, J = np.meshgrid(np.arange(nx), np.arange(ny))
    I = I.ravel(); J = J.ravel()
    sw, se, ne_, nw = nid(I, J), nid(I + 1, J), nid(I + 1, J + 1), nid(I, J + 1)
    t1 = np.stack([sw, se, ne_], axis=1)
    t2 = np.stack([sw, ne_, nw], axis=1)
    tri = np.empty((2 * nx * ny, 3), dtype=np.int32)
    tri[0::2] = t1
    tri[1::2] = t2
    bnd, btype = [], []
    for i in range(nx):
        bnd.append((nid(i, 0), nid(i + 1, 0))); btype.append(types[0])
    for j in range(ny):
        bnd.append((nid(nx, j), nid(nx, j + 1))); btype.append(types[1])
    for i in range(nx):
        bnd.append((nid(i + 1, ny), nid(i, ny))); btype.append(types[2])
    for j in range(ny):
        bnd.append((nid(0, j + 1), nid(0, j))); btype.append(types[3])
    if callable(hb):
        hbn = np.asarray(hb(xy[:, 0], xy[:, 1]), dtype=np.float64)
    else:
        hbn = np.full(xy.shape[0], float(hb))
    return Mesh(xy, hbn, tri, np.asarray(bnd, dtype=np.int32),
                np.asarray(btype, dtype=np.int32),
                {"kind": "rect", "nx": nx, "ny": ny, "lx": lx, "ly": ly})


def _coastline(seed: int):
    rng = np.random.default_rng(seed)
    amps = rng.uniform(0.0, 3.0e3, 3)
    waves = rng.integers(2, 13, 3)
    phases = rng.uniform(0.0, 2.0 * np.pi, 3)

    def xc(y):
        y = np.asarray(y, dtype=np.float64)
        out = 270.0e3 + 8.0e3 * np.sin(2.0 * np.pi * y / 120.0e3)
        for a, k, p in zip(amps, waves, phases):
            out = out + a * np.sin(2.0 * np.pi * k * y / 600.0e3 + p)
        return out

    return xc


def _graded_points(gamma, xc, rng, lx, ly, hmin, hmax, jitter=0.12):
    """Points on curves of constant distance d = xc(y) - x from the coast.

    Successive curves are one equilateral row height apart; along a curve the
    spacing is the local target edge length h(d) = clamp(hmin + gamma|d|).
    Every point is jittered by up to `jitter`*h.  Boundary points are laid
    along the four sides with the local spacing.
    """
    def h_of(d):
        return np.clip(hmin + gamma * np.abs(d), hmin, hmax)

    # d-levels: outward from the coastline in both directions
    dmax = 300.0e3 + 20.0e3
    levels = [0.0]
    d = 0.0
    while d < dmax:
        d += h_of(d) * math.sqrt(3.0) / 2.0
        levels.append(d)
    d = 0.0
    while d > -lx:
        d -= h_of(d) * math.sqrt(3.0) / 2.0
        levels.append(d)
    levels = np.sort(np.asarray(levels))
    pts = []
    for idx, dl in enumerate(levels):
        hl = float(h_of(dl))
        n = max(int(math.ceil(ly / hl)), 1)
        off = 0.5 if (idx % 2) else 0.0
        y = (np.arange(n) + off) * (ly / n)
        jit = rng.uniform(-jitter, jitter, size=(n, 2)) * hl
        y = y + jit[:, 1]
        x = xc(y) - dl + jit[:, 0]
        keep = (x > 0.45 * hl) & (x < lx - 0.45 * hl) & (y > 0.45 * hl) & (y < ly - 0.45 * hl)
        if np.any(keep):
            pts.append(np.stack([x[keep], y[keep]], axis=1))
    interior = np.concatenate(pts, axis=0)

    # boundary points with local spacing
    def walk(p0, p1):
        p0 = np.asarray(p0, float); p1 = np.asarray(p1, float)
        L = float(np.hypot(*(p1 - p0)))
        s, out = 0.0, []
        while s < L:
            q = p0 + (p1 - p0) * (s / L)
            out.append(q)
            s += float(h_of(xc(q[1]) - q[0]))
        return out

    b = []
    b += walk((0.0, 0.0), (lx, 0.0))
    b += walk((lx, 0.0), (lx, ly))
    b += walk((lx, ly), (0.0, ly))
    b += walk((0.0, ly), (0.0, 0.0))
    bpts = np.asarray(b)
    return interior, bpts


def coastal_mesh(n_target: int, seed: int, lx=300.0e3, ly=600.0e3,
                 hmin=50.0, hmax=5000.0, h0=H0) -> Mesh:
    """Graded unstructured coastal mesh of about `n_target` triangles.

    Domain [0,lx] (cross-shore) x [0,ly] (alongshore); coastline
    x_c(y) = 270 km + 8 km sin(2 pi y / 120 km) + three seeded modes
    (amplitude <= 3 km).  d = x_c(y) - x is positive offshore.  Target edge
    length h(d) = clamp(50 m + gamma |d|, 50 m, 5 km), gamma found by
    bisection on the point count.  Bathymetry h_b = 3000 m * d / 270 km
    offshore and -2 m * min(1, |d|/30 km) on land (dry).  The x = 0 side is
    the open ocean boundary; the other three sides are land.
    """
    from scipy.spatial import Delaunay

    xc = _coastline(seed)

    def count(gamma):
        rng = np.random.default_rng(seed + 7)
        a, b = _graded_points(gamma, xc, rng, lx, ly, hmin, hmax)
        return 2 * (a.shape[0] + b.shape[0]) - b.shape[0] - 2

    lo, hi = 1e-4, 10.0
    # bisection in log(gamma); the triangle count decreases with gamma
    gamma = None
    for _ in range(40):
        mid = math.sqrt(lo * hi)
        c = count(mid)
        if abs(c - n_target) <= 0.01 * n_target:
            gamma = mid
            break
        if c > n_target:
            lo = mid
        else:
            hi = mid
    if gamma is None:
        gamma = math.sqrt(lo * hi)
    rng = np.random.default_rng(seed + 7)
    interior, bpts = _graded_points(gamma, xc, rng, lx, ly, hmin, hmax)
    pts = np.concatenate([bpts, interior], axis=0)
    dl = Delaunay(pts)
    tri = dl.simplices.astype(np.int64)
    # orient counter-clockwise, drop degenerate slivers on the hull
    p = pts[tri]
    ar = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    neg = ar < 0
    tri[neg] = tri[neg][:, [0, 2, 1]]
    ar = np.abs(ar)
    tri = tri[ar > 1e-6 * hmin * hmin]
    # drop unused points and renumber
    used = np.zeros(pts.shape[0], dtype=bool)
    used[tri.ravel()] = True
    newid = -np.ones(pts.shape[0], dtype=np.int64)
    newid[used] = np.arange(int(used.sum()))
    pts = pts[used]
    tri = newid[tri]
    # boundary edges: edges with exactly one triangle
    e = np.concatenate([tri[:, [1, 2]], tri[:, [2, 0]], tri[:, [0, 1]]], axis=0)
    key = np.minimum(e[:, 0], e[:, 1]) * pts.shape[0] + np.maximum(e[:, 0], e[:, 1])
    uniq, inv, cnt = np.unique(key, return_inverse=True, return_counts=True)
    once = cnt[inv] == 1
    bnd = e[once]
    bx = pts[bnd, 0]
    btype = np.where((bx[:, 0] < 1e-6) & (bx[:, 1] < 1e-6), BC_OCEAN, BC_LAND)
    d = xc(pts[:, 1]) - pts[:, 0]
    hb = np.where(d >= 0.0, 3000.0 * d / 270.0e3, -2.0 * np.minimum(1.0, np.abs(d) / 30.0e3))
    return Mesh(pts.astype(np.float64), hb.astype(np.float64), tri.astype(np.int32),
                bnd.astype(np.int32), btype.astype(np.int32),
                {"kind": "coastal", "n_target": n_target, "seed": seed, "gamma": gamma,
                 "xc": xc, "lx": lx, "ly": ly})


def coastal_initial_state(mesh: Mesh) -> np.ndarray:
    """Sea at rest (zeta = 0) where the bed is below the geoid; bare land
    (zeta = -h_b, no water) above it.  No element starts with its mean depth
    on the wet/dry threshold."""
    zn = np.where(mesh.hb > 0.0, 0.0, -mesh.hb)
    return state_from_nodal(mesh.tri, zn)


# --------------------------------------------------------------------------
# parameter sets
# --------------------------------------------------------------------------
def default_params(**kw) -> dict:
    p = dict(p=1, precision=0, g=G, rho0=RHO0, h0=H0, cfl=0.2, dt_fixed=0.0,
             dt_max=0.0, limiter=1, wetdry=1, rk=22, flux=0, chunk=0, waves=0, persistent=0)
    p.update(kw)
    return p


def default_forcing(**kw) -> dict:
    f = dict(manning_n=0.0, manning_n_elem=None,
             tide_amp=[], tide_omega=[], tide_phase=[], tide_offset=0.0,
             wind_tau=None, patm=None,
             holland=0, x0=0.0, y0=0.0, vx=0.0, vy=0.0, dp=0.0, pn=101300.0,
             rmax=40.0e3, B=1.5, rho_air=1.15, coriolis_f=7.07e-5, wind_factor=0.9,
             coriolis=0.0, rain=0.0)
    f.update(kw)
    return f


def m2_tide(amp=1.0) -> dict:
    """zeta_b(t) = amp * sin(omega t) written as amp * cos(omega t - pi/2)."""
    return dict(tide_amp=[amp], tide_omega=[M2_OMEGA], tide_phase=[-0.5 * np.pi], tide_offset=0.0)


@dataclass
class Workload:
    name: str
    mesh: Mesh
    w0: np.ndarray
    params: dict
    forcing: dict
    steps: int
    # the initial state needs the stage post-processing once (wet/dry
    # fronts cut through elements)
    postprocess_initial: bool = False


def cfg_gaussian_1600(steps=200) -> Workload:
    """Closed 20 km x 10 km basin, 40x20 quads split in two (1,600 elements),
    flat 10 m bed, Gaussian hump (0.1 m, sigma 1 km) at the centre, walls."""
    m = rect_mesh(40, 20, 20.0e3, 10.0e3, hb=10.0)
    x, y = m.xy[:, 0], m.xy[:, 1]
    zn = 0.1 * np.exp(-((x - 10.0e3) ** 2 + (y - 5.0e3) ** 2) / (2.0 * 1.0e3 ** 2))
    w0 = state_from_nodal(m.tri, zn)
    return Workload("gaussian_hump_1600", m, w0, default_params(), default_forcing(), steps)


def cfg_coastal_tide(n_target=600_000, steps=2000, seed=BASE_SEED + 2) -> Workload:
    """Graded coastal mesh, wet/dry land, M2 tide (1 m) on the open boundary,
    Manning n = 0.025."""
    m = coastal_mesh(n_target, seed)
    w0 = coastal_initial_state(m)
    f = default_forcing(manning_n=0.025, **m2_tide(1.0))
    return Workload(f"coastal_tide_{m.n_elems}", m, w0, default_params(), f, steps, True)


def holland_track(mesh: Mesh, speed=5.0, heading=0.0, offshore=100.0e3, y0=300.0e3,
                  dp=6000.0, rmax=40.0e3) -> dict:
    xc = mesh.meta["xc"]
    x0 = float(xc(y0)) - offshore
    return dict(holland=1, x0=x0, y0=y0, vx=speed * math.cos(heading), vy=speed * math.sin(heading),
                dp=dp, pn=101300.0, rmax=rmax, B=1.5, rho_air=1.15, coriolis_f=7.07e-5,
                wind_factor=0.9)


def cfg_hurricane(n_target=4_000_000, steps=1000, seed=BASE_SEED + 3) -> Workload:
    """Graded coastal mesh with a Holland hurricane (60 hPa, Rmax 40 km)
    crossing the shelf at 5 m/s, M2 tide, Manning n = 0.025, wet/dry."""
    m = coastal_mesh(n_target, seed)
    w0 = coastal_initial_state(m)
    f = default_forcing(manning_n=0.025, **m2_tide(1.0), **holland_track(m))
    return Workload(f"hurricane_{m.n_elems}", m, w0, default_params(), f, steps, True)


def cfg_ensemble(n_members=64, n_meshes=8, min_elems=50_000, max_elems=500_000, steps=500,
                 seed=BASE_SEED + 1000) -> list:
    """Storm-surge ensemble: n_members independent coastal solves, each with
    its own Holland track (heading uniform in +-30 degrees about onshore,
    speed 3-8 m/s, start 100-160 km offshore at y 200-400 km, like the
    single hurricane case: a vortex starting over the shallow shelf drives
    1 cm-deep cells through the explicit friction term's stability limit)
    and Manning n uniform in [0.015, 0.035], M2 tide.  The step is capped at
    0.3 s (the paper's fixed step for its hurricane run): on these coarser
    meshes the CFL step reaches 1.8 s, at which the explicit Manning term of
    centimetre-deep cells under hurricane winds exceeds its stability limit
    (g n^2 |Q| dt / H^(7/3) > 2) and the state diverges, in the FP64 oracle
    as on the GPU.  Mesh sizes are uniform in [min_elems, max_elems]; to
    keep generation time bounded the members share n_meshes distinct meshes
    (member i uses mesh i mod n_meshes)."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(min_elems, max_elems + 1, size=n_meshes)
    meshes = [coastal_mesh(int(n), seed + 1 + k, hmin=50.0 if n > 200_000 else 100.0) for k, n in enumerate(sizes)]
    out = []
    for i in range(n_members):
        m = meshes[i % n_meshes]
        heading = float(rng.uniform(-np.pi / 6.0, np.pi / 6.0))
        speed = float(rng.uniform(3.0, 8.0))
        offshore = float(rng.uniform(100e3, 160e3))
        y0 = float(rng.uniform(200e3, 400e3))
        n = float(rng.uniform(0.015, 0.035))
        f = default_forcing(manning_n=n, **m2_tide(1.0),
                            **holland_track(m, speed=speed, heading=heading, offshore=offshore, y0=y0))
        out.append(Workload(f"ensemble_{i}_{m.n_elems}", m, coastal_initial_state(m), default_params(dt_max=0.3), f,
                            steps, True))
    return out


def ensemble_orders(n_members=64, seed=BASE_SEED + 1000 + 999) -> list:
    """The polynomial order of each ensemble member: 1 or 2 with equal
    probability, seeded."""
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.integers(1, 3, size=n_members)]


@dataclass
class Request:
    """One solve request of the serving workload: a mesh, its forcing and
    initial state, a horizon in steps and an arrival time in units of the
    mean inter-arrival gap (scale by 1 / rate)."""
    rid: int
    mesh: Mesh
    forcing: dict
    w0: np.ndarray
    horizon: int
    arrival: float


def serving_meshes(n_meshes=10, min_elems=10_000, max_elems=1_000_000, seed=BASE_SEED + 5000) -> list:
    """The distinct meshes of the serving workload, log-spaced in size from
    min_elems to max_elems (coarser coastlines for the small ones)."""
    sizes = np.geomspace(min_elems, max_elems, n_meshes)
    out = []
    for k, n in enumerate(sizes):
        n = int(round(n))
        if n < 30_000:
            m = coastal_mesh(n, seed + 1 + k, hmin=1000.0, hmax=15000.0)
        elif n < 200_000:
            m = coastal_mesh(n, seed + 1 + k, hmin=200.0)
        else:
            m = coastal_mesh(n, seed + 1 + k, hmin=50.0)
        out.append(m)
    return out


def cfg_serving(n_requests=100, meshes=None, min_steps=100, max_steps=5000, seed=BASE_SEED + 5000) -> list:
    """Serving workload: requests with mesh sizes log-uniform over the
    serving meshes (10k-1M triangles), horizons uniform in [min_steps,
    max_steps], a random forcing (M2 tide of random amplitude, or a Holland
    storm track as in the ensemble), Poisson arrivals (exponential gaps of
    mean 1, to be scaled to the wanted load).  The step is capped at 0.3 s as
    in the ensemble (explicit friction of shallow cells on coarse meshes)."""
    if meshes is None:
        meshes = serving_meshes(seed=seed)
    rng = np.random.default_rng(seed + 1)
    t = 0.0
    out = []
    states = {}
    for i in range(n_requests):
        t += float(rng.exponential(1.0))
        m = meshes[int(rng.integers(0, len(meshes)))]
        if rng.uniform() < 0.5:
            f = default_forcing(manning_n=float(rng.uniform(0.015, 0.035)), **m2_tide(float(rng.uniform(0.5, 1.5))))
        else:
            f = default_forcing(manning_n=float(rng.uniform(0.015, 0.035)), **m2_tide(1.0),
                                **holland_track(m, speed=float(rng.uniform(3.0, 8.0)),
                                                heading=float(rng.uniform(-np.pi / 6.0, np.pi / 6.0)),
                                                offshore=float(rng.uniform(100e3, 160e3)),
                                                y0=float(rng.uniform(200e3, 400e3))))
        if id(m) not in states:
            states[id(m)] = coastal_initial_state(m)
        out.append(Request(i, m, f, states[id(m)], int(rng.integers(min_steps, max_steps + 1)), t))
    return out
