"""ctypes binding of the plain C oracle (test infrastructure only).

The oracle's C source is `dgswe_oracle.c` beside this file; `build_oracle()`
compiles it with gcc -O2 -ffp-contract=off -fopenmp.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dgswe_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_SANITIZE = os.path.join(HERE, "liboracle_asan.so")
# DGSWE_ORACLE_LIB names another build of the oracle (the sanitizer build)
LIB_OVERRIDE = os.environ.get("DGSWE_ORACLE_LIB")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
SOURCE_FN = C.CFUNCTYPE(None, C.c_double, C.c_int32, _dp, _dp, C.c_void_p)


def build_oracle(verbose=False, sanitize=False) -> str:
    """gcc -O2 -ffp-contract=off -fopenmp.  sanitize=True: liboracle_asan.so,
    built by clang under AddressSanitizer + UndefinedBehaviorSanitizer (the
    runtime of the sanitized HIP library's host code) without OpenMP (the
    oracle's results do not depend on its thread count)."""
    if sanitize:
        clang = "/opt/rocm/llvm/bin/clang"
        out = LIB_SANITIZE
        cmd = [clang, "-O1", "-g", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-Wall",
               "-Wno-unused-function", "-Wno-unknown-pragmas", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-shared-libasan", SRC, "-o", out + ".tmp",
               "-lm"]
    else:
        out = LIB
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-Wall", "-Wno-unused-function", SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib = None


def load_oracle():
    global _lib
    if _lib is not None:
        return _lib
    if LIB_OVERRIDE:
        L = C.CDLL(LIB_OVERRIDE)
    else:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build_oracle()
        L = C.CDLL(LIB)
    L.or_create.restype = C.c_void_p
    L.or_create.argtypes = [C.c_int32, _dp, _dp, C.c_int32, _ip, C.c_int32, _ip, _ip, _ip]
    L.or_destroy.argtypes = [C.c_void_p]
    L.or_set_params.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double,
                                C.c_double, C.c_double, C.c_int32, C.c_int32]
    L.or_set_params.restype = C.c_int32
    L.or_set_forcing.argtypes = [C.c_void_p, C.c_double, _dp, C.c_int32, _dp, _dp, _dp, C.c_double,
                                 _dp, _dp, C.c_int32, _dp]
    L.or_set_forcing.restype = C.c_int32
    L.or_set_extra_source.argtypes = [C.c_void_p, SOURCE_FN, C.c_void_p]
    L.or_set_state.argtypes = [C.c_void_p, C.c_double, _dp]
    L.or_set_state.restype = C.c_int32
    L.or_get_state.argtypes = [C.c_void_p, _dp, _dp, _dp, C.POINTER(C.c_int64)]
    L.or_info.argtypes = [C.c_void_p, _ip]
    L.or_geometry.argtypes = [C.c_void_p, _dp, _dp, _ip, _ip, _ip, _dp, _dp, _dp]
    L.or_rhs.argtypes = [C.c_void_p, _dp, C.c_double, _dp]
    L.or_rhs.restype = C.c_int32
    L.or_postprocess.argtypes = [C.c_void_p, _dp, _dp]
    L.or_postprocess.restype = C.c_int32
    L.or_dt_raw.argtypes = [C.c_void_p, _dp]
    L.or_dt_raw.restype = C.c_double
    L.or_step.argtypes = [C.c_void_p, C.c_int32]
    L.or_step.restype = C.c_int32
    L.or_diagnostics.argtypes = [C.c_void_p, _dp, _dp]
    L.or_basis.argtypes = [C.c_double, C.c_double, _dp, _dp]
    L.or_area_rule.argtypes = [_dp, _dp]
    L.or_edge_rule.argtypes = [_dp, _dp]
    L.or_llf.argtypes = [C.c_double, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_int32,
                         C.c_int32, _dp]
    L.or_wall.argtypes = [C.c_double, _dp, C.c_double, C.c_double, C.c_double, C.c_int32, _dp]
    L.or_set_sources.argtypes = [C.c_void_p, C.c_double, C.c_double]
    L.or_set_sources.restype = C.c_int32
    L.or_set_flux.argtypes = [C.c_void_p, C.c_int32]
    L.or_set_flux.restype = C.c_int32
    L.or_roe.argtypes = [C.c_double, _dp, _dp, C.c_double, C.c_double, C.c_double, _dp]
    L.or_set_scheme.argtypes = [C.c_void_p, C.c_int32]
    L.or_set_scheme.restype = C.c_int32
    L.or_set_order.argtypes = [C.c_void_p, C.c_int32]
    L.or_set_order.restype = C.c_int32
    L.or_basis2.argtypes = [C.c_double, C.c_double, _dp, _dp]
    L.or_area_rule2.argtypes = [_dp, _dp]
    L.or_edge_rule2.argtypes = [_dp, _dp]
    L.or_mass2.argtypes = [_dp]
    _lib = L
    return L


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


class OracleError(RuntimeError):
    pass


HOLLAND_KEYS = ("x0", "y0", "vx", "vy", "dp", "pn", "rmax", "B", "rho_air", "coriolis_f", "wind_factor")


class Oracle:
    """One mesh + state, stepped by the plain C oracle."""

    def __init__(self, mesh, params: dict | None = None, forcing: dict | None = None, order: int = 1):
        """order: polynomial degree p (1 or 2); the state is (3, nm, ne) with
        nm = 3 (p = 1) or 6 (p = 2) modes per variable."""
        L = load_oracle()
        self.L = L
        self.mesh = mesh
        self._keep = []
        xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
        hb = np.ascontiguousarray(mesh.hb, dtype=np.float64)
        tri = np.ascontiguousarray(mesh.tri, dtype=np.int32)
        bnd = np.ascontiguousarray(mesh.bnd, dtype=np.int32).reshape(-1, 2)
        bt = np.ascontiguousarray(mesh.bnd_type, dtype=np.int32)
        st = C.c_int32(0)
        h = L.or_create(xy.shape[0], _d(xy), _d(hb), tri.shape[0], _i(tri), bnd.shape[0],
                        _i(bnd) if bnd.size else None, _i(bt) if bt.size else None, C.byref(st))
        if not h:
            raise OracleError(f"or_create failed with status {st.value}")
        self.h = h
        self.status = st.value
        self.ne = tri.shape[0]
        self.nn = xy.shape[0]
        info = np.zeros(4, dtype=np.int32)
        L.or_info(h, _i(info))
        self.ned = int(info[2])
        self.order = int(order)
        self.nm = 6 if self.order == 2 else 3
        if self.order != 1:
            r = L.or_set_order(h, self.order)
            if r:
                raise OracleError(f"or_set_order: {r}")
        if params:
            self.set_params(params)
        if forcing:
            self.set_forcing(forcing)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.L.or_destroy(h)
            self.h = None

    def set_params(self, p: dict):
        r = self.L.or_set_params(self.h, p.get("g", 9.81), p.get("rho0", 1000.0), p.get("h0", 0.01),
                                 p.get("cfl", 0.2), p.get("dt_fixed", 0.0), p.get("dt_max", 0.0),
                                 int(p.get("limiter", 1)), int(p.get("wetdry", 1)))
        if r:
            raise OracleError(f"or_set_params: {r}")
        if int(p.get("limiter", 1)) == 2 and self.order == 2:
            raise OracleError("the vertex-based limiter (limiter = 2) is defined for p = 1 only")
        r = self.L.or_set_scheme(self.h, int(p.get("rk", 22)))
        if r:
            raise OracleError(f"or_set_scheme: {r}")
        r = self.L.or_set_flux(self.h, int(p.get("flux", 0)))
        if r:
            raise OracleError(f"or_set_flux: {r}")

    def set_forcing(self, f: dict):
        me = f.get("manning_n_elem")
        me = None if me is None else np.ascontiguousarray(me, dtype=np.float64)
        amp = np.ascontiguousarray(f.get("tide_amp", []), dtype=np.float64)
        om = np.ascontiguousarray(f.get("tide_omega", []), dtype=np.float64)
        ph = np.ascontiguousarray(f.get("tide_phase", []), dtype=np.float64)
        wt = f.get("wind_tau")
        wt = None if wt is None else np.ascontiguousarray(wt, dtype=np.float64)
        pa = f.get("patm")
        pa = None if pa is None else np.ascontiguousarray(pa, dtype=np.float64)
        hp = np.array([float(f.get(k, 0.0)) for k in HOLLAND_KEYS], dtype=np.float64)
        r = self.L.or_set_forcing(self.h, float(f.get("manning_n", 0.0)), None if me is None else _d(me),
                                  int(amp.size), _d(amp), _d(om), _d(ph), float(f.get("tide_offset", 0.0)),
                                  None if wt is None else _d(wt), None if pa is None else _d(pa),
                                  int(f.get("holland", 0)), _d(hp))
        if r:
            raise OracleError(f"or_set_forcing: {r}")
        self.L.or_set_sources(self.h, float(f.get("coriolis", 0.0)), float(f.get("rain", 0.0)))

    def set_extra_source(self, fn):
        """fn(t, xy (npts,2)) -> array (3, npts): added to s at area points."""
        if fn is None:
            self.L.or_set_extra_source(self.h, SOURCE_FN(0), None)
            return

        def cb(t, npts, xy_p, out_p, ctx):
            xy = np.ctypeslib.as_array(xy_p, shape=(npts, 2))
            out = np.ctypeslib.as_array(out_p, shape=(3, npts))
            out[:] = fn(t, xy)

        cfun = SOURCE_FN(cb)
        self._keep.append(cfun)
        self.L.or_set_extra_source(self.h, cfun, None)

    def set_state(self, w, t=0.0, postprocess=False):
        """postprocess=True applies the stage post-processing (limiter, then
        wet/dry) once to `w` before it becomes the state."""
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(3, self.nm, self.ne)
        if postprocess:
            w = self.postprocess(w)
        self.L.or_set_state(self.h, float(t), _d(w))

    def state(self):
        w = np.empty((3, self.nm, self.ne), dtype=np.float64)
        t = C.c_double(0); dtl = C.c_double(0); s = C.c_int64(0)
        self.L.or_get_state(self.h, _d(w), C.byref(t), C.byref(dtl), C.byref(s))
        self.t, self.dt_last, self.steps = t.value, dtl.value, s.value
        return w

    def step(self, n=1):
        r = self.L.or_step(self.h, int(n))
        if r:
            raise OracleError(f"or_step: status {r}")

    def rhs(self, w, t=0.0):
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(3, self.nm, self.ne)
        dw = np.empty_like(w)
        self.L.or_rhs(self.h, _d(w), float(t), _d(dw))
        return dw

    def postprocess(self, w):
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(3, self.nm, self.ne)
        out = np.empty_like(w)
        self.L.or_postprocess(self.h, _d(w), _d(out))
        return out

    def dt_raw(self, w):
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(3, self.nm, self.ne)
        return float(self.L.or_dt_raw(self.h, _d(w)))

    def diagnostics(self, w=None):
        if w is None:
            w = self.state()
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(3, self.nm, self.ne)
        out = np.zeros(4)
        self.L.or_diagnostics(self.h, _d(w), _d(out))
        return dict(mass=out[0], volume=out[1], n_wet=int(out[2]), n_dry=int(out[3]))

    def geometry(self):
        ne, ned = self.ne, self.ned
        area = np.empty(ne); inr2 = np.empty(ne); nb = np.empty((ne, 3), np.int32)
        ed_el = np.empty((ned, 2), np.int32); ed_type = np.empty(ned, np.int32)
        ed_len = np.empty(ned); ed_n = np.empty((ned, 2)); qxy = np.empty((ne, 6 if self.order == 2 else 3, 2))
        self.L.or_geometry(self.h, _d(area), _d(inr2), _i(nb), _i(ed_el), _i(ed_type), _d(ed_len),
                           _d(ed_n), _d(qxy))
        return dict(area=area, inr2=inr2, el_nb=nb, ed_el=ed_el, ed_type=ed_type, ed_len=ed_len,
                    ed_n=ed_n, qxy=qxy)


def basis(xi, eta):
    L = load_oracle()
    phi = np.zeros(3); dphi = np.zeros(6)
    L.or_basis(float(xi), float(eta), _d(phi), _d(dphi))
    return phi, dphi.reshape(3, 2)


def area_rule():
    L = load_oracle()
    b = np.zeros(9); w = np.zeros(3)
    L.or_area_rule(_d(b), _d(w))
    return b.reshape(3, 3), w


def edge_rule():
    L = load_oracle()
    s = np.zeros(3); w = np.zeros(3)
    L.or_edge_rule(_d(s), _d(w))
    return s, w


def llf(g, wl, wr, hb, n, wetl=1, wetr=1):
    L = load_oracle()
    wl = np.ascontiguousarray(wl, dtype=np.float64); wr = np.ascontiguousarray(wr, dtype=np.float64)
    out = np.zeros(3)
    L.or_llf(g, _d(wl), _d(wr), hb, n[0], n[1], int(wetl), int(wetr), _d(out))
    return out


def roe(g, wl, wr, hb, n):
    L = load_oracle()
    wl = np.ascontiguousarray(wl, dtype=np.float64); wr = np.ascontiguousarray(wr, dtype=np.float64)
    out = np.zeros(3)
    L.or_roe(g, _d(wl), _d(wr), hb, n[0], n[1], _d(out))
    return out


def wall(g, w, hb, n, wet=1):
    L = load_oracle()
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros(3)
    L.or_wall(g, _d(w), hb, n[0], n[1], int(wet), _d(out))
    return out


def holland(params: dict, x, y, t=0.0):
    L = load_oracle()
    L.or_holland_at.argtypes = [_dp, C.c_double, C.c_double, C.c_double, _dp]
    hp = np.array([float(params.get(k, 0.0)) for k in HOLLAND_KEYS], dtype=np.float64)
    out = np.zeros(3)
    L.or_holland_at(_d(hp), float(x), float(y), float(t), _d(out))
    return out


def basis2(xi, eta):
    """p = 2 Dubiner basis values (6,) and reference gradients (6, 2)."""
    L = load_oracle()
    phi = np.zeros(6); dphi = np.zeros(12)
    L.or_basis2(float(xi), float(eta), _d(phi), _d(dphi))
    return phi, dphi.reshape(6, 2)


def area_rule2():
    L = load_oracle()
    b = np.zeros(18); w = np.zeros(6)
    L.or_area_rule2(_d(b), _d(w))
    return b.reshape(6, 3), w


def edge_rule2():
    L = load_oracle()
    s = np.zeros(4); w = np.zeros(4)
    L.or_edge_rule2(_d(s), _d(w))
    return s, w


def mass2():
    L = load_oracle()
    mu = np.zeros(6)
    L.or_mass2(_d(mu))
    return mu
