"""ctypes binding of the gfx950 library `libdgswe.so` (include/dgswe.h).

Argument marshalling only: every step of the method runs in the HIP kernels.
The functions keep the C names; `Solver` is a thin owner of one handle.
There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# DGSWE_LIB names another build of the same library (e.g. the host-code
# sanitizer build, libdgswe_asan.so)
LIB_PATH = os.environ.get("DGSWE_LIB") or os.path.join(HERE, "libdgswe.so")

DGSWE_OK = 0
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_MESH", 3: "E_NOMEM", 4: "E_DEVICE",
                5: "E_NONFINITE", 6: "E_ALLDRY"}
DGSWE_FP64 = 0
DGSWE_MIXED = 1

EXPORTED = ("dgswe_default_params", "dgswe_create_mesh", "dgswe_set_state", "dgswe_set_forcing",
            "dgswe_step", "dgswe_read_state", "dgswe_destroy", "dgswe_last_error", "dgswe_profile",
            "dgswe_profile_read", "dgswe_mesh_info", "dgswe_create_batch", "dgswe_member_count",
            "dgswe_member_set_state", "dgswe_member_set_forcing", "dgswe_member_read_state",
            "dgswe_member_info", "dgswe_create_pool", "dgswe_prepare_mesh", "dgswe_prepared_free",
            "dgswe_prepared_elems", "dgswe_member_add_prepared", "dgswe_member_add", "dgswe_member_remove",
            "dgswe_pool_usage", "dgswe_use_graphs", "dgswe_member_read_state_device", "dgswe_step_pair")


class dgswe_params(C.Structure):
    _fields_ = [("p", C.c_int32), ("precision", C.c_int32), ("g", C.c_double), ("rho0", C.c_double),
                ("h0", C.c_double), ("cfl", C.c_double), ("dt_fixed", C.c_double), ("dt_max", C.c_double),
                ("limiter", C.c_int32), ("wetdry", C.c_int32), ("rk", C.c_int32), ("flux", C.c_int32),
                ("chunk", C.c_int32), ("waves", C.c_int32), ("persistent", C.c_int32)]


_dp = C.POINTER(C.c_double)


class dgswe_forcing(C.Structure):
    _fields_ = [("manning_n", C.c_double), ("manning_n_elem", _dp), ("n_tide", C.c_int32),
                ("tide_amp", _dp), ("tide_omega", _dp), ("tide_phase", _dp), ("tide_offset", C.c_double),
                ("wind_tau", _dp), ("patm", _dp), ("holland", C.c_int32),
                ("x0", C.c_double), ("y0", C.c_double), ("vx", C.c_double), ("vy", C.c_double),
                ("dp", C.c_double), ("pn", C.c_double), ("rmax", C.c_double), ("B", C.c_double),
                ("rho_air", C.c_double), ("coriolis_f", C.c_double), ("wind_factor", C.c_double),
                ("coriolis", C.c_double), ("rain", C.c_double)]


class dgswe_mesh(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("node_xy", _dp), ("node_hb", _dp), ("n_elems", C.c_int32),
                ("tri", C.POINTER(C.c_int32)), ("n_bnd", C.c_int32), ("bnd_nodes", C.POINTER(C.c_int32)),
                ("bnd_type", C.POINTER(C.c_int32))]


class dgswe_diag(C.Structure):
    _fields_ = [("t", C.c_double), ("dt_last", C.c_double), ("mass", C.c_double), ("volume", C.c_double),
                ("steps", C.c_int64), ("n_wet", C.c_int32), ("n_dry", C.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libdgswe.so (built by paper_2508_21208_amd.build) and declare its ABI."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it with `python -m paper_2508_21208_amd.build` "
                           "(there is no non-HIP fallback)")
    # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7 under
    # the same soname as ROCm's; load it first so libdgswe binds to the same
    # runtime (device memory and streams are shared with torch).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    ip = C.POINTER(C.c_int32)
    vp = C.c_void_p
    L.dgswe_default_params.argtypes = [C.POINTER(dgswe_params)]
    L.dgswe_default_params.restype = None
    L.dgswe_create_mesh.argtypes = [C.c_int32, _dp, _dp, C.c_int32, ip, C.c_int32, ip, ip,
                                    C.POINTER(dgswe_params), vp, C.POINTER(vp)]
    L.dgswe_create_mesh.restype = C.c_int
    L.dgswe_set_state.argtypes = [vp, C.c_double, _dp, C.c_int32]
    L.dgswe_set_state.restype = C.c_int
    L.dgswe_set_forcing.argtypes = [vp, C.POINTER(dgswe_forcing)]
    L.dgswe_set_forcing.restype = C.c_int
    L.dgswe_step.argtypes = [vp, C.c_int32]
    L.dgswe_step.restype = C.c_int
    L.dgswe_read_state.argtypes = [vp, _dp, C.POINTER(dgswe_diag)]
    L.dgswe_read_state.restype = C.c_int
    L.dgswe_destroy.argtypes = [vp]
    L.dgswe_destroy.restype = None
    L.dgswe_last_error.argtypes = [vp]
    L.dgswe_last_error.restype = C.c_char_p
    L.dgswe_profile.argtypes = [vp, C.c_int32]
    L.dgswe_profile.restype = C.c_int
    L.dgswe_profile_read.argtypes = [vp, C.c_int32, C.c_char_p, _dp, C.POINTER(C.c_int64), ip]
    L.dgswe_profile_read.restype = C.c_int
    L.dgswe_mesh_info.argtypes = [vp, C.POINTER(C.c_int64)]
    L.dgswe_mesh_info.restype = C.c_int
    L.dgswe_create_batch.argtypes = [C.c_int32, C.POINTER(dgswe_mesh), C.POINTER(dgswe_params), vp, C.POINTER(vp)]
    L.dgswe_create_batch.restype = C.c_int
    L.dgswe_member_count.argtypes = [vp]
    L.dgswe_member_count.restype = C.c_int32
    L.dgswe_member_set_state.argtypes = [vp, C.c_int32, C.c_double, _dp, C.c_int32]
    L.dgswe_member_set_state.restype = C.c_int
    L.dgswe_member_set_forcing.argtypes = [vp, C.c_int32, C.POINTER(dgswe_forcing)]
    L.dgswe_member_set_forcing.restype = C.c_int
    L.dgswe_member_read_state.argtypes = [vp, C.c_int32, _dp, C.POINTER(dgswe_diag)]
    L.dgswe_member_read_state.restype = C.c_int
    L.dgswe_member_info.argtypes = [vp, C.c_int32, C.POINTER(C.c_int64)]
    L.dgswe_member_info.restype = C.c_int
    L.dgswe_create_pool.argtypes = [C.c_int64, C.c_int32, C.POINTER(dgswe_params), vp, C.POINTER(vp)]
    L.dgswe_create_pool.restype = C.c_int
    L.dgswe_prepare_mesh.argtypes = [C.POINTER(dgswe_mesh), C.POINTER(dgswe_params), C.POINTER(vp)]
    L.dgswe_prepare_mesh.restype = C.c_int
    L.dgswe_prepared_free.argtypes = [vp]
    L.dgswe_prepared_free.restype = None
    L.dgswe_prepared_elems.argtypes = [vp]
    L.dgswe_prepared_elems.restype = C.c_int64
    L.dgswe_member_add_prepared.argtypes = [vp, vp, ip]
    L.dgswe_member_add_prepared.restype = C.c_int
    L.dgswe_member_add.argtypes = [vp, C.POINTER(dgswe_mesh), ip]
    L.dgswe_member_add.restype = C.c_int
    L.dgswe_member_remove.argtypes = [vp, C.c_int32]
    L.dgswe_member_remove.restype = C.c_int
    L.dgswe_pool_usage.argtypes = [vp, C.POINTER(C.c_int64)]
    L.dgswe_pool_usage.restype = C.c_int
    L.dgswe_use_graphs.argtypes = [vp, C.c_int32]
    L.dgswe_use_graphs.restype = C.c_int
    L.dgswe_member_read_state_device.argtypes = [vp, C.c_int32, vp, vp]
    L.dgswe_member_read_state_device.restype = C.c_int
    L.dgswe_step_pair.argtypes = [vp, vp, C.c_int32]
    L.dgswe_step_pair.restype = C.c_int
    _lib = L
    return L


class DgsweError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _d(a):
    return a.ctypes.data_as(_dp)


# ---- C names -----------------------------------------------------------------
def dgswe_default_params() -> dgswe_params:
    p = dgswe_params()
    load_library().dgswe_default_params(C.byref(p))
    return p


def dgswe_create_mesh(xy, hb, tri, bnd, bnd_type, prm: dgswe_params, hip_stream=None):
    L = load_library()
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    hb = np.ascontiguousarray(hb, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    bnd = np.ascontiguousarray(bnd, dtype=np.int32).reshape(-1, 2)
    bt = np.ascontiguousarray(bnd_type, dtype=np.int32)
    ip = C.POINTER(C.c_int32)
    h = C.c_void_p()
    st = L.dgswe_create_mesh(xy.shape[0], _d(xy), _d(hb), tri.shape[0], tri.ctypes.data_as(ip), bnd.shape[0],
                             bnd.ctypes.data_as(ip), bt.ctypes.data_as(ip), C.byref(prm),
                             C.c_void_p(hip_stream) if hip_stream else None, C.byref(h))
    if st != DGSWE_OK:
        raise DgsweError(st, L.dgswe_last_error(None).decode())
    return h


def _mesh_desc(m, keep):
    """dgswe_mesh view of an object with xy, hb, tri, bnd, bnd_type (the
    arrays are appended to `keep`, which must outlive the call)."""
    ip = C.POINTER(C.c_int32)
    xy = np.ascontiguousarray(m.xy, dtype=np.float64)
    hb = np.ascontiguousarray(m.hb, dtype=np.float64)
    tri = np.ascontiguousarray(m.tri, dtype=np.int32)
    bnd = np.ascontiguousarray(m.bnd, dtype=np.int32).reshape(-1, 2)
    bt = np.ascontiguousarray(m.bnd_type, dtype=np.int32)
    keep += [xy, hb, tri, bnd, bt]
    return dgswe_mesh(xy.shape[0], _d(xy), _d(hb), tri.shape[0], tri.ctypes.data_as(ip), bnd.shape[0],
                      bnd.ctypes.data_as(ip), bt.ctypes.data_as(ip))


def dgswe_create_pool(max_elems, max_members, prm: dgswe_params, hip_stream=None):
    L = load_library()
    h = C.c_void_p()
    st = L.dgswe_create_pool(int(max_elems), int(max_members), C.byref(prm),
                             C.c_void_p(hip_stream) if hip_stream else None, C.byref(h))
    if st != DGSWE_OK:
        raise DgsweError(st, L.dgswe_last_error(None).decode())
    return h


def dgswe_prepare_mesh(mesh, prm: dgswe_params):
    """Host-only preprocessing (thread safe; the GIL is released meanwhile)."""
    L = load_library()
    keep = []
    desc = _mesh_desc(mesh, keep)
    h = C.c_void_p()
    st = L.dgswe_prepare_mesh(C.byref(desc), C.byref(prm), C.byref(h))
    if st != DGSWE_OK:
        raise DgsweError(st, L.dgswe_last_error(None).decode())
    return h


def dgswe_prepared_free(h):
    load_library().dgswe_prepared_free(h)


def dgswe_member_add_prepared(h, prep):
    """Returns the member slot; raises DgsweError (status 3) when the pool has
    no room, in which case the caller still owns `prep`."""
    L = load_library()
    slot = C.c_int32(-1)
    _check(h, L.dgswe_member_add_prepared(h, prep, C.byref(slot)))
    return slot.value


def dgswe_member_add(h, mesh):
    L = load_library()
    keep = []
    desc = _mesh_desc(mesh, keep)
    slot = C.c_int32(-1)
    _check(h, L.dgswe_member_add(h, C.byref(desc), C.byref(slot)))
    return slot.value


def dgswe_member_remove(h, member):
    _check(h, load_library().dgswe_member_remove(h, int(member)))


def dgswe_pool_usage(h):
    out = (C.c_int64 * 5)()
    _check(h, load_library().dgswe_pool_usage(h, out))
    return dict(elems_used=out[0], elems_cap=out[1], members=out[2], slots=out[3], device_bytes=out[4])


def dgswe_create_batch(meshes, prm: dgswe_params, hip_stream=None):
    """meshes: objects with xy, hb, tri, bnd, bnd_type (e.g. workloads.Mesh)."""
    L = load_library()
    keep = []
    descs = (dgswe_mesh * len(meshes))()
    for i, m in enumerate(meshes):
        descs[i] = _mesh_desc(m, keep)
    h = C.c_void_p()
    st = L.dgswe_create_batch(len(meshes), descs, C.byref(prm), C.c_void_p(hip_stream) if hip_stream else None,
                              C.byref(h))
    if st != DGSWE_OK:
        raise DgsweError(st, L.dgswe_last_error(None).decode())
    return h


def _check(h, st):
    if st != DGSWE_OK:
        raise DgsweError(st, load_library().dgswe_last_error(h).decode())


def dgswe_set_state(h, t, w, postprocess=False, member=None):
    w = np.ascontiguousarray(w, dtype=np.float64)
    L = load_library()
    if member is None:
        _check(h, L.dgswe_set_state(h, float(t), _d(w), int(bool(postprocess))))
    else:
        _check(h, L.dgswe_member_set_state(h, int(member), float(t), _d(w), int(bool(postprocess))))


HOLLAND_KEYS = ("x0", "y0", "vx", "vy", "dp", "pn", "rmax", "B", "rho_air", "coriolis_f", "wind_factor")


def dgswe_set_forcing(h, f: dict, n_elems: int | None = None, n_nodes: int | None = None, member=None):
    keep = []

    def arr(x, n=None):
        if x is None:
            return None
        a = np.ascontiguousarray(x, dtype=np.float64).ravel()
        if n is not None and a.size != n:
            raise ValueError(f"forcing array of size {a.size}, expected {n}")
        keep.append(a)
        return _d(a)

    amp = f.get("tide_amp", []) or []
    fs = dgswe_forcing()
    fs.manning_n = float(f.get("manning_n", 0.0))
    fs.manning_n_elem = arr(f.get("manning_n_elem"), n_elems)
    fs.n_tide = len(amp)
    fs.tide_amp = arr(amp) if len(amp) else None
    fs.tide_omega = arr(f.get("tide_omega")) if len(amp) else None
    fs.tide_phase = arr(f.get("tide_phase")) if len(amp) else None
    fs.tide_offset = float(f.get("tide_offset", 0.0))
    fs.wind_tau = arr(f.get("wind_tau"), None if n_nodes is None else 2 * n_nodes)
    fs.patm = arr(f.get("patm"), n_nodes)
    fs.holland = int(f.get("holland", 0))
    for k in HOLLAND_KEYS:
        setattr(fs, k, float(f.get(k, 0.0)))
    fs.coriolis = float(f.get("coriolis", 0.0))
    fs.rain = float(f.get("rain", 0.0))
    L = load_library()
    if member is None:
        _check(h, L.dgswe_set_forcing(h, C.byref(fs)))
    else:
        _check(h, L.dgswe_member_set_forcing(h, int(member), C.byref(fs)))


def dgswe_step(h, n_steps):
    _check(h, load_library().dgswe_step(h, int(n_steps)))


def dgswe_step_pair(h1, h2, n_steps):
    _check(h1, load_library().dgswe_step_pair(h1, h2, int(n_steps)))


def dgswe_use_graphs(h, steps_per_graph):
    _check(h, load_library().dgswe_use_graphs(h, int(steps_per_graph)))


def dgswe_read_state(h, w_out=None, diag=True, member=None):
    d = dgswe_diag()
    L = load_library()
    wp = None if w_out is None else _d(w_out)
    dd = C.byref(d) if diag else None
    st = L.dgswe_read_state(h, wp, dd) if member is None else L.dgswe_member_read_state(h, int(member), wp, dd)
    _check(h, st)
    return d


def dgswe_member_read_state_device(h, member, w_dev_ptr, diag_dev_ptr):
    """Enqueue the member's post-processed state and its 8 diagnostics into
    caller-owned device memory (integer addresses, 0 for none) on the
    solver's stream; allocates nothing and does not wait."""
    _check(h, load_library().dgswe_member_read_state_device(h, int(member), C.c_void_p(int(w_dev_ptr) or None),
                                                                C.c_void_p(int(diag_dev_ptr) or None)))


def dgswe_destroy(h):
    if h:
        load_library().dgswe_destroy(h)


def dgswe_profile(h, enable):
    _check(h, load_library().dgswe_profile(h, int(enable)))


def dgswe_profile_read(h, max_kernels=16):
    names = C.create_string_buffer(32 * max_kernels)
    ms = np.zeros(max_kernels)
    n = np.zeros(max_kernels, dtype=np.int64)
    cnt = C.c_int32(0)
    _check(h, load_library().dgswe_profile_read(h, max_kernels, names, _d(ms),
                                                n.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(cnt)))
    out = {}
    for i in range(cnt.value):
        nm = names.raw[32 * i:32 * (i + 1)].split(b"\0")[0].decode()
        out[nm] = (float(ms[i]), int(n[i]))
    return out


def dgswe_mesh_info(h, member=None):
    out = (C.c_int64 * 4)()
    L = load_library()
    st = L.dgswe_mesh_info(h, out) if member is None else L.dgswe_member_info(h, int(member), out)
    _check(h, st)
    return dict(n_nodes=out[0], n_elems=out[1], n_edges=out[2], n_boundary=out[3])


# ---- owner class -------------------------------------------------------------
def params_from_dict(p: dict) -> dgswe_params:
    prm = dgswe_default_params()
    for k, v in p.items():
        if hasattr(prm, k):
            setattr(prm, k, type(getattr(prm, k))(v))
    return prm


def modes_per_variable(params: dict | None) -> int:
    """3 modes per variable at p = 1, 6 at p = 2"""
    return 6 if int((params or {}).get("p", 1)) == 2 else 3


class Solver:
    """One mesh and its device-resident state (shape (3, nm, ne): zeta, Qx,
    Qy, each with nm = 3 (p = 1) or 6 (p = 2) modes)."""

    def __init__(self, mesh, params: dict | None = None, forcing: dict | None = None, hip_stream=None):
        self.h = None
        self.mesh = mesh
        self.ne = int(mesh.tri.shape[0])
        self.nn = int(mesh.xy.shape[0])
        self.nm = modes_per_variable(params)
        self.h = dgswe_create_mesh(mesh.xy, mesh.hb, mesh.tri, mesh.bnd, mesh.bnd_type,
                                   params_from_dict(params or {}), hip_stream)
        if forcing:
            self.set_forcing(forcing)

    def set_forcing(self, f: dict):
        dgswe_set_forcing(self.h, f, self.ne, self.nn)

    def set_state(self, w, t=0.0, postprocess=False):
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(3, self.nm, self.ne)
        dgswe_set_state(self.h, t, w, postprocess)

    def step(self, n=1):
        dgswe_step(self.h, n)

    def use_graphs(self, steps_per_graph):
        dgswe_use_graphs(self.h, steps_per_graph)

    def state(self):
        w = np.empty((3, self.nm, self.ne), dtype=np.float64)
        self.diag = dgswe_read_state(self.h, w)
        return w

    def diagnostics(self):
        d = dgswe_read_state(self.h, None, True)
        return dict(t=d.t, dt_last=d.dt_last, mass=d.mass, volume=d.volume, steps=d.steps,
                    n_wet=d.n_wet, n_dry=d.n_dry)

    def info(self):
        return dgswe_mesh_info(self.h)

    def close(self):
        if self.h:
            dgswe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several independent meshes advanced together (one stage launch for
    all); member i is meshes[i]."""

    def __init__(self, meshes, params: dict | None = None, forcings=None, hip_stream=None):
        self.h = None
        self.meshes = list(meshes)
        self.nm = modes_per_variable(params)
        self.h = dgswe_create_batch(self.meshes, params_from_dict(params or {}), hip_stream)
        for i, f in enumerate(forcings or []):
            if f:
                self.set_forcing(i, f)

    def __len__(self):
        return len(self.meshes)

    def set_forcing(self, i, f: dict):
        m = self.meshes[i]
        dgswe_set_forcing(self.h, f, int(m.tri.shape[0]), int(m.xy.shape[0]), member=i)

    def set_state(self, i, w, t=0.0, postprocess=False):
        ne = int(self.meshes[i].tri.shape[0])
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(3, self.nm, ne)
        dgswe_set_state(self.h, t, w, postprocess, member=i)

    def step(self, n=1):
        dgswe_step(self.h, n)

    def use_graphs(self, steps_per_graph):
        dgswe_use_graphs(self.h, steps_per_graph)

    def state(self, i):
        w = np.empty((3, self.nm, int(self.meshes[i].tri.shape[0])), dtype=np.float64)
        dgswe_read_state(self.h, w, True, member=i)
        return w

    def diagnostics(self, i):
        d = dgswe_read_state(self.h, None, True, member=i)
        return dict(t=d.t, dt_last=d.dt_last, mass=d.mass, volume=d.volume, steps=d.steps,
                    n_wet=d.n_wet, n_dry=d.n_dry)

    def info(self, i=None):
        return dgswe_mesh_info(self.h, i)

    def close(self):
        if self.h:
            dgswe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Ensemble:
    """Members of both polynomial orders advanced together.  A batch holds
    one order (its state layout has one mode count per variable), so the
    ensemble keeps one batch per order present, and dgswe_step_pair
    advances them together (fused=True, the default): per RK stage one
    post-processing launch for the p = 2 members and one stage launch for
    every member of both orders, on the p = 1 batch's stream.  fused=False
    steps the batches in turn.  Member i is
    meshes[i] at order orders[i]; order_params[p] overrides params for the
    batch of order p (e.g. a smaller CFL number at p = 2).  Each member's
    result equals its solo run at its order, bitwise."""

    def __init__(self, meshes, orders, params: dict | None = None, forcings=None, hip_stream=None,
                 order_params: dict | None = None, fused=True):
        self.batches = {}
        self.fused = bool(fused)
        self.where = []  # member -> (order, index in that order's batch)
        meshes = list(meshes)
        orders = [int(o) for o in orders]
        if len(orders) != len(meshes) or any(o not in (1, 2) for o in orders):
            raise DgsweError(1, "one order (1 or 2) per mesh")
        forcings = list(forcings) if forcings else [None] * len(meshes)
        count = {1: 0, 2: 0}
        for o in orders:
            self.where.append((o, count[o]))
            count[o] += 1
        try:
            for p in (1, 2):
                idx = [i for i, o in enumerate(orders) if o == p]
                if idx:
                    prm = dict(params or {}, **((order_params or {}).get(p, {})), p=p)
                    self.batches[p] = Batch([meshes[i] for i in idx], prm, [forcings[i] for i in idx],
                                            hip_stream=hip_stream)
        except Exception:
            self.close()
            raise

    def __len__(self):
        return len(self.where)

    def _member(self, i):
        o, j = self.where[i]
        return self.batches[o], j

    def set_forcing(self, i, f: dict):
        b, j = self._member(i)
        b.set_forcing(j, f)

    def set_state(self, i, w, t=0.0, postprocess=False):
        """w: (3, 3, n_elems) for a p = 1 member, (3, 6, n_elems) for p = 2
        (a (3, 3, n) state given to a p = 2 member fills the linear modes)."""
        b, j = self._member(i)
        w = np.asarray(w, dtype=np.float64)
        if b.nm == 6 and w.shape[1] == 3:
            w6 = np.zeros((3, 6, w.shape[2]))
            w6[:, :3] = w
            w = w6
        b.set_state(j, w, t, postprocess)

    def step(self, n=1):
        if self.fused and len(self.batches) == 2:
            dgswe_step_pair(self.batches[1].h, self.batches[2].h, n)
            return
        for p in sorted(self.batches):
            self.batches[p].step(n)

    def use_graphs(self, steps_per_graph):
        for b in self.batches.values():
            b.use_graphs(steps_per_graph)

    def state(self, i):
        b, j = self._member(i)
        return b.state(j)

    def diagnostics(self, i):
        b, j = self._member(i)
        return b.diagnostics(j)

    def close(self):
        for b in self.batches.values():
            b.close()
        self.batches = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """A serving pool (dgswe_create_pool): members join and leave between
    steps; a member's state has shape (3, nm, its n_elems)."""

    def __init__(self, max_elems, max_members, params: dict | None = None, hip_stream=None):
        self.h = None
        self.params = dict(params or {})
        self.prm = params_from_dict(self.params)
        self.nm = modes_per_variable(params)
        self.h = dgswe_create_pool(max_elems, max_members, self.prm, hip_stream)
        self.ne = {}

    def prepare(self, mesh):
        """host-only preprocessing; returns a handle for add()"""
        return dgswe_prepare_mesh(mesh, self.prm)

    def prepare_with(self, mesh, params: dict):
        """host-only preprocessing with other launch tuning (chunk) than the
        pool's own; order and precision must match the pool's"""
        return dgswe_prepare_mesh(mesh, params_from_dict(params))

    def add(self, mesh=None, prepared=None, forcing=None, w=None, t=0.0, postprocess=False):
        """Admit a mesh (or a prepared handle); returns the member slot.
        Raises DgsweError with status 3 when it does not fit.

        A prepared handle belongs to the pool once the admission itself has
        succeeded; if setting the forcing or the state fails after that, the
        member is removed again and the exception carries
        `prepared_consumed = True` (the caller must not free the handle).
        Any earlier failure leaves the handle with the caller
        (`prepared_consumed = False`)."""
        own = prepared is None
        if own:
            prepared = self.prepare(mesh)
        try:
            slot = dgswe_member_add_prepared(self.h, prepared)
        except DgsweError as e:
            if own:
                dgswe_prepared_free(prepared)
            e.prepared_consumed = False
            raise
        try:
            info = dgswe_mesh_info(self.h, slot)
            self.ne[slot] = info["n_elems"]
            if forcing:
                dgswe_set_forcing(self.h, forcing, info["n_elems"], info["n_nodes"], member=slot)
            if w is not None:
                self.set_state(slot, w, t, postprocess)
        except Exception as e:
            try:
                self.remove(slot)
            finally:
                e.prepared_consumed = True
            raise
        return slot

    def set_state(self, slot, w, t=0.0, postprocess=False):
        w = np.ascontiguousarray(w, dtype=np.float64).reshape(3, self.nm, self.ne[slot])
        dgswe_set_state(self.h, t, w, postprocess, member=slot)

    def remove(self, slot):
        dgswe_member_remove(self.h, slot)
        self.ne.pop(slot, None)

    def step(self, n=1):
        dgswe_step(self.h, n)

    def use_graphs(self, steps_per_graph):
        dgswe_use_graphs(self.h, steps_per_graph)

    def state(self, slot):
        w = np.empty((3, self.nm, self.ne[slot]), dtype=np.float64)
        d = dgswe_read_state(self.h, w, True, member=slot)
        return w, d

    def diagnostics(self, slot):
        d = dgswe_read_state(self.h, None, True, member=slot)
        return dict(t=d.t, dt_last=d.dt_last, mass=d.mass, volume=d.volume, steps=d.steps,
                    n_wet=d.n_wet, n_dry=d.n_dry)

    def usage(self):
        return dgswe_pool_usage(self.h)

    def close(self):
        if self.h:
            dgswe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
