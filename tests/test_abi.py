"""The C ABI library loads and exports every symbol include/dgswe.h declares;
the ctypes structures match the C layout; host-side validation errors are
reported before any device work (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2508_21208_amd import dgswe as D
from paper_2508_21208_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgswe.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dgswe_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("dgswe_create_mesh", "dgswe_set_forcing", "dgswe_step", "dgswe_read_state",
                     "dgswe_set_state", "dgswe_destroy", "dgswe_last_error"):
        assert required in names
    assert set(names) == set(D.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = D.load_library()
    for name in declared_symbols():
        assert hasattr(L, name), name
    nm = subprocess.run(["nm", "-D", "--defined-only", D.LIB_PATH], capture_output=True, text=True).stdout
    for name in declared_symbols():
        assert re.search(rf"\bT {name}$", nm, flags=re.M), name


def test_struct_layouts_match_c(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(f"""
#include <stdio.h>
#include <stddef.h>
#include "{HEADER}"
int main(void) {{
  printf("%zu %zu %zu\\n", sizeof(dgswe_params), sizeof(dgswe_forcing), sizeof(dgswe_diag));
  printf("%zu %zu %zu\\n", offsetof(dgswe_params, wetdry), offsetof(dgswe_forcing, wind_factor),
         offsetof(dgswe_diag, n_dry));
  return 0;
}}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    got = [int(x) for x in out]
    assert got[:3] == [C.sizeof(D.dgswe_params), C.sizeof(D.dgswe_forcing), C.sizeof(D.dgswe_diag)]
    assert got[3] == D.dgswe_params.wetdry.offset
    assert got[4] == D.dgswe_forcing.wind_factor.offset
    assert got[5] == D.dgswe_diag.n_dry.offset


def test_default_params():
    p = D.dgswe_default_params()
    assert (p.p, p.precision, p.g, p.rho0, p.h0, p.cfl, p.dt_fixed, p.limiter, p.wetdry) == \
        (1, 0, 9.81, 1000.0, 0.01, 0.2, 0.0, 1, 1)


def _create(mesh, **kw):
    prm = D.params_from_dict(kw)
    return D.dgswe_create_mesh(mesh.xy, mesh.hb, mesh.tri, mesh.bnd, mesh.bnd_type, prm)


def test_mesh_validation_before_device_work():
    m = W.rect_mesh(3, 2, 3.0, 2.0)
    with pytest.raises(D.DgsweError) as ei:
        _create(W.Mesh(m.xy, m.hb, m.tri[:, [0, 2, 1]].copy(), m.bnd, m.bnd_type))
    assert ei.value.status == 2 and "counter-clockwise" in str(ei.value)
    with pytest.raises(D.DgsweError) as ei:
        _create(W.Mesh(m.xy, m.hb, m.tri, m.bnd[:-1], m.bnd_type[:-1]))
    assert ei.value.status == 2
    with pytest.raises(D.DgsweError) as ei:
        _create(W.Mesh(m.xy, m.hb, m.tri, m.bnd, np.full_like(m.bnd_type, 3)))
    assert ei.value.status == 1  # river boundaries are reserved
    bad = m.tri.copy(); bad[0, 0] = 10_000
    with pytest.raises(D.DgsweError) as ei:
        _create(W.Mesh(m.xy, m.hb, bad, m.bnd, m.bnd_type))
    assert ei.value.status == 2
    # empty and degenerate input
    empty = W.Mesh(m.xy, m.hb, np.zeros((0, 3), np.int32), np.zeros((0, 2), np.int32), np.zeros(0, np.int32))
    with pytest.raises(D.DgsweError) as ei:
        _create(empty)
    assert ei.value.status == 1
    line = W.Mesh(np.array([[0.0, 0.0], [1.0, 0.0], [2.0, 0.0]]), np.ones(3), np.array([[0, 1, 2]], np.int32),
                  np.array([[0, 1], [1, 2], [2, 0]], np.int32), np.ones(3, np.int32))
    with pytest.raises(D.DgsweError) as ei:
        _create(line)  # zero area
    assert ei.value.status == 2
    for field in ("xy", "hb"):
        xy, hb = m.xy.copy(), m.hb.copy()
        (xy if field == "xy" else hb).flat[4] = np.nan
        with pytest.raises(D.DgsweError) as ei:
            _create(W.Mesh(xy, hb, m.tri, m.bnd, m.bnd_type))
        assert ei.value.status == 2 and "non-finite" in str(ei.value), field
    # an edge shared by three triangles
    t3 = np.concatenate([m.tri, m.tri[:1]], axis=0)
    with pytest.raises(D.DgsweError) as ei:
        _create(W.Mesh(m.xy, m.hb, t3, m.bnd, m.bnd_type))
    assert ei.value.status == 2
    for bad_p in (0, 3):
        with pytest.raises(D.DgsweError) as ei:
            _create(m, p=bad_p)
        assert ei.value.status == 1
    with pytest.raises(D.DgsweError) as ei:
        _create(m, h0=-1.0)
    assert ei.value.status == 1
    with pytest.raises(D.DgsweError) as ei:
        _create(m, precision=2)
    assert ei.value.status == 1


def test_batch_validation_before_device_work():
    m = W.rect_mesh(3, 2, 3.0, 2.0)
    bad = W.Mesh(m.xy, m.hb, m.tri[:, [0, 2, 1]].copy(), m.bnd, m.bnd_type)
    with pytest.raises(D.DgsweError) as ei:
        D.dgswe_create_batch([m, bad], D.dgswe_default_params())
    assert ei.value.status == 2 and "mesh 1" in str(ei.value)
    with pytest.raises(D.DgsweError) as ei:
        D.dgswe_create_batch([], D.dgswe_default_params())
    assert ei.value.status == 1
    with pytest.raises(D.DgsweError) as ei:
        D.dgswe_create_batch([m, m], D.params_from_dict(dict(p=3)))
    assert ei.value.status == 1
    # limiter: 0, 1, or 2 (vertex-based, p = 1 only)
    for bad_p in (dict(limiter=3), dict(limiter=-1), dict(limiter=2, p=2)):
        with pytest.raises(D.DgsweError) as ei:
            D.dgswe_create_batch([m, m], D.params_from_dict(bad_p))
        assert ei.value.status == 1, bad_p
    L = D.load_library()
    assert L.dgswe_member_count(None) == 0
    out = (C.c_int64 * 4)()
    assert L.dgswe_member_info(None, 0, out) == 1


def test_prepare_mesh_and_pool_validation_on_host():
    """dgswe_prepare_mesh is host-only work: it runs (and validates) without a
    device; pool capacities are checked before any device work."""
    m = W.rect_mesh(6, 4, 600.0, 400.0)
    L = D.load_library()
    prep = D.dgswe_prepare_mesh(m, D.dgswe_default_params())
    assert L.dgswe_prepared_elems(prep) == m.n_elems
    D.dgswe_prepared_free(prep)
    prep2 = D.dgswe_prepare_mesh(m, D.params_from_dict(dict(p=2)))
    assert L.dgswe_prepared_elems(prep2) == m.n_elems
    D.dgswe_prepared_free(prep2)
    bad = W.Mesh(m.xy, m.hb, m.tri[:, [0, 2, 1]].copy(), m.bnd, m.bnd_type)
    with pytest.raises(D.DgsweError) as ei:
        D.dgswe_prepare_mesh(bad, D.dgswe_default_params())
    assert ei.value.status == 2
    with pytest.raises(D.DgsweError) as ei:
        D.dgswe_prepare_mesh(m, D.params_from_dict(dict(p=3)))
    assert ei.value.status == 1
    for cap, slots in ((0, 4), (1000, 0), (1 << 31, 4)):
        with pytest.raises(D.DgsweError) as ei:
            D.dgswe_create_pool(cap, slots, D.dgswe_default_params())
        assert ei.value.status == 1
    # NULL handles
    out = (C.c_int64 * 5)()
    assert L.dgswe_pool_usage(None, out) == 1
    assert L.dgswe_member_remove(None, 0) == 1
    assert L.dgswe_prepared_elems(None) == 0
    L.dgswe_prepared_free(None)


def test_mesh_whose_chunks_overflow_is_rechunked_not_refused():
    """a valid mesh whose 256-element chunks have more local edges than the
    stage kernel takes (768 > 512: no two triangles share an edge) is
    prepared with smaller chunks instead of being refused"""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from _cases import isolated_triangles
    m = isolated_triangles(700)
    L = D.load_library()
    for prec in (0, 1):
        prep = D.dgswe_prepare_mesh(m, D.params_from_dict(dict(precision=prec)))
        assert L.dgswe_prepared_elems(prep) == m.n_elems
        D.dgswe_prepared_free(prep)


def test_ensemble_order_validation_before_device_work():
    m = W.rect_mesh(3, 2, 3.0, 2.0)
    with pytest.raises(D.DgsweError) as ei:
        D.Ensemble([m, m], [1], {})
    assert ei.value.status == 1
    with pytest.raises(D.DgsweError):
        D.Ensemble([m], [3], {})
    orders = W.ensemble_orders()
    assert len(orders) == 64 and set(orders) == {1, 2} and orders == W.ensemble_orders()
