"""C-ABI checks that need no GPU.

* libdgw.so loads and exports every function declared in include/dgw.h;
* the library's host-side reference operators (Silvester product basis +
  Gauss quadrature in long double) agree with the oracle's exact-rational
  operators to a few ulps -- two independent constructions of one matrix;
* input validation rejects bad meshes, materials and call orders with the
  documented status codes before any device work.
"""

import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import refelem
from paper_2205_11052_amd import _lib
from paper_2205_11052_amd import dgw as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dgw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dgw_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.SIGNATURES)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6])
def test_library_operators_match_oracle(N):
    Dr, Ds, Dt, M, LIFT = D.ref_operators(N)
    ops = refelem.operators(N)
    for a, b in ((Dr, ops["Dr"]), (Ds, ops["Ds"]), (Dt, ops["Dt"]),
                 (M, ops["M"]), (LIFT, ops["LIFT"])):
        scale = np.abs(b).max()
        assert np.max(np.abs(a - b)) <= 8 * np.finfo(float).eps * scale * N
    rst = D.ref_nodes(N)
    lat = np.array(refelem.lattice(N), float)
    assert np.array_equal(rst, -1 + 2 * lat / N)


def _ctx(order=2, precision=64, nshots=1):
    return D.Solver(order, precision, nshots, torch_allocator=False)


def test_create_rejects_bad_arguments():
    lib = _lib.load()
    ctx = C.c_void_p()
    for args in ((0, 64, 1), (7, 64, 1), (3, 16, 1), (3, 64, 0)):
        assert lib.dgw_create(*args, None, C.byref(ctx)) == -1
    assert lib.dgw_create(3, 64, 1, None, None) == -1
    with pytest.raises(D.DGWError) as e:
        D.Solver(9)
    assert e.value.status == "DGW_EINVAL"


def test_mesh_validation_errors():
    mesh = W.kuhn_cube(1, 1.0)
    # negatively oriented element
    s = _ctx()
    bad = mesh["etov"].copy()
    bad[0, [2, 3]] = bad[0, [3, 2]]
    with pytest.raises(D.DGWError) as e:
        s.set_mesh(mesh["vxyz"], bad, None, mesh["face_bc"])
    assert e.value.status == "DGW_EMESH"
    # a face shared by three elements
    s = _ctx()
    et = np.vstack([mesh["etov"], mesh["etov"][:1]])
    bc = np.vstack([mesh["face_bc"], mesh["face_bc"][:1]])
    with pytest.raises(D.DGWError) as e:
        s.set_mesh(mesh["vxyz"], et, None, bc)
    assert e.value.status == "DGW_EMESH"
    # boundary face without a tag
    s = _ctx()
    with pytest.raises(D.DGWError) as e:
        s.set_mesh(mesh["vxyz"], mesh["etov"], None,
                   np.zeros_like(mesh["face_bc"]))
    assert e.value.status == "DGW_EMESH"
    # vertex index out of range
    s = _ctx()
    et = mesh["etov"].copy()
    et[0, 0] = 10 ** 6
    with pytest.raises(D.DGWError) as e:
        s.set_mesh(mesh["vxyz"], et, None, mesh["face_bc"])
    assert e.value.status == "DGW_EMESH"
    # periodic identification that folds a face onto itself (2 cells)
    m2 = W.kuhn_cube(2, 1.0, periodic=True)
    s = _ctx()
    with pytest.raises(D.DGWError) as e:
        s.set_mesh(m2["vxyz"], m2["etov"], m2["vertex_periodic_id"], None)
    assert e.value.status == "DGW_EMESH"


def test_call_order_errors():
    s = _ctx()
    with pytest.raises(D.DGWError) as e:
        s.set_material(np.ones(6), np.ones(6), np.ones(6))
    assert e.value.status == "DGW_ESTATE"
    with pytest.raises(D.DGWError) as e:
        s.step(1)
    assert e.value.status == "DGW_ESTATE"
    with pytest.raises(D.DGWError) as e:
        s.set_dt(-1.0)
    assert e.value.status == "DGW_EINVAL"


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU is present")
def test_valid_mesh_without_gpu_reports_hip_error():
    mesh = W.kuhn_cube(1, 1.0)
    s = _ctx()
    with pytest.raises(D.DGWError) as e:
        s.set_mesh_dict(mesh)
    assert e.value.status == "DGW_EHIP"
