"""Pins of the input meshes and of the oracle's geometry and connectivity."""

import numpy as np
import pytest

import workloads as W
from oracle import refelem, setup


@pytest.mark.parametrize("n,L,periodic", [(1, 1.0, False), (2, 3.0, False),
                                          (3, 1.0, True), (4, 10.0, False)])
def test_kuhn_volumes_and_faces(n, L, periodic):
    mesh = W.kuhn_cube(n, L, periodic=periodic)
    geo = setup.geometry(mesh)
    assert abs(geo["volume"].sum() - L ** 3) < 1e-12 * L ** 3
    assert np.allclose(geo["volume"], (L / n) ** 3 / 6.0)
    EToE, EToF, bc, gid = setup.connectivity(mesh)
    K = EToE.shape[0]
    interior = bc == 0
    # reciprocity of the face pairing
    k2, f2 = EToE[interior], EToF[interior]
    kk, ff = np.nonzero(interior)
    assert np.all(EToE[k2, f2] == kk) and np.all(EToF[k2, f2] == ff)
    assert np.all(k2 != kk)
    nbnd = np.count_nonzero(~interior)
    assert nbnd == (0 if periodic else 12 * n * n)
    if not periodic:
        # free surface exactly on the top face
        V = mesh["vxyz"][mesh["etov"]]
        for k, f in zip(*np.nonzero(bc == 1)):
            z = V[k, [a for a in range(4) if a != f], 2]
            assert np.allclose(z, L)
        assert np.count_nonzero(bc == 1) == 2 * n * n


@pytest.mark.parametrize("n", [1, 2])
def test_geometry_identities(n):
    mesh = W.kuhn_cube(n, 2.0)
    # a randomly perturbed interior vertex keeps the mesh valid and generic
    rng = np.random.default_rng(1)
    mesh["vxyz"] = mesh["vxyz"] + 0.05 * rng.standard_normal(mesh["vxyz"].shape)
    geo = setup.geometry(mesh)
    gl = np.linalg.norm(geo["gradl"], axis=2)
    assert np.allclose(gl, geo["area"] / (3 * geo["volume"][:, None]),
                       rtol=1e-13)
    closure = np.einsum("kf,kfc->kc", geo["area"], geo["normals"])
    assert np.max(np.abs(closure)) < 1e-13
    # outward: normal points away from the opposite vertex
    V = mesh["vxyz"][mesh["etov"]]
    for f in range(4):
        face_pt = V[:, [a for a in range(4) if a != f]].mean(1)
        assert np.all(np.einsum("kc,kc->k", geo["normals"][:, f],
                                face_pt - V[:, f]) > 0)


@pytest.mark.parametrize("periodic,n", [(False, 2), (True, 3)])
@pytest.mark.parametrize("N", [1, 3, 4])
def test_face_node_map_geometric(periodic, n, N):
    L = 1.0
    mesh = W.kuhn_cube(n, L, periodic=periodic)
    EToE, EToF, bc, gid = setup.connectivity(mesh)
    nb = setup.face_node_map(N, EToE, EToF, bc, gid)
    x = W.lattice_node_coords(mesh, N)                    # [K, Np, 3]
    Fm = np.array(refelem.face_masks(N))
    for f in range(4):
        own = x[:, Fm[f]]                                 # [K, Nfp, 3]
        oth = x[EToE[:, f][:, None], nb[:, f]]
        d = oth - own
        if periodic:
            # equal modulo the period in each coordinate
            d = d - L * np.round(d / L)
        assert np.max(np.abs(d)) < 1e-13


def test_nonmanifold_and_missing_tags_rejected():
    mesh = W.kuhn_cube(1, 1.0)
    bad = dict(mesh)
    bad["etov"] = np.vstack([mesh["etov"], mesh["etov"][:1]])
    bad["face_bc"] = np.vstack([mesh["face_bc"], mesh["face_bc"][:1]])
    with pytest.raises(setup.MeshError):
        setup.connectivity(bad)
    bad = dict(mesh)
    bad["face_bc"] = np.zeros_like(mesh["face_bc"])
    with pytest.raises(setup.MeshError):
        setup.connectivity(bad)


def test_point_location_tie_break_and_dt():
    mesh = W.kuhn_cube(2, 1.0)
    geo = setup.geometry(mesh)
    # the cube centre is a vertex shared by many tetrahedra: lowest id wins
    k, rst = setup.locate(mesh, geo, np.array([0.5, 0.5, 0.5]))
    V = mesh["vxyz"][mesh["etov"]]
    owners = [kk for kk in range(len(V))
              if np.any(np.all(np.isclose(V[kk], 0.5), axis=1))]
    assert k == min(owners)
    with pytest.raises(setup.MeshError):
        setup.locate(mesh, geo, np.array([1.5, 0.5, 0.5]))
    # inradius of the Kuhn tetrahedron: h / (2 (1 + sqrt 2))
    rho, lam, mu = W.homogeneous_medium(len(V))
    dt = setup.suggest_dt(geo, rho, lam, mu, 3, 0.5)
    rin = 0.5 / (2 * (1 + np.sqrt(2)))
    assert abs(dt - 0.5 * 2 * rin / np.sqrt(3) / 16) < 1e-15
