"""General meshes and element orderings (host side, no GPU).

* The general-mesh recipe: positive orientation, every relative face
  orientation present, elements traceable to the Kuhn split.
* ``dgw_order_elements``: both methods return permutations, agree with
  independent implementations of their definitions (Morton key by explicit
  bit interleaving; reverse Cuthill-McKee by breadth-first search over the
  oracle's face connectivity) and restore locality on a shuffled mesh.
* The oracle's right-hand side is invariant under relabelling elements,
  vertices and local vertex orders (a property of the method: the
  discretisation depends on the geometry only), which pins the oracle on
  general meshes.
"""

import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W
from oracle import setup as OS
from oracle import solver as O
from paper_2205_11052_amd import _lib, order_elements, permute_mesh

FACE_VERTS = [[a for a in range(4) if a != f] for f in range(4)]


def _neighbour_pairs(mesh):
    EToE, EToF, bc, gid = OS.connectivity(mesh)
    K = EToE.shape[0]
    k = np.repeat(np.arange(K), 4)
    j = EToE.reshape(-1)
    keep = (bc.reshape(-1) == 0) & (k < j)
    return k[keep], j[keep], EToE, EToF, bc


def test_general_mesh_recipe():
    m = W.general_mesh(3, 2.0, seed=4)
    V = m["vxyz"][m["etov"]]
    det = np.einsum("ki,ki->k", V[:, 1] - V[:, 0],
                    np.cross(V[:, 2] - V[:, 0], V[:, 3] - V[:, 0]))
    assert np.all(det > 0)
    # each element is a jittered copy of its Kuhn element: same vertex set
    kuhn = W.kuhn_cube(3, 2.0)
    src = m["vert_from_kuhn"][m["etov"]]
    assert np.array_equal(np.sort(src, axis=1),
                          np.sort(kuhn["etov"][m["elem_from_kuhn"]], axis=1))
    # interior faces meet in all six relative vertex orders
    _, _, EToE, EToF, bc = _neighbour_pairs(m)
    rel = set()
    et = m["etov"]
    for k in range(et.shape[0]):
        for f in range(4):
            if bc[k, f]:
                continue
            k2, f2 = EToE[k, f], EToF[k, f]
            mine = [et[k, a] for a in FACE_VERTS[f]]
            theirs = [et[k2, a] for a in FACE_VERTS[f2]]
            rel.add(tuple(theirs.index(v) for v in mine))
    assert len(rel) == 6
    # boundary tags: 6 n^2 * 2 boundary faces, the top ones free surface
    nb = int((bc > 0).sum())
    assert nb == 2 * 6 * 3 * 3
    top = int((bc == 1).sum())
    assert top == 2 * 3 * 3


def _morton_reference(vxyz, etov):
    """Morton order written out from its definition: centroid, 21-bit grid
    coordinate per axis over the centroids' bounding box, bit b of x, y, z
    to key bits 3b, 3b+1, 3b+2; sort by (key, index)."""
    c = vxyz[etov].mean(axis=1)
    lo, hi = c.min(axis=0), c.max(axis=0)
    top = float((1 << 21) - 1)
    g = np.clip((c - lo) / np.where(hi > lo, hi - lo, 1.0) * top, 0, top)
    g = g.astype(np.uint64)
    keys = []
    for row in g:
        key = 0
        for b in range(21):
            for d in range(3):
                key |= ((int(row[d]) >> b) & 1) << (3 * b + d)
        keys.append(key)
    return np.array(sorted(range(len(keys)), key=lambda i: (keys[i], i)))


def _rcm_reference(mesh):
    """Reverse Cuthill-McKee from its definition over the oracle's face
    connectivity: components started at the minimum (degree, index),
    neighbours queued by (degree, index), the sequence reversed."""
    EToE, _, bc, _ = OS.connectivity(mesh)
    K = EToE.shape[0]
    nbrs = [[int(EToE[k, f]) for f in range(4) if bc[k, f] == 0 and EToE[k, f] != k]
            for k in range(K)]
    deg = [len(x) for x in nbrs]
    seen = [False] * K
    order = []
    for s in sorted(range(K), key=lambda i: (deg[i], i)):
        if seen[s]:
            continue
        seen[s] = True
        queue = [s]
        head = 0
        while head < len(queue):
            k = queue[head]
            head += 1
            new = [j for j in nbrs[k] if not seen[j]]
            for j in new:
                seen[j] = True
            queue.extend(sorted(new, key=lambda i: (deg[i], i)))
        order.extend(queue)
    return np.array(order[::-1])


@pytest.mark.parametrize("n", [2, 5])
def test_morton_matches_definition(n):
    m = W.general_mesh(n, 3.0, seed=n)
    got = order_elements(m["vxyz"], m["etov"], "morton")
    assert np.array_equal(got, _morton_reference(m["vxyz"], m["etov"]))


@pytest.mark.parametrize("n", [2, 5])
def test_rcm_matches_definition(n):
    m = W.general_mesh(n, 3.0, seed=10 + n)
    got = order_elements(m["vxyz"], m["etov"], "rcm")
    assert np.array_equal(got, _rcm_reference(m))


def test_rcm_periodic_identification():
    # periodic Kuhn mesh: every face has a neighbour once vertices are
    # identified, so every element has degree 4
    m = W.kuhn_cube(3, 1.0, periodic=True)
    p = order_elements(m["vxyz"], m["etov"], "rcm", m["vertex_periodic_id"])
    assert sorted(p.tolist()) == list(range(m["etov"].shape[0]))
    assert np.array_equal(p, _rcm_reference(m))


def _mean_gap(mesh):
    k, j, *_ = _neighbour_pairs(mesh)
    return float(np.abs(k - j).mean())


def test_orderings_restore_locality():
    m = W.general_mesh(8, 1.0, seed=2)           # shuffled numbering
    K = m["etov"].shape[0]
    gap_shuffled = _mean_gap(m)
    assert gap_shuffled > K / 5
    for method in ("morton", "rcm"):
        p = order_elements(m["vxyz"], m["etov"], method)
        assert sorted(p.tolist()) == list(range(K))
        gap = _mean_gap(permute_mesh(m, p))
        assert gap < gap_shuffled / 10, (method, gap, gap_shuffled)
        # deterministic
        assert np.array_equal(p, order_elements(m["vxyz"], m["etov"], method))


def test_order_elements_errors():
    lib = _lib.load()
    m = W.general_mesh(2, 1.0, seed=0)
    V = np.ascontiguousarray(m["vxyz"], dtype=np.float64)
    E = np.ascontiguousarray(m["etov"], dtype=np.int32)
    K, nv = E.shape[0], V.shape[0]
    perm = np.empty(K, dtype=np.int64)
    dp = V.ctypes.data_as(C.POINTER(C.c_double))
    ep = E.ctypes.data_as(C.POINTER(C.c_int32))
    pp = perm.ctypes.data_as(C.POINTER(C.c_int64))
    assert lib.dgw_order_elements(nv, dp, K, ep, None, 0, pp) == 0
    assert lib.dgw_order_elements(nv, None, K, ep, None, 0, pp) == -1
    assert lib.dgw_order_elements(nv, dp, K, None, None, 0, pp) == -1
    assert lib.dgw_order_elements(nv, dp, K, ep, None, 0, None) == -1
    assert lib.dgw_order_elements(nv, dp, 0, ep, None, 0, pp) == -1
    assert lib.dgw_order_elements(nv, dp, K, ep, None, 2, pp) == -1
    bad = E.copy()
    bad[0, 0] = nv
    assert lib.dgw_order_elements(nv, dp, K, bad.ctypes.data_as(C.POINTER(C.c_int32)),
                                  None, 0, pp) == -1
    # a degenerate face (repeated vertex) is a mesh error for RCM
    deg = E.copy()
    deg[0, 1] = deg[0, 0]
    assert lib.dgw_order_elements(nv, dp, K, deg.ctypes.data_as(C.POINTER(C.c_int32)),
                                  None, 1, pp) == -3


def _field(x):
    """A smooth state: 9 components, each a different low-degree mix."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    comps = [np.sin(X + 2 * Y) * np.cos(Z), X * Y - Z, np.exp(0.3 * Z) * Y,
             X ** 2 - Y * Z, np.cos(X - Z), Y ** 3 * 0.1 + X, np.sin(Y) * Z,
             X * Z + 0.5, np.cos(2 * Y + Z) * X]
    return np.stack(comps, axis=1)   # [K, 9, Np]


def test_oracle_rhs_invariant_under_relabelling():
    N = 3
    g = W.general_mesh(3, 2.0, seed=7)
    # the same jittered geometry in Kuhn numbering and vertex order
    kuhn = W.kuhn_cube(3, 2.0)
    to_new = np.argsort(g["vert_from_kuhn"])          # old vertex -> new id
    ref = dict(kuhn)
    ref["vxyz"] = g["vxyz"][to_new]
    # a per-element discontinuity (tied to the Kuhn element), so interior
    # faces carry jumps and the flux and neighbour-node mapping are exercised
    jump = np.random.default_rng(3).uniform(-0.5, 0.5, size=(kuhn["etov"].shape[0], 9))
    src = (np.arange(kuhn["etov"].shape[0]), g["elem_from_kuhn"])
    meshes = (ref, g)
    out = []
    for mesh, s in zip(meshes, src):
        P = O.Problem(mesh, N)
        x = W.lattice_node_coords(mesh, N)             # [K, Np, 3]
        f = _field(x) + jump[s][:, :, None] * np.cos(x[..., 0] - 2 * x[..., 2])[:, None, :]
        q = torch.as_tensor(f)
        cen = W.element_centroids(mesh)
        rho = torch.as_tensor(1.0 + 0.1 * cen[:, 2])
        lam = torch.as_tensor(2.0 + 0.2 * cen[:, 0])
        mu = torch.as_tensor(1.0 + 0.1 * cen[:, 1])
        out.append((O.rhs(P, q, rho, lam, mu).numpy(), x))
    (r0, x0), (r1, x1) = out
    e_src = g["elem_from_kuhn"]
    worst = 0.0
    for i in range(r1.shape[0]):
        k = e_src[i]
        # match nodes by physical position
        d = np.linalg.norm(x1[i][:, None, :] - x0[k][None, :, :], axis=2)
        match = d.argmin(axis=1)
        assert np.all(d[np.arange(d.shape[0]), match] < 1e-12)
        worst = max(worst, float(np.abs(r1[i] - r0[k][:, match]).max()))
    scale = float(np.abs(r0).max())
    assert worst <= 1e-12 * scale, (worst, scale)
