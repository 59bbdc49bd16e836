"""Connectivity, face node maps, affine geometry and point location.

Oracle (test infrastructure).  Textbook nodal-DG mesh bookkeeping
(Hesthaven and Warburton 2008, chapters 3 and 6), stated here in full:

* Faces.  Face f of element k is the face opposite local vertex f.  Its key is
  the sorted triple of the (periodically identified) global ids of its three
  vertices.  Two faces with equal keys are neighbours; a key that occurs more
  than twice is a non-manifold mesh.  An unmatched face takes the boundary tag
  given with the mesh (1 = free surface, 2 = absorbing).
* Face node map.  A face node is identified by its lattice barycentrics
  attached to the global ids of the face's three vertices; the neighbour's node
  is the one carrying the same barycentric on each of the same global ids.
  This is purely combinatorial (no coordinate tolerance).
* Geometry.  X = [v1 - v0, v2 - v0, v3 - v0] / 2 maps the reference element
  (x = v0 + X (r+1, s+1, t+1)); J = det X = volume / (4/3) > 0; the rows of
  X^-1 are grad r, grad s, grad t.  grad l1 = grad r / 2, grad l2 = grad s / 2,
  grad l3 = grad t / 2, grad l0 = -(grad l1 + grad l2 + grad l3); the outward
  unit normal of face f is -grad l_f / |grad l_f|; A_f is the face area from
  the cross product of its edges; Fscale_f = A_f / J.
* Point location.  The barycentrics of x in element k are
  (l1, l2, l3) = (1/2) X^-1 (x - v0), l0 = 1 - l1 - l2 - l3; x belongs to the
  lowest element id whose four barycentrics are all >= -1e-12; its reference
  coordinates are r = 2 l1 - 1, s = 2 l2 - 1, t = 2 l3 - 1.
"""

import numpy as np

from . import refelem


class MeshError(ValueError):
    pass


def _face_vertices():
    return [[a for a in range(4) if a != f] for f in range(4)]


def connectivity(mesh):
    """EToE, EToF [K, 4] (self and own face on boundary faces) and
    bc [K, 4] (0 = interior neighbour, 1 = free surface, 2 = absorbing)."""
    etov = np.asarray(mesh["etov"], dtype=np.int64)
    K = etov.shape[0]
    pid = mesh.get("vertex_periodic_id")
    gid = etov if pid is None else np.asarray(pid, dtype=np.int64)[etov]
    fv = _face_vertices()
    table = {}
    for k in range(K):
        for f in range(4):
            key = tuple(sorted(int(gid[k, a]) for a in fv[f]))
            if len(set(key)) != 3:
                raise MeshError("degenerate face at element %d" % k)
            table.setdefault(key, []).append((k, f))
    EToE = np.repeat(np.arange(K)[:, None], 4, axis=1)
    EToF = np.repeat(np.arange(4)[None, :], K, axis=0)
    bc = np.zeros((K, 4), dtype=np.int64)
    face_bc = np.asarray(mesh["face_bc"], dtype=np.int64)
    for key, lst in table.items():
        if len(lst) > 2:
            raise MeshError("non-manifold face %s" % (key,))
        if len(lst) == 2:
            (k1, f1), (k2, f2) = lst
            EToE[k1, f1], EToF[k1, f1] = k2, f2
            EToE[k2, f2], EToF[k2, f2] = k1, f1
        else:
            k1, f1 = lst[0]
            if face_bc[k1, f1] not in (1, 2):
                raise MeshError("unmatched face without boundary tag")
            bc[k1, f1] = face_bc[k1, f1]
    return EToE, EToF, bc, gid


def face_node_map(N, EToE, EToF, bc, gid):
    """nbr_node[k, f, m]: volume node index, inside element EToE[k, f], of the
    node matching face node m of face f of element k (own node on boundary
    faces)."""
    bary = np.array(refelem.lattice_barycentric(N), dtype=np.int64)
    Fmask = np.array(refelem.face_masks(N), dtype=np.int64)
    K = EToE.shape[0]
    Nfp = Fmask.shape[1]
    # node index from the lattice triple (b1, b2, b3)
    lat_index = -np.ones((N + 1,) * 3, dtype=np.int64)
    for n, b in enumerate(bary):
        lat_index[b[1], b[2], b[3]] = n
    out = np.empty((K, 4, Nfp), dtype=np.int64)
    for f in range(4):
        k2 = EToE[:, f]
        # where2[k, a]: local vertex of the neighbour carrying global id
        # gid[k, a] (-1 where none does, e.g. the vertex opposite the face)
        eq = gid[:, :, None] == gid[k2][:, None, :]           # [K, 4, 4]
        where2 = np.where(eq.any(axis=2), eq.argmax(axis=2), -1)
        b_own = bary[Fmask[f]]                                # [Nfp, 4]
        b2 = np.zeros((K, Nfp, 4), dtype=np.int64)
        for a in range(4):
            if a == f:
                continue
            tgt = where2[:, a]                                # [K]
            interior = bc[:, f] == 0
            if np.any(tgt[interior] < 0):
                raise MeshError("face vertices do not match the neighbour")
            b2[interior, :, tgt[interior]] = b_own[None, :, a]
        nb = lat_index[b2[..., 1], b2[..., 2], b2[..., 3]]    # [K, Nfp]
        out[:, f] = np.where((bc[:, f] == 0)[:, None], nb, Fmask[f][None, :])
    return out


def geometry(mesh):
    """Affine geometry per element: Xinv [K,3,3] (rows grad r, grad s,
    grad t), J [K], normals [K,4,3], area [K,4], Fscale [K,4], volume [K]."""
    V = np.asarray(mesh["vxyz"], dtype=np.float64)[np.asarray(mesh["etov"])]
    X = np.stack([V[:, 1] - V[:, 0], V[:, 2] - V[:, 0], V[:, 3] - V[:, 0]],
                 axis=2) / 2.0                              # columns
    J = np.linalg.det(X)
    if np.any(J <= 0):
        raise MeshError("non-positive Jacobian")
    Xinv = np.linalg.inv(X)
    gl = np.empty((V.shape[0], 4, 3))
    gl[:, 1:4] = Xinv / 2.0
    gl[:, 0] = -(gl[:, 1] + gl[:, 2] + gl[:, 3])
    normals = -gl / np.linalg.norm(gl, axis=2, keepdims=True)
    area = np.empty((V.shape[0], 4))
    for f, vs in enumerate(_face_vertices()):
        a, b, c = V[:, vs[0]], V[:, vs[1]], V[:, vs[2]]
        area[:, f] = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    return dict(Xinv=Xinv, J=J, normals=normals, area=area,
                Fscale=area / J[:, None], volume=J * 4.0 / 3.0, gradl=gl)


def locate(mesh, geo, x, tol=1e-12):
    """(element, reference coordinates) of point x; raises if outside."""
    V = np.asarray(mesh["vxyz"], dtype=np.float64)[np.asarray(mesh["etov"])]
    lam123 = 0.5 * np.einsum("kij,kj->ki", geo["Xinv"], x[None, :] - V[:, 0])
    lam0 = 1.0 - lam123.sum(axis=1)
    ok = np.all(lam123 >= -tol, axis=1) & (lam0 >= -tol)
    idx = np.nonzero(ok)[0]
    if idx.size == 0:
        raise MeshError("point %s outside the mesh" % (x,))
    k = int(idx[0])
    return k, 2.0 * lam123[k] - 1.0


def suggest_dt(geo, rho, lam, mu, N, cfl):
    """dt = cfl * 2 * min_k (r_in,k / cp_k) / (N+1)^2, r_in = 3 V / sum A_f."""
    rin = 3.0 * geo["volume"] / geo["area"].sum(axis=1)
    cp = np.sqrt((np.asarray(lam) + 2.0 * np.asarray(mu)) / np.asarray(rho))
    return float(cfl * 2.0 * np.min(rin / cp) / (N + 1) ** 2)
