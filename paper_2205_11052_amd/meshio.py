"""Tetrahedral meshes from and to files: Gmsh's MSH 2.2 ASCII format.

Read: 4-node tetrahedra (element type 4) and 3-node triangles (type 2) whose
first tag (the physical group) names a boundary condition through
``bc_map`` {physical id: 1 free surface | 2 absorbing}; a boundary face with
no tagged triangle (or a tag not in the map) gets ``default_bc``.  Node ids
may be any positive integers (renumbered densely in file order).  A
negatively oriented tetrahedron has its last two vertices swapped (which
keeps its face set).  Other element types are ignored.

Write: the mesh's vertices, its tetrahedra, and one triangle per boundary
face carrying the physical id ``bc_physical[face_bc]`` (defaults 1 for free
surface, 2 for absorbing), so a written mesh reads back with
``bc_map = {1: 1, 2: 2}``.

The returned dict has the keys ``dgw_set_mesh`` takes (``vxyz``, ``etov``,
``vertex_periodic_id`` (None), ``face_bc``).  Host-side I/O only.
"""

import numpy as np

FACE_VERTS = ((1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2))   # face f opposite v f


def _sections(lines):
    out, name, body = {}, None, []
    for ln in lines:
        s = ln.strip()
        if s.startswith("$End"):
            out[name] = body
            name, body = None, []
        elif s.startswith("$"):
            name, body = s[1:], []
        elif name is not None:
            body.append(s)
    return out


def _boundary_faces(etov):
    """(element, face) pairs of faces that no other element shares, and
    their sorted vertex triples."""
    K = etov.shape[0]
    tri = np.sort(etov[:, FACE_VERTS], axis=2).reshape(K * 4, 3)
    keys, inv, cnt = np.unique(tri, axis=0, return_inverse=True, return_counts=True)
    inv = inv.reshape(-1)
    single = cnt[inv] == 1
    idx = np.nonzero(single)[0]
    return idx // 4, idx % 4, tri[idx]


def read_msh(path, bc_map=None, default_bc=2):
    bc_map = {} if bc_map is None else dict(bc_map)
    with open(path) as fh:
        sec = _sections(fh.read().splitlines())
    fmt = sec.get("MeshFormat")
    if not fmt or not fmt[0].split()[0].startswith("2") or fmt[0].split()[1] != "0":
        raise ValueError("only MSH 2.x ASCII files are read")
    nodes = sec["Nodes"]
    nn = int(nodes[0])
    ids = np.empty(nn, dtype=np.int64)
    vxyz = np.empty((nn, 3))
    for i in range(nn):
        p = nodes[1 + i].split()
        ids[i] = int(p[0])
        vxyz[i] = [float(p[1]), float(p[2]), float(p[3])]
    where = {int(v): i for i, v in enumerate(ids)}
    tets, tris, tags = [], [], []
    els = sec["Elements"]
    for ln in els[1:1 + int(els[0])]:
        p = [int(x) for x in ln.split()]
        typ, ntag = p[1], p[2]
        vs = [where[v] for v in p[3 + ntag:]]
        if typ == 4:
            tets.append(vs[:4])
        elif typ == 2:
            tris.append(sorted(vs[:3]))
            tags.append(p[3] if ntag > 0 else 0)
    etov = np.asarray(tets, dtype=np.int64).reshape(-1, 4)
    if etov.shape[0] == 0:
        raise ValueError("no tetrahedra in %s" % path)
    V = vxyz[etov]
    det = np.einsum("ki,ki->k", V[:, 1] - V[:, 0],
                    np.cross(V[:, 2] - V[:, 0], V[:, 3] - V[:, 0]))
    neg = det < 0
    etov[neg, 2], etov[neg, 3] = etov[neg, 3].copy(), etov[neg, 2].copy()
    face_bc = np.zeros(etov.shape, dtype=np.int8)
    ke, kf, tri = _boundary_faces(etov)
    tag_of = {tuple(t): g for t, g in zip(tris, tags)}
    for e, f, t in zip(ke, kf, tri):
        g = tag_of.get(tuple(int(x) for x in t))
        face_bc[e, f] = bc_map.get(g, default_bc) if g is not None else default_bc
    return {"vxyz": vxyz, "etov": etov.astype(np.int32), "vertex_periodic_id": None,
            "face_bc": face_bc}


def write_msh(path, mesh, bc_physical=None):
    phys = {1: 1, 2: 2} if bc_physical is None else dict(bc_physical)
    vxyz = np.asarray(mesh["vxyz"], dtype=np.float64)
    etov = np.asarray(mesh["etov"], dtype=np.int64)
    face_bc = np.asarray(mesh["face_bc"])
    ke, kf, _ = _boundary_faces(etov)
    lines = ["$MeshFormat", "2.2 0 8", "$EndMeshFormat", "$Nodes", str(len(vxyz))]
    lines += ["%d %.17g %.17g %.17g" % (i + 1, *v) for i, v in enumerate(vxyz)]
    lines += ["$EndNodes", "$Elements", str(len(ke) + len(etov))]
    n = 0
    for e, f in zip(ke, kf):
        n += 1
        vs = etov[e, list(FACE_VERTS[f])] + 1
        g = phys.get(int(face_bc[e, f]), 0)
        lines.append("%d 2 2 %d %d %d %d %d" % (n, g, g, *vs))
    for e in range(len(etov)):
        n += 1
        lines.append("%d 4 2 0 0 %d %d %d %d" % (n, *(etov[e] + 1)))
    lines.append("$EndElements")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
