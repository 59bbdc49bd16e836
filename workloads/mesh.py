"""Structured tetrahedral meshes of a cube (Kuhn / Freudenthal split).

The cube [0, L]^3 is cut into n^3 cells; cell (i, j, k) has index
c = i + n*(j + n*k).  Every cell is split into 6 tetrahedra, one per
permutation p of the axes (taken in the order xyz, xzy, yxz, yzx, zxy, zyx):
v0 is the cell's lower corner, v1 = v0 + h*e_p1, v2 = v1 + h*e_p2,
v3 = v2 + h*e_p3.  When the vertex order gives a negative volume, v2 and v3
are swapped so every tetrahedron is positively oriented.  Tetrahedron id is
6*c + p.  The split is translation invariant, so it is conforming across cells
and across periodic boundaries.

Local face f of a tetrahedron is the face opposite local vertex f; this is the
face numbering of the C ABI.
"""

import numpy as np

_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]

BC_NONE = 0
BC_FREE_SURFACE = 1
BC_ABSORBING = 2


def kuhn_cube(n, L=1.0, periodic=False, top_free_surface=True):
    """Return a dict describing the Kuhn-split cube mesh.

    Keys: ``vxyz`` float64 [nvert, 3]; ``etov`` int32 [K, 4];
    ``vertex_periodic_id`` int32 [nvert] or None; ``face_bc`` int8 [K, 4]
    (only read where a face has no neighbour: 1 = free surface, 2 =
    absorbing); ``n``, ``L``, ``h``.

    Boundary tags: faces lying on z = L are free surface when
    ``top_free_surface`` is set, every other boundary face is absorbing.
    Periodic meshes tag nothing (every face has a neighbour).
    """
    n = int(n)
    if n < 1:
        raise ValueError("n must be >= 1")
    h = L / n
    m = n + 1
    ii, jj, kk = np.meshgrid(np.arange(m), np.arange(m), np.arange(m),
                             indexing="ij")
    # vertex index v = i + m*(j + m*k)
    vid = lambda i, j, k: i + m * (j + m * k)
    nvert = m ** 3
    vxyz = np.empty((nvert, 3), dtype=np.float64)
    idx = vid(ii, jj, kk).ravel()
    vxyz[idx, 0] = ii.ravel() * h
    vxyz[idx, 1] = jj.ravel() * h
    vxyz[idx, 2] = kk.ravel() * h

    K = 6 * n ** 3
    etov = np.empty((K, 4), dtype=np.int64)
    c = 0
    for k in range(n):
        for j in range(n):
            for i in range(n):
                cell = i + n * (j + n * k)
                for p, perm in enumerate(_PERMS):
                    pos = np.array([i, j, k])
                    verts = [vid(*pos)]
                    for ax in perm:
                        pos = pos.copy()
                        pos[ax] += 1
                        verts.append(vid(*pos))
                    etov[6 * cell + p] = verts
                    c += 1
    # orientation fix: swap v2, v3 where the signed volume is negative
    a = vxyz[etov[:, 1]] - vxyz[etov[:, 0]]
    b = vxyz[etov[:, 2]] - vxyz[etov[:, 0]]
    d = vxyz[etov[:, 3]] - vxyz[etov[:, 0]]
    det = np.einsum("ki,ki->k", a, np.cross(b, d))
    neg = det < 0
    etov[neg, 2], etov[neg, 3] = etov[neg, 3].copy(), etov[neg, 2].copy()
    etov = etov.astype(np.int32)

    pid = None
    face_bc = np.zeros((K, 4), dtype=np.int8)
    if periodic:
        pid = (np.mod(ii, n) + n * (np.mod(jj, n) + n * np.mod(kk, n)))
        tmp = np.empty(nvert, dtype=np.int32)
        tmp[idx] = pid.ravel()
        pid = tmp
    else:
        for f in range(4):
            others = [a_ for a_ in range(4) if a_ != f]
            fv = vxyz[etov[:, others]]                     # [K, 3, 3]
            top = np.all(np.isclose(fv[:, :, 2], L, rtol=0, atol=1e-12 * L),
                         axis=1)
            face_bc[:, f] = BC_ABSORBING
            if top_free_surface:
                face_bc[top, f] = BC_FREE_SURFACE
    return {"vxyz": vxyz, "etov": etov, "vertex_periodic_id": pid,
            "face_bc": face_bc, "n": n, "L": float(L), "h": h}


def kuhn_box(nx, ny, nz, Lx, Ly, Lz, periodic=(False, False, False), free_faces=()):
    """The Kuhn split of the box [0, Lx] x [0, Ly] x [0, Lz] cut into
    nx x ny x nz cells (the same six tetrahedra per cell as ``kuhn_cube``,
    cell c = i + nx (j + ny k), tetrahedron 6 c + p).  ``periodic`` marks the
    axes whose opposite faces are identified (each needs at least 3 cells);
    boundary faces on the box faces listed in ``free_faces`` ("x-" is x = 0,
    "z+" is z = Lz, ...) are free surfaces, every other boundary face is
    absorbing.  Same keys as ``kuhn_cube`` plus ``shape`` and ``lengths``."""
    n = np.array([nx, ny, nz], dtype=np.int64)
    Ls = np.array([Lx, Ly, Lz], dtype=np.float64)
    m = n + 1
    ii, jj, kk = np.meshgrid(np.arange(m[0]), np.arange(m[1]), np.arange(m[2]),
                             indexing="ij")
    vid = lambda i, j, k: i + m[0] * (j + m[1] * k)
    nvert = int(m.prod())
    vxyz = np.empty((nvert, 3), dtype=np.float64)
    idx = vid(ii, jj, kk).ravel()
    h = Ls / n
    vxyz[idx, 0] = ii.ravel() * h[0]
    vxyz[idx, 1] = jj.ravel() * h[1]
    vxyz[idx, 2] = kk.ravel() * h[2]
    K = int(6 * n.prod())
    etov = np.empty((K, 4), dtype=np.int64)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                cell = i + nx * (j + ny * k)
                for p, perm in enumerate(_PERMS):
                    pos = np.array([i, j, k])
                    verts = [vid(*pos)]
                    for ax in perm:
                        pos = pos.copy()
                        pos[ax] += 1
                        verts.append(vid(*pos))
                    etov[6 * cell + p] = verts
    a = vxyz[etov[:, 1]] - vxyz[etov[:, 0]]
    b = vxyz[etov[:, 2]] - vxyz[etov[:, 0]]
    d = vxyz[etov[:, 3]] - vxyz[etov[:, 0]]
    det = np.einsum("ki,ki->k", a, np.cross(b, d))
    neg = det < 0
    etov[neg, 2], etov[neg, 3] = etov[neg, 3].copy(), etov[neg, 2].copy()
    pid = None
    if any(periodic):
        wrap = [np.mod(g, n[a_]) if periodic[a_] else g
                for a_, g in enumerate((ii, jj, kk))]
        p_ = wrap[0] + m[0] * (wrap[1] + m[1] * wrap[2])
        pid = np.empty(nvert, dtype=np.int32)
        pid[idx] = p_.ravel()
    face_bc = np.full((K, 4), BC_ABSORBING, dtype=np.int8)
    for name in free_faces:
        ax = "xyz".index(name[0])
        at = 0.0 if name[1] == "-" else Ls[ax]
        for f in range(4):
            fv = vxyz[etov[:, [a_ for a_ in range(4) if a_ != f]]]   # [K, 3, 3]
            on = np.all(np.isclose(fv[:, :, ax], at, rtol=0, atol=1e-12 * Ls[ax]), axis=1)
            face_bc[on, f] = BC_FREE_SURFACE
    return {"vxyz": vxyz, "etov": etov.astype(np.int32), "vertex_periodic_id": pid,
            "face_bc": face_bc, "shape": (nx, ny, nz), "lengths": (Lx, Ly, Lz),
            "h": float(h.min())}


# the 12 even permutations of (0, 1, 2, 3): relabelling an element's vertices
# by one of them keeps its orientation positive
EVEN_PERMS = [p for p in
              [(a, b, c, d) for a in range(4) for b in range(4)
               for c in range(4) for d in range(4)
               if len({a, b, c, d}) == 4]
              if sum(1 for i in range(4) for j in range(i + 1, 4)
                     if p[i] > p[j]) % 2 == 0]


def general_mesh(n, L=1.0, seed=0, jitter=0.15, top_free_surface=True):
    """An unstructured-looking tetrahedral mesh of the cube [0, L]^3 from the
    Kuhn split with every structured regularity removed (seeded):

    * interior vertices moved by up to ``jitter * h`` per axis (boundary
      vertices stay on their planes, so the domain and its boundary tags are
      unchanged), so every element has its own affine map and normals;
    * each element's local vertex order relabelled by a random even
      permutation (orientation stays positive; face tags follow their faces),
      so matched faces meet in every relative orientation;
    * elements and vertex ids randomly renumbered.

    Same keys as ``kuhn_cube`` plus ``elem_from_kuhn`` (the Kuhn element each
    element came from) and ``vert_from_kuhn``.
    """
    m = kuhn_cube(n, L, periodic=False, top_free_surface=top_free_surface)
    rng = np.random.default_rng(seed)
    h = m["h"]
    V = m["vxyz"].copy()
    inner = np.all((V > 1e-9 * L) & (V < L - 1e-9 * L), axis=1)
    V[inner] += rng.uniform(-jitter * h, jitter * h, size=(int(inner.sum()), 3))
    etov = m["etov"].astype(np.int64)
    bc = m["face_bc"].copy()
    K = etov.shape[0]
    sig = np.asarray(EVEN_PERMS)[rng.integers(0, len(EVEN_PERMS), size=K)]
    etov = np.take_along_axis(etov, sig, axis=1)
    bc = np.take_along_axis(bc, sig, axis=1)    # face f is opposite vertex f
    pe = rng.permutation(K)
    etov, bc = etov[pe], bc[pe]
    pv = rng.permutation(V.shape[0])            # new id of old vertex v
    Vn = np.empty_like(V)
    Vn[pv] = V
    etov = pv[etov]
    a = Vn[etov[:, 1]] - Vn[etov[:, 0]]
    b = Vn[etov[:, 2]] - Vn[etov[:, 0]]
    d = Vn[etov[:, 3]] - Vn[etov[:, 0]]
    det = np.einsum("ki,ki->k", a, np.cross(b, d))
    if not np.all(det > 0):
        raise ValueError("jitter too large: an element turned over")
    inv_pv = np.empty_like(pv)
    inv_pv[pv] = np.arange(pv.size)
    return {"vxyz": Vn, "etov": etov.astype(np.int32), "vertex_periodic_id": None,
            "face_bc": bc.astype(np.int8), "n": n, "L": float(L), "h": h,
            "elem_from_kuhn": pe, "vert_from_kuhn": inv_pv}


def element_centroids(mesh):
    """Mean of the 4 vertex coordinates of every element, [K, 3]."""
    return mesh["vxyz"][mesh["etov"]].mean(axis=1)


def lattice_node_coords(mesh, N):
    """Physical coordinates of the nodal points, [K, Np, 3].

    Node contract of the library: the equispaced lattice of order N on the
    reference tetrahedron, node (i, j, k) with i + j + k <= N has barycentric
    coordinates (1 - (i+j+k)/N, i/N, j/N, k/N) with respect to the element's
    vertices (v0, v1, v2, v3); nodes are ordered k outermost, then j, then i.
    """
    lam = []
    for k in range(N + 1):
        for j in range(N + 1 - k):
            for i in range(N + 1 - j - k):
                lam.append((N - i - j - k, i, j, k))
    lam = np.asarray(lam, dtype=np.float64) / N            # [Np, 4]
    V = mesh["vxyz"][mesh["etov"]]                          # [K, 4, 3]
    return np.einsum("na,kac->knc", lam, V)
