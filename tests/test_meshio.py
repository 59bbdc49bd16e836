"""Mesh files (Gmsh MSH 2.2 ASCII), host side.

* A general mesh written and read back is the same mesh: vertices exact,
  element vertex lists, boundary tags.
* A hand-written file: node ids that are not 1..n, a negatively oriented
  tetrahedron (its last two vertices swapped on reading), boundary
  triangles whose physical tags map to boundary conditions, untagged
  boundary faces getting the default, other element types ignored.
"""

import numpy as np

import workloads as W
from oracle import solver as O
from paper_2205_11052_amd.meshio import read_msh, write_msh


def test_round_trip(tmp_path):
    m = W.general_mesh(3, 2.0, seed=8)
    p = tmp_path / "g.msh"
    write_msh(p, m)
    r = read_msh(p, bc_map={1: 1, 2: 2})
    assert np.array_equal(r["vxyz"], m["vxyz"])
    assert np.array_equal(r["etov"], m["etov"])
    # tags are read where a face has no neighbour (the recipe tags every
    # face; the reader writes 0 on interior ones)
    bnd = r["face_bc"] > 0
    assert bnd.sum() == 2 * 6 * 3 * 3
    assert np.array_equal(r["face_bc"][bnd], m["face_bc"][bnd])
    O.Problem(r, 2)          # a valid mesh for the oracle


TEXT = """$MeshFormat
2.2 0 8
$EndMeshFormat
$Nodes
5
10 0 0 0
20 1 0 0
30 0 1 0
40 0 0 1
50 1 1 1
$EndNodes
$Elements
5
1 15 2 0 10 10
2 2 2 7 3 10 20 30
3 4 2 0 1 10 20 30 40
4 4 2 0 1 20 40 30 50
5 1 2 0 0 10 20
$EndElements
"""


def test_hand_written_file(tmp_path):
    p = tmp_path / "two.msh"
    p.write_text(TEXT)
    r = read_msh(p, bc_map={7: 1}, default_bc=2)
    assert r["vxyz"].shape == (5, 3) and r["etov"].shape == (2, 4)
    # first tetrahedron (0,1,2,3) is positive; the second, listed as
    # (1,3,2,4), is negative and read as (1,3,4,2)
    assert r["etov"].tolist() == [[0, 1, 2, 3], [1, 3, 4, 2]]
    V = r["vxyz"][r["etov"]]
    det = np.einsum("ki,ki->k", V[:, 1] - V[:, 0],
                    np.cross(V[:, 2] - V[:, 0], V[:, 3] - V[:, 0]))
    assert np.all(det > 0)
    # the shared face (1,2,3) is interior (tag 0): face 0 of element 0,
    # face 2 of element 1; the tagged triangle (0,1,2) is face 3 of element
    # 0: free surface; every other boundary face is absorbing
    bc = r["face_bc"]
    assert bc[0, 0] == 0 and bc[1, 2] == 0
    assert bc[0, 3] == 1
    assert sorted(bc.reshape(-1).tolist()) == [0, 0, 1, 2, 2, 2, 2, 2]
