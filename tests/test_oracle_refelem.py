"""Pins of the oracle's reference operators against facts outside the oracle.

* differentiation matrices reproduce the analytic derivative of every
  monomial r^a s^b t^c of degree <= N;
* the mass and face-mass matrices reproduce integrals computed by an
  independent collapsed-coordinate Gauss-Jacobi (Stroud conical product)
  quadrature from scipy, never through the oracle's own simplex formula;
* the P1 operators equal the textbook closed forms stored in
  tests/golden/p1_operators.json;
* LIFT satisfies M LIFT = E.
"""

import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import roots_jacobi

from oracle import refelem

REF_V = np.array([[-1, -1, -1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)


def nodes_rst(N):
    lat = np.array(refelem.lattice(N), dtype=float)
    return -1.0 + 2.0 * lat / N


def monomials(N):
    return [(a, b, c) for a in range(N + 1) for b in range(N + 1)
            for c in range(N + 1) if a + b + c <= N]


def mono_eval(e, x):
    return x[:, 0] ** e[0] * x[:, 1] ** e[1] * x[:, 2] ** e[2]


def _gj(n, alpha):
    x, w = roots_jacobi(n, alpha, 0.0)
    # map [-1, 1] with weight (1-x)^alpha to [0, 1] with weight (1-u)^alpha
    return (x + 1.0) / 2.0, w / 2.0 ** (alpha + 1)


def tet_quadrature(n):
    """Points [P,3] (reference rst) and weights integrating over the
    reference tetrahedron (volume 4/3) exactly up to degree 2n-1."""
    a, wa = _gj(n, 2.0)
    b, wb = _gj(n, 1.0)
    c, wc = _gj(n, 0.0)
    pts, wts = [], []
    for (ai, wai), (bi, wbi), (ci, wci) in itertools.product(
            zip(a, wa), zip(b, wb), zip(c, wc)):
        l1 = ai
        l2 = bi * (1 - ai)
        l3 = ci * (1 - ai) * (1 - bi)
        pts.append([2 * l1 - 1, 2 * l2 - 1, 2 * l3 - 1])
        wts.append(wai * wbi * wci * 8.0)     # unit simplex -> reference
    return np.array(pts), np.array(wts)


def face_quadrature(f, n):
    """Points on reference face f and weights of (1/|F|) int_F."""
    a, wa = _gj(n, 1.0)
    b, wb = _gj(n, 0.0)
    verts = REF_V[[v for v in range(4) if v != f]]
    pts, wts = [], []
    for (ai, wai), (bi, wbi) in itertools.product(zip(a, wa), zip(b, wb)):
        m1 = ai
        m2 = bi * (1 - ai)
        m0 = 1 - m1 - m2
        pts.append(m0 * verts[0] + m1 * verts[1] + m2 * verts[2])
        wts.append(wai * wbi * 2.0)           # area-normalised
    return np.array(pts), np.array(wts)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_derivatives_exact_on_monomials(N):
    ops = refelem.operators(N)
    x = nodes_rst(N)
    for e in monomials(N):
        p = mono_eval(e, x)
        for d, D in enumerate((ops["Dr"], ops["Ds"], ops["Dt"])):
            ee = list(e)
            if ee[d] == 0:
                exact = np.zeros(len(x))
            else:
                k = ee[d]
                ee[d] -= 1
                exact = k * mono_eval(ee, x)
            assert np.max(np.abs(D @ p - exact)) < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_mass_matrix_against_quadrature(N):
    ops = refelem.operators(N)
    x = nodes_rst(N)
    qp, qw = tet_quadrature(N + 2)
    M = ops["M"]
    assert np.allclose(M, M.T, atol=0)
    assert np.min(np.linalg.eigvalsh(M)) > 0
    assert abs(M.sum() - 4.0 / 3.0) < 1e-14
    for e1 in monomials(N):
        for e2 in monomials(N):
            exact = np.sum(qw * mono_eval(e1, qp) * mono_eval(e2, qp))
            got = mono_eval(e1, x) @ M @ mono_eval(e2, x)
            assert abs(got - exact) < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_face_mass_and_lift(N):
    ops = refelem.operators(N)
    x = nodes_rst(N)
    Nfp = ops["Nfp"]
    for f in range(4):
        qp, qw = face_quadrature(f, N + 2)
        Ef = ops["E"][:, f * Nfp:(f + 1) * Nfp]
        xf = x[ops["Fmask"][f]]
        for e1 in monomials(N):
            for e2 in monomials(N):
                exact = np.sum(qw * mono_eval(e1, qp) * mono_eval(e2, qp))
                got = mono_eval(e1, x) @ Ef @ mono_eval(e2, xf)
                assert abs(got - exact) < 1e-12
    assert np.max(np.abs(ops["M"] @ ops["LIFT"] - ops["E"])) < 1e-13
    # each face block of E integrates the face: total weight 1 per face
    for f in range(4):
        assert abs(ops["E"][:, f * Nfp:(f + 1) * Nfp].sum() - 1.0) < 1e-13


def test_face_masks_lie_on_faces():
    for N in (1, 2, 3, 4, 6):
        x = nodes_rst(N)
        Fm = refelem.face_masks(N)
        lam = np.c_[1 - (x + 1).sum(1) / 2, (x + 1) / 2]
        for f in range(4):
            assert len(Fm[f]) == (N + 1) * (N + 2) // 2
            assert np.allclose(lam[Fm[f], f], 0.0)


def test_p1_golden():
    path = os.path.join(os.path.dirname(__file__), "golden",
                        "p1_operators.json")
    g = json.load(open(path))
    ex = refelem.exact_operators(1)
    assert [[str(v) for v in row] for row in ex["M"]] == g["M"]
    for name, key in (("Dr", "Dr_row"), ("Ds", "Ds_row"), ("Dt", "Dt_row")):
        for row in ex[name]:
            assert [str(v) for v in row] == g[key]
    Fm = refelem.face_masks(1)
    for f in range(4):
        cols = [ex["E"][i][f * 3:(f + 1) * 3] for i in Fm[f]]
        assert [[str(v) for v in r] for r in cols] == g["face_mass_over_area"]
    assert refelem.VREF == Fraction(g["volume"])


def test_lagrange_at_is_partition_of_unity_and_interpolates():
    N = 3
    rng = np.random.default_rng(3)
    lam = rng.dirichlet(np.ones(4), 5)
    rst = 2 * lam[:, 1:] - 1
    ell = refelem.lagrange_at(N, rst)
    assert np.allclose(ell.sum(1), 1.0, atol=1e-14)
    x = nodes_rst(N)
    for e in monomials(N):
        assert np.allclose(ell @ mono_eval(e, x), mono_eval(e, rst),
                           atol=1e-13)
