"""Pins of the oracle's boundary ghost states through an exact energy balance.

The discrete energy E(q) = 1/2 q^T W q is a quadratic form, so its rate of
change along the semi-discrete right-hand side r = L q is exactly
dE/dt = q^T W r = (E(q + r) - E(q - r)) / 2.  For the strong-form nodal DG
scheme with exact mass and face-mass matrices (affine element, constant
material) the volume terms integrate by parts exactly, and the rate is a sum
of face integrals of degree-2N polynomials:

    dE/dt = sum_f int_f ( v.t* + t.v* - t.v ) dS,

with (v, t = sigma n) the element's own trace and (v*, t*) the flux states.
On a single element every face is a boundary face.  The ghost states fix the
flux states and with them the integrand, split into normal and tangential
parts (Zp for the normal part, Zs for the tangential part):

* absorbing (ghost v+ = 0, sigma+ = 0): t* = (t - Z v)/2, v* = (v - t/Z)/2,
  so the integrand is -(Zp v_n^2 + Zs |v_T|^2 + t_n^2/Zp + |t_T|^2/Zs)/2;
* free surface (ghost v+ = v, sigma+ = -sigma): t* = 0, v* = v - t/Z, so the
  integrand is -(t_n^2/Zp + |t_T|^2/Zs).

The right-hand side of this balance is computed here without any oracle code:
the element's fields are fitted by monomials in physical coordinates at the
physical node positions, evaluated at the points of a collapsed Gauss-Jacobi
rule on each physical face (exact for the degree-2N integrand), with the
normal and area from the face's own vertices.  Mapping absorbing faces to the
free-surface ghost (or the reverse) changes the balance, and a test below
checks that such a planted mistake is caught.
"""

import itertools

import numpy as np
import pytest
import torch
from scipy.special import roots_jacobi

import workloads as W
from oracle import solver as O

VERTS = np.array([[0.0, 0.0, 0.0], [1.1, 0.1, -0.05], [0.2, 0.9, 0.1],
                  [0.05, 0.15, 1.2]])


def one_element(face_bc):
    return {"vxyz": VERTS.copy(), "etov": np.array([[0, 1, 2, 3]], np.int32),
            "vertex_periodic_id": None,
            "face_bc": np.array([face_bc], np.int8)}


def _gj(n, alpha):
    x, w = roots_jacobi(n, alpha, 0.0)
    return (x + 1.0) / 2.0, w / 2.0 ** (alpha + 1)


def triangle_rule(a, b, c, n):
    """Points and weights of int over the physical triangle (a, b, c),
    exact to degree 2n - 1 (collapsed coordinates)."""
    u, wu = _gj(n, 1.0)
    v, wv = _gj(n, 0.0)
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a))
    pts, wts = [], []
    for (ui, wi), (vi, wj) in itertools.product(zip(u, wu), zip(v, wv)):
        m1, m2 = ui, vi * (1 - ui)
        pts.append((1 - m1 - m2) * a + m1 * b + m2 * c)
        wts.append(wi * wj * 2.0 * area)
    return np.array(pts), np.array(wts)


def monomial_fit(x_nodes, values, N):
    """Coefficients of the degree-N polynomial interpolating values [Np, m]
    at x_nodes [Np, 3], and an evaluator."""
    exps = [(a, b, c) for a in range(N + 1) for b in range(N + 1)
            for c in range(N + 1) if a + b + c <= N]
    V = lambda x: np.stack([x[:, 0] ** e[0] * x[:, 1] ** e[1] * x[:, 2] ** e[2]
                            for e in exps], axis=1)
    coef = np.linalg.solve(V(x_nodes), values)
    return lambda x: V(x) @ coef


def boundary_power(q, N, face_bc, rho, lam, mu):
    """Right-hand side of the balance for a single element (see above)."""
    x = W.lattice_node_coords(one_element(face_bc), N)[0]        # [Np, 3]
    ev = monomial_fit(x, q.T, N)                                  # 9 fields
    zp, zs = np.sqrt(rho * (lam + 2 * mu)), np.sqrt(rho * mu)
    total = 0.0
    for f in range(4):
        a, b, c = VERTS[[v for v in range(4) if v != f]]
        n = np.cross(b - a, c - a)
        n /= np.linalg.norm(n)
        if np.dot(n, VERTS[f] - a) > 0:                           # outward
            n = -n
        pts, wts = triangle_rule(a, b, c, N + 1)
        val = ev(pts)                                             # [P, 9]
        v = val[:, 0:3]
        sxx, syy, szz, syz, sxz, sxy = (val[:, i] for i in range(3, 9))
        t = np.stack([sxx * n[0] + sxy * n[1] + sxz * n[2],
                      sxy * n[0] + syy * n[1] + syz * n[2],
                      sxz * n[0] + syz * n[1] + szz * n[2]], axis=1)
        vn, tn = v @ n, t @ n
        vT, tT = v - vn[:, None] * n, t - tn[:, None] * n
        if face_bc[f] == 2:
            dens = -0.5 * (zp * vn ** 2 + zs * (vT ** 2).sum(1)
                           + tn ** 2 / zp + (tT ** 2).sum(1) / zs)
        else:
            dens = -(tn ** 2 / zp + (tT ** 2).sum(1) / zs)
        total += float(np.dot(wts, dens))
    return total


def oracle_rate(P, q, rho, lam, mu):
    t = lambda v: torch.tensor([v], dtype=torch.float64)
    qq = torch.as_tensor(q[None].copy())
    r = O.rhs(P, qq, t(rho), t(lam), t(mu))
    ep = O.energy(P, qq + r, t(rho), t(lam), t(mu)).item()
    em = O.energy(P, qq - r, t(rho), t(lam), t(mu)).item()
    return 0.5 * (ep - em)


CASES = [(2, 2, 2, 2), (1, 1, 1, 1), (2, 1, 2, 1), (1, 2, 2, 1)]


@pytest.mark.parametrize("face_bc", CASES)
@pytest.mark.parametrize("N", [1, 2, 3])
def test_energy_rate_equals_boundary_power(face_bc, N):
    rng = np.random.default_rng(100 + N + 7 * sum(face_bc))
    rho, cp, ratio = rng.uniform(1, 3), rng.uniform(1.5, 3), rng.uniform(1.5, 2.2)
    lam, mu = W.lame_from_velocities(np.array([cp]), np.array([cp / ratio]),
                                     np.array([rho]))[1:]
    lam, mu = float(lam[0]), float(mu[0])
    P = O.Problem(one_element(face_bc), N)
    q = rng.standard_normal((9, P.Np))
    got = oracle_rate(P, q, rho, lam, mu)
    want = boundary_power(q, N, face_bc, rho, lam, mu)
    assert want < 0
    assert abs(got - want) <= 1e-12 * abs(want), (got, want)


def test_swapped_ghost_states_are_caught():
    """A planted mistake in the oracle (absorbing faces given the free-surface
    ghost and the reverse) breaks the balance."""
    N, face_bc = 2, (2, 1, 2, 1)
    rho, lam, mu = 2.0, 1.3, 0.8
    P = O.Problem(one_element(face_bc), N)
    q = np.random.default_rng(7).standard_normal((9, P.Np))
    want = boundary_power(q, N, face_bc, rho, lam, mu)
    assert abs(oracle_rate(P, q, rho, lam, mu) - want) <= 1e-12 * abs(want)
    P.free, P.absorb = P.absorb, P.free
    bad = oracle_rate(P, q, rho, lam, mu)
    assert abs(bad - want) > 1e-3 * abs(want)
