"""Pins of fluid (mu = 0, acoustic) elements in the oracle.

* An acoustic plane wave (the elastic P wave with mu = 0) in a periodic
  fluid box converges to the closed-form solution under mesh refinement at
  observed order >= N + 1/2.
* Fluid-solid interfaces: with the central flux the exact rate of change of
  the quadratic energy, dE/dt = (E(q + Lq) - E(q - Lq))/2, is zero on a
  periodic mixed mesh (fluid stress isotropic, as the fluid energy assumes);
  the upwind flux dissipates.
* A fluid element's stress rate is isotropic: its shear components vanish
  and its three normal components are equal, exactly.
* The fluid energy term, tr^T M tr / (9 lambda), is the mu -> 0 limit of the
  elastic one for isotropic stress.
"""

import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import solver as O
from workloads.planewave import plane_wave_state


def _fluid_plane_wave_error(n, N, T=0.25):
    mesh = W.kuhn_cube(n, 1.0, periodic=True)
    K = mesh["etov"].shape[0]
    rho, lam, mu = np.full(K, 1.2), np.full(K, 2.7), np.zeros(K)
    P = O.Problem(mesh, N)
    x = W.lattice_node_coords(mesh, N)
    d, kw = (1.0, 1.0, 0.0), 2.0 * math.pi * math.sqrt(2.0)
    q0 = plane_wave_state(x, 0.0, "P", d, kw, 1.2, 2.7, 0.0).transpose(0, 2, 1)
    dt0 = P.suggest_dt(rho, lam, mu, 0.4)
    steps = int(math.ceil(T / dt0))
    dt = T / steps
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a))
    q, _ = O.run(P, t(q0), t(rho), t(lam), t(mu), dt, steps)
    ex = plane_wave_state(x, T, "P", d, kw, 1.2, 2.7, 0.0).transpose(0, 2, 1)
    return float(np.sqrt(np.mean((q.numpy() - ex) ** 2)))


@pytest.mark.parametrize("N,levels", [(2, (4, 6)), (3, (3, 6))])
def test_fluid_plane_wave_converges(N, levels):
    # fixed, deterministic configurations (observed orders 3.4 and 4.1; the
    # elastic P wave on the same meshes converges alike)
    e1 = _fluid_plane_wave_error(levels[0], N, T=0.1)
    e2 = _fluid_plane_wave_error(levels[1], N, T=0.1)
    rate = math.log(e1 / e2) / math.log(levels[1] / levels[0])
    assert e2 < e1
    assert rate >= N + 0.5, (e1, e2, rate)


def _mixed_problem(N, seed):
    mesh = W.kuhn_cube(3, 1.0, periodic=True)
    K = mesh["etov"].shape[0]
    cen = W.element_centroids(mesh)
    fluid = cen[:, 2] < 0.5
    rng = np.random.default_rng(seed)
    cp = rng.uniform(1.5, 3.0, K)
    cs = np.where(fluid, 0.0, cp / rng.uniform(1.5, 2.2, K))
    rho = rng.uniform(1.0, 3.0, K)
    rho_, lam, mu = W.lame_from_velocities(cp, cs, rho)
    P = O.Problem(mesh, N)
    q = rng.standard_normal((K, 9, P.Np))
    # fluid stress isotropic: -p I
    p = q[fluid, 3]
    q[fluid, 3:6] = p[:, None, :]
    q[fluid, 6:9] = 0.0
    t = torch.as_tensor
    return P, t(q), t(rho_), t(lam), t(mu), fluid


def _rate(P, q, rho, lam, mu):
    r = O.rhs(P, q, rho, lam, mu)
    return 0.5 * (O.energy(P, q + r, rho, lam, mu).item()
                  - O.energy(P, q - r, rho, lam, mu).item()), r


@pytest.mark.parametrize("N", [1, 2, 3])
def test_fluid_solid_energy_central_and_upwind(N):
    P, q, rho, lam, mu, fluid = _mixed_problem(N, 11 + N)
    assert 0 < fluid.sum() < len(fluid)
    P.flux_tau = 0.0
    r0, r = _rate(P, q, rho, lam, mu)
    E = O.energy(P, q, rho, lam, mu).item()
    scale = float(torch.sum(r ** 2).sqrt()) * math.sqrt(E)
    P.flux_tau = 1.0
    r1, _ = _rate(P, q, rho, lam, mu)
    assert abs(r0) <= 1e-12 * scale, (r0, scale)
    assert r1 < -1e-6 * scale


def test_fluid_stress_rate_is_isotropic():
    P, q, rho, lam, mu, fluid = _mixed_problem(3, 4)
    # any state, also a non-isotropic one
    q = q + torch.as_tensor(np.random.default_rng(1).standard_normal(tuple(q.shape)))
    for tau in (1.0, 0.0):
        P.flux_tau = tau
        r = O.rhs(P, q, rho, lam, mu)[torch.as_tensor(fluid)]
        assert torch.all(r[:, 6:9] == 0)
        assert torch.equal(r[:, 3], r[:, 4]) and torch.equal(r[:, 3], r[:, 5])


def test_fluid_energy_is_the_shear_free_limit():
    mesh = W.kuhn_cube(2, 1.0)
    K = mesh["etov"].shape[0]
    P = O.Problem(mesh, 2)
    rng = np.random.default_rng(2)
    q = rng.standard_normal((K, 9, P.Np))
    q[:, 4] = q[:, 3]
    q[:, 5] = q[:, 3]
    q[:, 6:9] = 0.0
    q = torch.as_tensor(q)
    rho = torch.as_tensor(rng.uniform(1, 2, K))
    lam = torch.as_tensor(rng.uniform(1, 3, K))
    e0 = O.energy(P, q, rho, lam, torch.zeros(K, dtype=torch.float64)).item()
    eps = O.energy(P, q, rho, lam, torch.full((K,), 1e-9, dtype=torch.float64)).item()
    assert abs(e0 - eps) <= 1e-8 * e0
