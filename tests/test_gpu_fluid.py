"""Fluid (mu = 0, acoustic) elements coupled to solid ones, on the GPU
against the oracle: a fluid layer over a solid (free surface on the fluid's
top, absorbing elsewhere), orders 3 and 4, both kernel variants, FP64
<= 1e-12 and FP32 <= 1e-5 (relative L2, fields and traces), the device
energy with fluid elements against the oracle's, and the full-size
82944-element order-4 mesh with a water layer in the benchmark's launch
shapes.  The gradient is refused with fluid elements; negative mu is
refused.
"""

import numpy as np
import pytest
import torch

import workloads as W
from oracle import solver as O
from paper_2205_11052_amd.dgw import DGWError
from gpu_helpers import (gpu_solver, oracle_problem, oracle_run, rel_l2,
                         random_fields, say)

pytestmark = pytest.mark.gpu


def _fluid_over_solid(mesh, seed, z_fluid):
    K = mesh["etov"].shape[0]
    cen = W.element_centroids(mesh)
    fluid = cen[:, 2] > z_fluid
    rng = np.random.default_rng(seed)
    cp = rng.uniform(1.5, 3.0, K)
    cs = np.where(fluid, 0.0, cp / rng.uniform(1.5, 2.2, K))
    rho = rng.uniform(1.0, 3.0, K)
    return W.lame_from_velocities(cp, cs, rho), fluid


def _isotropic_in_fluid(q, fluid):
    q = q.copy()
    q[fluid, 4] = q[fluid, 3]
    q[fluid, 5] = q[fluid, 3]
    q[fluid, 6:9] = 0.0
    return q


@pytest.mark.parametrize("N,kernel,prec", [(3, 0, 64), (3, 1, 64), (4, 0, 64),
                                           (4, 1, 64), (4, 1, 32), (4, 0, 32),
                                           (3, 2, 64), (4, 2, 64), (4, 2, 32)])
def test_fluid_solid_matches_oracle(N, kernel, prec):
    mesh = W.kuhn_cube(3, 1.0)          # free-surface top, absorbing sides
    (rho, lam, mu), fluid = _fluid_over_solid(mesh, 80 + N, 0.6)
    K = mesh["etov"].shape[0]
    say("case fluid/solid N=%d kernel=%d fp%d K=%d fluid=%d" % (N, kernel, prec, K,
                                                               fluid.sum()))
    P = oracle_problem(mesh, N)
    dt = P.suggest_dt(rho, lam, mu, 0.5)
    q0 = _isotropic_in_fluid(random_fields(K, P.Np, 90 + N), fluid)
    src = W.element_centroids(mesh)[7]
    rec = W.element_centroids(mesh)[[3, 100, 150]]
    moment = (1.0, 1.0, 1.0, 0.0, 0.0, 0.0)
    P.set_source(src, 3.0, 0.1, 2.0, moment=moment)
    P.set_receivers(rec)
    s = gpu_solver(mesh, N, rho, lam, mu, dt, precision=prec, kernel=kernel)
    s.set_source(0, src, 3.0, 0.1, 2.0, moment=moment)
    s.set_receivers(0, rec, 16)
    s.set_fields(0, q0)
    nst = 7
    s.step(nst)
    q_ora, tr_ora = oracle_run(P, q0, rho, lam, mu, dt, nst, record=True)
    err = rel_l2(s.get_fields(0), q_ora)
    terr = rel_l2(s.read_traces(0), tr_ora)
    say("fluid/solid fields %.3e traces %.3e" % (err, terr))
    tol = 1e-12 if prec == 64 else 1e-5
    assert err <= tol and terr <= tol
    if prec == 64:
        t = lambda a: torch.as_tensor(np.asarray(a))
        e_ora = O.energy(P, t(q_ora), t(rho), t(lam), t(mu)).item()
        assert abs(s.energy(0) - e_ora) <= 1e-13 * e_ora


def test_full_size_water_layer_fp64():
    """The full 82944-element order-4 mesh with a fluid layer above z = 8
    (a water column over the layered solid), random fields, two steps
    against the oracle in the benchmark's launch shapes."""
    w = W.build_workload("c1_layered_n24")
    cen = W.element_centroids(w["mesh"])
    fluid = cen[:, 2] > 8.0
    mu = np.where(fluid, 0.0, w["mu"])
    lam = np.where(fluid, w["lam"] + 2.0 * w["mu"], w["lam"])   # same cp
    rho = w["rho"]
    say("case full water layer K=%d fluid=%d" % (w["K"], fluid.sum()))
    P = oracle_problem(w["mesh"], w["N"])
    dt = P.suggest_dt(rho, lam, mu, w["cfl"])
    q0 = _isotropic_in_fluid(random_fields(w["K"], P.Np, 12), fluid)
    P.set_source(w["source"], w["f0"], 0.05, w["amp"])
    P.set_receivers(w["receivers"])
    q_ora, tr_ora = oracle_run(P, q0, rho, lam, mu, dt, 2, record=True)
    s = gpu_solver(w["mesh"], w["N"], rho, lam, mu, dt)
    s.set_source(0, w["source"], w["f0"], 0.05, w["amp"])
    s.set_receivers(0, w["receivers"], 8)
    for shape in ((1, 7, 0), (0, 7, 0), (1, 3, 0)):
        s.set_launch(*shape)
        s.set_fields(0, q0)
        s.step(2)
        err = rel_l2(s.get_fields(0), q_ora)
        terr = rel_l2(s.read_traces(0), tr_ora)
        say("full water layer shape %s fields %.3e traces %.3e" % (shape, err, terr))
        assert err <= 1e-12 and terr <= 1e-12


def test_gradient_and_negative_mu_refused():
    mesh = W.kuhn_cube(2, 1.0)
    (rho, lam, mu), fluid = _fluid_over_solid(mesh, 3, 0.5)
    s = gpu_solver(mesh, 2, rho, lam, mu, 1e-3)
    s.set_receivers(0, np.array([[0.5, 0.5, 0.25]]), 4)
    with pytest.raises(DGWError) as e:
        s.forward_checkpointed(4, 2, np.zeros((1, 1, 3, 4)))
    assert e.value.code == -5
    bad = mu.copy()
    bad[0] = -1e-3
    with pytest.raises(DGWError) as e:
        s.set_material(rho, lam, bad)
    assert e.value.code == -1
