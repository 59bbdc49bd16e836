"""Features together: three batched shots of uneven length (one launch per
stage over all shots) on a general mesh in Morton order with the blended
flux (tau = 0.5), both kernel variants, FP64; once with a fluid layer, once
with a fully anisotropic medium and a sponge layer.  Every shot's fields
and traces at the end of its own length against the oracle run of that
shot alone (<= 1e-12).
"""

import numpy as np
import pytest

import workloads as W
from paper_2205_11052_amd import Solver, order_elements, permute_mesh
from gpu_helpers import oracle_problem, oracle_run, rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kernel", [0, 1])
def test_batched_general_fluid_blended_flux(kernel):
    g = W.general_mesh(4, 2.0, seed=61)
    mesh = permute_mesh(g, order_elements(g["vxyz"], g["etov"], "morton"))
    K = mesh["etov"].shape[0]
    cen = W.element_centroids(mesh)
    fluid = cen[:, 2] > 1.4
    rng = np.random.default_rng(62)
    cp = rng.uniform(1.5, 3.0, K)
    cs = np.where(fluid, 0.0, cp / rng.uniform(1.5, 2.2, K))
    rho, lam, mu = W.lame_from_velocities(cp, cs, rng.uniform(1.0, 3.0, K))
    N, tau = 3, 0.5
    P = oracle_problem(mesh, N)
    P.flux_tau = tau
    dt = P.suggest_dt(rho, lam, mu, 0.5)
    shots = [(cen[11], 9), (cen[200], 4), (cen[333], 7)]     # (source, length)
    rec = cen[[5, 120, 260]]
    moment = (1.0, -0.5, 0.25, 0.3, -0.2, 0.1)
    say("case combined kernel=%d K=%d fluid=%d" % (kernel, K, fluid.sum()))
    s = Solver(N, 64, len(shots))
    s.set_mesh_dict(mesh)
    s.set_material(rho, lam, mu)
    s.set_dt(dt)
    s.set_flux(tau)
    s.set_launch(kernel)
    for i, (pos, n) in enumerate(shots):
        s.set_source(i, pos, 4.0, 0.1, 1.5, nsteps=n, moment=moment)
        s.set_receivers(i, rec, 16)
    s.zero_fields()
    s.step(12)                       # every shot stops at its own length
    P.set_receivers(rec)
    for i, (pos, n) in enumerate(shots):
        assert s.shot_steps(i) == n
        P.set_source(pos, 4.0, 0.1, 1.5, moment=moment)
        q_ora, tr_ora = oracle_run(P, np.zeros((K, 9, P.Np)), rho, lam, mu, dt, n,
                                   record=True)
        err = rel_l2(s.get_fields(i), q_ora)
        terr = rel_l2(s.read_traces(i)[:, :, :n], tr_ora)
        say("combined shot %d (%d steps) fields %.3e traces %.3e" % (i, n, err, terr))
        assert np.abs(q_ora).max() > 0
        assert err <= 1e-12 and terr <= 1e-12


@pytest.mark.parametrize("kernel", [0, 1])
def test_batched_general_anisotropic_sponge(kernel):
    """Three batched shots of uneven length on a Morton-ordered general mesh
    with a fully anisotropic heterogeneous medium, a sponge layer and the
    blended flux (tau = 0.5), both kernel variants, FP64, against the
    oracle run of each shot alone (<= 1e-12)."""
    import torch
    g = W.general_mesh(4, 2.0, seed=63)
    mesh = permute_mesh(g, order_elements(g["vxyz"], g["etov"], "morton"))
    K = mesh["etov"].shape[0]
    cen = W.element_centroids(mesh)
    rho, C = W.random_stiffness(K, 64)
    sig = W.sponge_profile(cen, hi=(2.0, 2.0, 2.0), width=0.5, sigma_max=4.0)
    N, tau = 3, 0.5
    P = oracle_problem(mesh, N)
    P.flux_tau = tau
    P.stiffness = torch.as_tensor(C)
    P.sponge = torch.as_tensor(sig)
    c2 = 2.0 * np.linalg.eigvalsh(C).max(axis=1) / rho
    dt = P.suggest_dt(rho, c2 * rho, 0.0 * rho, 0.5)
    shots = [(cen[21], 8), (cen[210], 5), (cen[350], 7)]
    rec = cen[[4, 130, 280]]
    moment = (1.0, -0.5, 0.25, 0.3, -0.2, 0.1)
    say("case combined aniso+sponge kernel=%d K=%d damped=%d" % (kernel, K, (sig > 0).sum()))
    s = Solver(N, 64, len(shots))
    s.set_mesh_dict(mesh)
    s.set_material(rho, np.ones(K), np.ones(K))
    s.set_stiffness(C)
    s.set_damping(sig)
    s.set_dt(dt)
    s.set_flux(tau)
    s.set_launch(kernel)
    for i, (pos, n) in enumerate(shots):
        s.set_source(i, pos, 4.0, 0.1, 1.5, nsteps=n, moment=moment)
        s.set_receivers(i, rec, 16)
    s.zero_fields()
    s.step(10)
    P.set_receivers(rec)
    one = np.ones(K)
    for i, (pos, n) in enumerate(shots):
        assert s.shot_steps(i) == n
        P.set_source(pos, 4.0, 0.1, 1.5, moment=moment)
        q_ora, tr_ora = oracle_run(P, np.zeros((K, 9, P.Np)), rho, one, one, dt, n,
                                   record=True)
        err = rel_l2(s.get_fields(i), q_ora)
        terr = rel_l2(s.read_traces(i)[:, :, :n], tr_ora)
        say("aniso+sponge shot %d (%d steps) fields %.3e traces %.3e" % (i, n, err, terr))
        assert np.abs(q_ora).max() > 0
        assert err <= 1e-12 and terr <= 1e-12
