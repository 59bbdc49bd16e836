"""Anisotropic elements (dgw_set_stiffness: Voigt C per element, exact
Riemann states from impedance matrices) on the GPU against the oracle with
the same stiffness: FP64 relative L2 <= 1e-12, FP32 <= 1e-5, fully
anisotropic heterogeneous media (every one of the 21 entries nonzero and
varying per element), every boundary type, blended flux, a moment source
and receivers; a general mesh; the full 82944-element order-4 mesh in the
benchmark's launch shapes of both kernels; the device energy; an isotropic
C against the isotropic path; the state rules of the entry point.
"""

import numpy as np
import pytest
import torch

import workloads as W
from oracle import solver as O
from paper_2205_11052_amd import Solver, order_elements, permute_mesh
from paper_2205_11052_amd.dgw import DGWError
from gpu_helpers import oracle_problem, oracle_run, rel_l2, random_fields, say

pytestmark = pytest.mark.gpu

MOMENT = (1.0, -0.5, 0.25, 0.3, -0.2, 0.1)


def _dt_aniso(P, rho, C, cfl=0.5):
    # the oracle's time step with cp replaced by a bound on the fastest
    # speed: the largest eigenvalue of 2 C / rho (|N(n)|^2 = 2)
    c2 = 2.0 * np.linalg.eigvalsh(C).max(axis=1) / rho
    return P.suggest_dt(rho, c2 * rho, 0.0 * rho, cfl)


def _solver(mesh, N, rho, C, dt, precision=64, nshots=1):
    s = Solver(N, precision, nshots)
    s.set_mesh_dict(mesh)
    lam, mu = np.ones_like(rho), np.ones_like(rho)    # replaced by C
    s.set_material(rho, lam, mu)
    s.set_stiffness(C)
    s.set_dt(dt)
    return s


def _run_case(mesh, N, prec, tau, seed, nst=6, shape=(0, 0, 0)):
    K = mesh["etov"].shape[0]
    rho, C = W.random_stiffness(K, seed)
    P = oracle_problem(mesh, N)
    P.stiffness = torch.as_tensor(C)
    P.flux_tau = tau
    dt = _dt_aniso(P, rho, C)
    q0 = random_fields(K, P.Np, seed + 1)
    cen = W.element_centroids(mesh)
    src, rec = cen[K // 3], cen[[1, K // 2, K - 2]]
    P.set_source(src, 3.0, 0.1, 2.0, moment=MOMENT)
    P.set_receivers(rec)
    s = _solver(mesh, N, rho, C, dt, prec)
    s.set_launch(*shape)
    s.set_flux(tau)
    s.set_source(0, src, 3.0, 0.1, 2.0, moment=MOMENT)
    s.set_receivers(0, rec, 16)
    s.set_fields(0, q0)
    s.step(nst)
    one = np.ones(K)
    q_ora, tr_ora = oracle_run(P, q0, rho, one, one, dt, nst, record=True)
    return s, P, rho, q_ora, tr_ora


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("N,prec,tau", [(2, 64, 1.0), (3, 64, 1.0), (4, 64, 1.0),
                                        (4, 64, 0.5), (4, 32, 1.0), (3, 32, 0.0)])
def test_anisotropic_matches_oracle(N, prec, tau, kernel):
    mesh = W.kuhn_cube(3, 1.0)                 # free-surface top, absorbing sides
    say("case aniso N=%d fp%d tau=%.1f kernel=%d" % (N, prec, tau, kernel))
    s, P, rho, q_ora, tr_ora = _run_case(mesh, N, prec, tau, 70 + N,
                                         shape=(kernel, 0, 0))
    err = rel_l2(s.get_fields(0), q_ora)
    terr = rel_l2(s.read_traces(0), tr_ora)
    say("aniso fields %.3e traces %.3e" % (err, terr))
    tol = 1e-12 if prec == 64 else 1e-5
    assert err <= tol and terr <= tol
    if prec == 64:
        K = q_ora.shape[0]
        e_ora = O.energy(P, torch.as_tensor(q_ora), torch.as_tensor(rho),
                         torch.ones(K, dtype=torch.float64),
                         torch.ones(K, dtype=torch.float64)).item()
        assert abs(s.energy(0) - e_ora) <= 1e-13 * e_ora


@pytest.mark.parametrize("kernel", [0, 1])
def test_anisotropic_general_mesh(kernel):
    g = W.general_mesh(4, 2.0, seed=77)
    mesh = permute_mesh(g, order_elements(g["vxyz"], g["etov"], "morton"))
    say("case aniso general mesh K=%d kernel=%d" % (mesh["etov"].shape[0], kernel))
    s, P, rho, q_ora, tr_ora = _run_case(mesh, 3, 64, 1.0, 90, shape=(kernel, 0, 0))
    err = rel_l2(s.get_fields(0), q_ora)
    terr = rel_l2(s.read_traces(0), tr_ora)
    say("aniso general mesh fields %.3e traces %.3e" % (err, terr))
    assert err <= 1e-12 and terr <= 1e-12


def test_full_size_anisotropic_fp64():
    """The 82944-element order-4 mesh with a fully anisotropic heterogeneous
    medium, two steps against the oracle in both kernels' launch shapes
    (one work-group per block, both block sizes, persistent)."""
    mesh = W.kuhn_cube(24, 10.0)
    K = mesh["etov"].shape[0]
    say("case full aniso K=%d" % K)
    rho, C = W.random_stiffness(K, 5)
    P = oracle_problem(mesh, 4)
    P.stiffness = torch.as_tensor(C)
    dt = _dt_aniso(P, rho, C)
    q0 = random_fields(K, P.Np, 6)
    one = np.ones(K)
    q_ora, _ = oracle_run(P, q0, rho, one, one, dt, 2)
    s = _solver(mesh, 4, rho, C, dt)
    # the autotuner's picks for this workload are persistent matrix-core
    # shapes (8 or 16 work-groups per CU)
    for shape in ((1, 7, 0), (1, 3, 0), (1, 7, 3), (1, 7, 8), (1, 7, 16), (0, 7, 0),
                  (0, 3, 0), (0, 7, 3)):
        s.set_launch(*shape)
        s.set_fields(0, q0)
        s.step(2)
        err = rel_l2(s.get_fields(0), q_ora)
        say("full aniso shape %s fields %.3e" % (shape, err))
        assert err <= 1e-12


def test_isotropic_stiffness_equals_isotropic_path():
    mesh = W.kuhn_cube(3, 1.0)
    K = mesh["etov"].shape[0]
    rng = np.random.default_rng(4)
    cp = rng.uniform(1.5, 3.0, K)
    rho, lam, mu = W.lame_from_velocities(cp, cp / rng.uniform(1.5, 2.2, K),
                                          rng.uniform(1.0, 3.0, K))
    q0 = random_fields(K, 35, 5)
    out, dts = [], []
    for aniso in (False, True):
        s = Solver(4, 64, 1)
        s.set_mesh_dict(mesh)
        s.set_material(rho, lam, mu)
        if aniso:
            s.set_stiffness(W.isotropic_stiffness(lam, mu))
        dts.append(s.suggest_dt(0.5))
        s.set_dt(1e-3)
        s.set_fields(0, q0)
        s.step(5)
        out.append((s.get_fields(0), s.energy(0)))
        s.close()
    err = rel_l2(out[1][0], out[0][0])
    say("isotropic C vs isotropic path %.3e" % err)
    assert err <= 1e-13
    assert abs(out[1][1] - out[0][1]) <= 1e-13 * out[0][1]
    # every direction has the P speed: the sampled maximum is exact
    assert abs(dts[1] - dts[0]) <= 1e-12 * dts[0]


def test_state_rules():
    mesh = W.kuhn_cube(2, 1.0)
    K = mesh["etov"].shape[0]
    rho, C = W.random_stiffness(K, 8)
    s = Solver(3, 64, 1)
    s.set_mesh_dict(mesh)
    with pytest.raises(DGWError) as e:          # material first
        s.set_stiffness(C)
    assert e.value.code == -5
    s.set_material(rho, np.ones(K), np.ones(K))
    s.set_launch(1)
    s.set_stiffness(C)
    bad = C.copy()
    bad[3] = -np.eye(6)
    with pytest.raises(DGWError) as e:
        s.set_stiffness(bad)
    assert e.value.code == -1
    s.set_dt(1e-3)
    s.set_receivers(0, np.array([[0.5, 0.5, 0.5]]), 4)
    s.zero_fields()
    with pytest.raises(DGWError) as e:
        s.forward_checkpointed(4, 2, np.zeros((1, 1, 3, 4)))
    assert e.value.code == -5
    # the refused stiffness left the previous one in place: parity with it
    P = oracle_problem(mesh, 3)
    P.stiffness = torch.as_tensor(C)
    q0 = random_fields(K, P.Np, 9)
    s.set_fields(0, q0)
    s.step(3)
    one = np.ones(K)
    q_ora, _ = oracle_run(P, q0, rho, one, one, 1e-3, 3)
    assert rel_l2(s.get_fields(0), q_ora) <= 1e-12
    # a new rho recomputes the impedances
    rho2 = rho * 1.3
    s.set_material(rho2, np.ones(K), np.ones(K))
    s.set_fields(0, q0)
    s.step(3)
    q_ora2, _ = oracle_run(P, q0, rho2, one, one, 1e-3, 3)
    assert rel_l2(s.get_fields(0), q_ora2) <= 1e-12
    # NULL returns to the isotropic elements, bit for bit
    s.set_stiffness(None)
    s.set_launch(1)
    s.set_fields(0, q0)
    s.step(3)
    t = Solver(3, 64, 1)
    t.set_mesh_dict(mesh)
    t.set_material(rho2, np.ones(K), np.ones(K))
    t.set_dt(1e-3)
    t.set_launch(1)
    t.set_fields(0, q0)
    t.step(3)
    assert np.array_equal(s.get_fields(0), t.get_fields(0))
