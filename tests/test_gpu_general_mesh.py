"""GPU parity on general meshes and reordered element numberings.

The general-mesh recipe (jittered interior vertices, random element and
vertex numbering, random even relabelling of each element's vertices, so
faces meet in every relative orientation) removes every regularity of the
structured meshes the other tests use.  Bars as elsewhere: FP64 relative L2
<= 1e-12 and FP32 <= 1e-5 against the FP64 oracle; a reordered numbering
gives exactly the relabelled result (each element's arithmetic does not
depend on its position).  Source and receivers sit at element centroids, so
no point lies on a face shared by two elements.
"""

import numpy as np
import pytest

import workloads as W
from paper_2205_11052_amd import order_elements, permute_mesh
from gpu_helpers import (gpu_solver, oracle_problem, oracle_run, rel_l2,
                         random_fields, say)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5
MOMENT = (1.0, -0.5, 0.25, 0.3, -0.2, 0.1)


def _random_medium(K, seed):
    rng = np.random.default_rng(seed)
    cp = rng.uniform(1.5, 3.0, K)
    cs = cp / rng.uniform(1.5, 2.2, K)
    rho = rng.uniform(1.0, 3.0, K)
    return W.lame_from_velocities(cp, cs, rho)


def _points(mesh, elems):
    return W.element_centroids(mesh)[list(elems)]


@pytest.mark.parametrize("N,kernel,prec", [(3, 0, 64), (3, 1, 64), (4, 0, 64),
                                           (4, 1, 64), (4, 0, 32), (4, 1, 32),
                                           (3, 2, 64), (4, 2, 64), (4, 2, 32)])
def test_general_mesh_matches_oracle(N, kernel, prec):
    mesh = W.general_mesh(4, 2.0, seed=21)
    K = mesh["etov"].shape[0]
    say("case general mesh N=%d kernel=%d fp%d K=%d" % (N, kernel, prec, K))
    rho, lam, mu = _random_medium(K, 31 + N)
    P = oracle_problem(mesh, N)
    dt = P.suggest_dt(rho, lam, mu, 0.5)
    q0 = random_fields(K, P.Np, 41 + N)
    src = _points(mesh, [17])[0]
    rec = _points(mesh, [3, 150, 301])
    P.set_source(src, 3.0, 0.1, 2.0, moment=MOMENT)
    P.set_receivers(rec)
    s = gpu_solver(mesh, N, rho, lam, mu, dt, precision=prec, kernel=kernel)
    s.set_source(0, src, 3.0, 0.1, 2.0, moment=MOMENT)
    s.set_receivers(0, rec, 16)
    s.set_fields(0, q0)
    nst = 6
    s.step(nst)
    q_ora, tr_ora = oracle_run(P, q0, rho, lam, mu, dt, nst, record=True)
    err = rel_l2(s.get_fields(0), q_ora)
    terr = rel_l2(s.read_traces(0), tr_ora)
    say("general mesh fields %.3e traces %.3e" % (err, terr))
    tol = FP64_TOL if prec == 64 else FP32_TOL
    assert err <= tol and terr <= tol


@pytest.mark.parametrize("method", ["morton", "rcm"])
def test_reordered_numbering_is_a_relabelling(method):
    mesh = W.general_mesh(6, 3.0, seed=5)
    K = mesh["etov"].shape[0]
    perm = order_elements(mesh["vxyz"], mesh["etov"], method)
    mesh2 = permute_mesh(mesh, perm)
    say("case reorder %s K=%d" % (method, K))
    rho, lam, mu = _random_medium(K, 9)
    q0 = random_fields(K, 35, 10)
    src = _points(mesh, [101])[0]
    rec = _points(mesh, [7, 500, 1200])
    dt = None
    for kernel in (0, 1, 2):
        outs = []
        for m, p in ((mesh, np.arange(K)), (mesh2, perm)):
            from paper_2205_11052_amd import Solver
            s = Solver(4, 64, 1)
            s.set_mesh_dict(m)
            s.set_material(rho[p], lam[p], mu[p])
            if dt is None:
                dt = s.suggest_dt(0.5)
            s.set_dt(dt)
            s.set_launch(kernel)
            s.set_source(0, src, 3.0, 0.1, 2.0, moment=MOMENT)
            s.set_receivers(0, rec, 16)
            s.set_fields(0, q0[p])
            s.step(10)
            outs.append((s.get_fields(0), s.read_traces(0)))
            s.close()
        (q1, t1), (q2, t2) = outs
        say("reorder %s kernel %d max diff %.3e" % (method, kernel,
                                                    np.abs(q2 - q1[perm]).max()))
        assert np.array_equal(q2, q1[perm])
        assert np.array_equal(t2, t1)


def test_full_size_general_mesh_fp64():
    """The full-size general mesh (82944 elements, order 4) in Morton order,
    in the launch shapes the benchmark's autotuner picks from, two steps
    against the oracle."""
    g = W.general_mesh(24, 10.0, seed=3)
    mesh = permute_mesh(g, order_elements(g["vxyz"], g["etov"], "morton"))
    K = mesh["etov"].shape[0]
    say("case full general mesh fp64 K=%d" % K)
    rho, lam, mu, _ = W.layered_medium(W.element_centroids(mesh))
    P = oracle_problem(mesh, 4)
    dt = P.suggest_dt(rho, lam, mu, 0.5)
    q0 = random_fields(K, 35, 23)
    src = _points(mesh, [K // 2])[0]
    rec = _points(mesh, [5, K // 3, K - 9])
    P.set_source(src, 2.0, 0.05, 1.0, moment=MOMENT)
    P.set_receivers(rec)
    q_ora, tr_ora = oracle_run(P, q0, rho, lam, mu, dt, 2, record=True)
    s = gpu_solver(mesh, 4, rho, lam, mu, dt)
    s.set_source(0, src, 2.0, 0.05, 1.0, moment=MOMENT)
    s.set_receivers(0, rec, 8)
    for shape in ((1, 7, 0), (1, 3, 0), (0, 7, 0), (0, 3, 0), (1, 7, 3), (2, 32, 0)):
        s.set_launch(*shape)
        s.set_fields(0, q0)
        s.step(2)
        err = rel_l2(s.get_fields(0), q_ora)
        terr = rel_l2(s.read_traces(0), tr_ora)
        say("full general mesh shape %s fields %.3e traces %.3e" % (shape, err, terr))
        assert err <= FP64_TOL and terr <= FP64_TOL


def test_mesh_read_from_file_matches_oracle(tmp_path):
    """A general mesh written to an MSH 2.2 file and read back runs to the
    FP64 bar against the oracle on the read mesh."""
    from paper_2205_11052_amd.meshio import read_msh, write_msh
    p = tmp_path / "general.msh"
    write_msh(p, W.general_mesh(4, 2.0, seed=33))
    mesh = read_msh(p, bc_map={1: 1, 2: 2})
    K = mesh["etov"].shape[0]
    say("case mesh from file K=%d" % K)
    rho, lam, mu = _random_medium(K, 44)
    P = oracle_problem(mesh, 4)
    dt = P.suggest_dt(rho, lam, mu, 0.5)
    q0 = random_fields(K, P.Np, 45)
    s = gpu_solver(mesh, 4, rho, lam, mu, dt, kernel=1)
    s.set_fields(0, q0)
    s.step(5)
    q_ora, _ = oracle_run(P, q0, rho, lam, mu, dt, 5)
    err = rel_l2(s.get_fields(0), q_ora)
    say("mesh from file fields %.3e" % err)
    assert err <= FP64_TOL
