"""Helpers for the GPU parity tests: build the library solver and the oracle
problem from the same seeded workload (test code)."""

import sys

import numpy as np
import torch

from oracle import solver as O
from paper_2205_11052_amd import Solver


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def gpu_solver(mesh, N, rho, lam, mu, dt, precision=64, nshots=1, kernel=0):
    s = Solver(N, precision, nshots)
    s.set_mesh_dict(mesh)
    s.set_material(rho, lam, mu)
    s.set_dt(dt)
    if kernel:
        s.set_launch(kernel)
    return s


def oracle_problem(mesh, N):
    return O.Problem(mesh, N)


def oracle_run(P, q0, rho, lam, mu, dt, nsteps, record=False):
    t = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64))
    q, tr = O.run(P, t(q0).clone(), t(rho), t(lam), t(mu), dt, nsteps,
                  record=record)
    return q.numpy(), (tr.numpy() if tr is not None else None)


def random_fields(K, Np, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((K, 9, Np))
