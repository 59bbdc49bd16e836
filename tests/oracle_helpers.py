"""Small helpers shared by the oracle pin tests (test code, not oracle code)."""

import numpy as np
import torch
from torch.func import vmap

import workloads as W
from oracle import solver


def random_medium(K, seed):
    rng = np.random.default_rng(seed)
    cp = rng.uniform(1.5, 3.0, K)
    cs = cp / rng.uniform(1.5, 2.2, K)
    rho = rng.uniform(1.0, 3.0, K)
    return W.lame_from_velocities(cp, cs, rho)


def tensors(*arrs):
    return [solver.as_tensor(a) for a in arrs]


def assemble_L(P, rho, lam, mu):
    """Dense matrix of q -> L q (no source), columns = unit vectors."""
    n = P.K * 9 * P.Np
    f = lambda e: solver.rhs(P, e.view(P.K, 9, P.Np), rho, lam, mu).reshape(-1)
    eye = torch.eye(n, dtype=torch.float64)
    cols = [vmap(f)(eye[s:s + 512]) for s in range(0, n, 512)]
    return torch.cat(cols).T.contiguous().numpy()


def energy_matrix(P, rho, lam, mu):
    """M_E with E(q) = 1/2 q^T M_E q (block diagonal per element)."""
    M = P.ops["M"]
    Np = P.Np
    blocks = []
    for k in range(P.K):
        r, l, m = float(rho[k]), float(lam[k]), float(mu[k])
        c = l / (2 * m * (3 * l + 2 * m))
        S = np.zeros((6, 6))
        S[:3, :3] = np.eye(3) / (2 * m) - c
        S[3:, 3:] = np.eye(3) / m
        W9 = np.zeros((9, 9))
        W9[:3, :3] = r * np.eye(3)
        W9[3:, 3:] = S
        blocks.append(float(P.J[k]) * np.kron(W9, M))
    n = P.K * 9 * Np
    ME = np.zeros((n, n))
    for k, b in enumerate(blocks):
        s = k * 9 * Np
        ME[s:s + 9 * Np, s:s + 9 * Np] = b
    return ME
