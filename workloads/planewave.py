"""Exact plane-wave solutions of the isotropic velocity-stress system.

For a unit direction d and a profile f(xi) = sin(k * xi):

* P wave (speed cp): v = d f(d.x - cp t),
  sigma = -(1/cp) (lambda I + 2 mu d d^T) f(d.x - cp t);
* S wave (speed cs, polarisation p orthogonal to d): v = p f(d.x - cs t),
  sigma = -(mu/cs) (p d^T + d p^T) f(d.x - cs t).

Substituting into rho v_t = div(sigma) and sigma_t = lambda div(v) I +
mu (grad v + grad v^T) gives cp^2 = (lambda + 2 mu)/rho and cs^2 = mu/rho.

Field order of the returned state: (vx, vy, vz, sxx, syy, szz, syz, sxz, sxy).
"""

import numpy as np


def plane_wave_state(x, t, kind, direction, wavenumber, rho, lam, mu,
                     polarization=None):
    """Evaluate the plane wave at points x [..., 3]; returns [..., 9]."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    x = np.asarray(x, dtype=np.float64)
    if kind == "P":
        c = np.sqrt((lam + 2.0 * mu) / rho)
        p = d
        S = -(lam * np.eye(3) + 2.0 * mu * np.outer(d, d)) / c
    elif kind == "S":
        c = np.sqrt(mu / rho)
        p = np.asarray(polarization, dtype=np.float64)
        p = p - np.dot(p, d) * d
        p = p / np.linalg.norm(p)
        S = -(mu / c) * (np.outer(p, d) + np.outer(d, p))
    else:
        raise ValueError(kind)
    f = np.sin(wavenumber * (x @ d - c * t))
    out = np.empty(x.shape[:-1] + (9,), dtype=np.float64)
    out[..., 0:3] = f[..., None] * p
    out[..., 3] = S[0, 0] * f
    out[..., 4] = S[1, 1] * f
    out[..., 5] = S[2, 2] * f
    out[..., 6] = S[1, 2] * f
    out[..., 7] = S[0, 2] * f
    out[..., 8] = S[0, 1] * f
    return out


def anisotropic_plane_wave_state(x, t, direction, wavenumber, rho, C, mode):
    """Plane wave in a homogeneous anisotropic medium (Voigt stiffness C
    [6, 6], order xx yy zz yz xz xy, engineering shears): with the
    Christoffel matrix G(d)_ik = sum_jl C_ijkl d_j d_l, mode m (0, 1, 2 by
    increasing speed) has G p = rho c^2 p, |p| = 1, and
    v = p f(d.x - c t), sigma = -(1/c) C e(p, d) f(d.x - c t), where
    e(p, d) is the Voigt strain of sym(p d^T).  Substituting into
    rho v_t = div(sigma) and sigma_t = C e(grad v) gives back G p = rho c^2 p.
    Returns [..., 9] at points x [..., 3]."""
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    C = np.asarray(C, dtype=np.float64)
    # full tensor from Voigt (index pairs 00 11 22 12 02 01)
    pairs = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    vi = {}
    for a, (i, j) in enumerate(pairs):
        vi[(i, j)] = vi[(j, i)] = a
    Ct = np.empty((3, 3, 3, 3))
    for i in range(3):
        for j in range(3):
            for k in range(3):
                for l in range(3):
                    Ct[i, j, k, l] = C[vi[(i, j)], vi[(k, l)]]
    G = np.einsum("ijkl,j,l->ik", Ct, d, d)
    w, V = np.linalg.eigh(G / rho)
    c = np.sqrt(w[mode])
    p = V[:, mode]
    sig = -np.einsum("ijkl,k,l->ij", Ct, p, d) / c        # symmetric in i, j
    f = np.sin(wavenumber * (np.asarray(x, dtype=np.float64) @ d - c * t))
    out = np.empty(f.shape + (9,), dtype=np.float64)
    out[..., 0:3] = f[..., None] * p
    for a, (i, j) in enumerate(pairs):
        out[..., 3 + a] = sig[i, j] * f
    return out
