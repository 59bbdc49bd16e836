"""Pins of the oracle's convolutional perfectly matched layer (oracle.pml).

* The directional split adds up to the scheme: for any state, on meshes with
  free-surface and absorbing faces, fluid elements and the blended flux,
  sum_b D_cb = rho (L q)_v_c and lambda tr(G) I + mu (G + G^T) = (L q)_sigma,
  where L is the scheme's right-hand side (pinned on its own elsewhere).
* Exactness on polynomials: for a globally linear state every jump vanishes,
  so on elements with no boundary face D_cb and G_cb are the exact partial
  derivatives d sigma_cb / dx_b and d v_c / dx_b of that state (a swapped
  index or a wrong component map fails this).
* With a zero profile a step is the plain scheme's step bit for bit and the
  memory variables stay zero; with d = 0 and a constant shift alpha the
  memory variables obey m_t = -alpha m, so they decay as exp(-alpha t) to
  the integrator's fourth-order error while the state is driven by them.
* The memory rate at m = 0 is -d_b times the directional derivative.
* Absorption: a P-wave pulse on a quasi-one-dimensional periodic column,
  measured against the same run on a column long enough that nothing returns:
  the reflection off a free surface behind the layer falls well below the
  sponge's at equal width (``test_pml_reflects_less_than_the_sponge``).
"""

import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import pml as OP
from oracle import solver as O
from oracle_helpers import random_medium, tensors


def _bounded_mesh():
    # free surface on top (kuhn_cube) plus absorbing elsewhere
    return W.kuhn_cube(2, 1.0)


@pytest.mark.parametrize("N", [1, 2, 3])
@pytest.mark.parametrize("tau,fluid", [(1.0, 0), (0.5, 0), (1.0, 10)])
def test_split_adds_up_to_the_scheme(N, tau, fluid):
    mesh = _bounded_mesh()
    K = mesh["etov"].shape[0]
    rho, lam, mu = random_medium(K, 3 + N)
    if fluid:
        mu = mu.copy()
        mu[np.random.default_rng(1).choice(K, fluid, replace=False)] = 0.0
    rho, lam, mu = tensors(rho, lam, mu)
    P = O.Problem(mesh, N)
    P.flux_tau = tau
    q = torch.as_tensor(np.random.default_rng(N).standard_normal((K, 9, P.Np)))
    D, G = OP.directional(P, q, rho, lam, mu)
    L = O.rhs(P, q, rho, lam, mu)
    sv = D.sum(dim=2) / rho[:, None, None]
    assert torch.allclose(sv, L[:, 0:3], rtol=0, atol=1e-12 * L[:, 0:3].abs().max())
    m = torch.zeros(K, 18, P.Np, dtype=torch.float64)
    m[:, 9:18] = G.reshape(K, 9, P.Np)
    Ls = OP.layer_terms(m, rho, lam, mu)
    assert torch.allclose(Ls[:, 3:9], L[:, 3:9], rtol=0,
                          atol=1e-12 * L[:, 3:9].abs().max())
    # and the velocity part of layer_terms is (1/rho) sum_b phi_cb
    m = torch.zeros(K, 18, P.Np, dtype=torch.float64)
    m[:, 0:9] = D.reshape(K, 9, P.Np)
    Lv = OP.layer_terms(m, rho, lam, mu)
    assert torch.allclose(Lv[:, 0:3], L[:, 0:3], rtol=0,
                          atol=1e-12 * L[:, 0:3].abs().max())


@pytest.mark.parametrize("N", [1, 3])
def test_directional_derivatives_of_a_linear_state(N):
    mesh = W.kuhn_cube(3, 1.0)
    K = mesh["etov"].shape[0]
    rho, lam, mu = tensors(*random_medium(K, 9))
    P = O.Problem(mesh, N)
    X = W.lattice_node_coords(mesh, N)                             # [K, Np, 3]
    A = np.random.default_rng(4).standard_normal((9, 3))           # d field_c / dx_b
    c0 = np.random.default_rng(5).standard_normal(9)
    q = torch.as_tensor(np.einsum("cb,knb->kcn", A, X) + c0[None, :, None])
    D, G = OP.directional(P, q, rho, lam, mu)
    inner = ~torch.as_tensor((P.bc > 0).any(axis=1))               # no boundary face
    assert inner.sum() > 0
    voigt = [[3, 8, 7], [8, 4, 6], [7, 6, 5]]
    for c in range(3):
        for b in range(3):
            want_D = A[voigt[c][b], b]
            want_G = A[c, b]
            assert torch.allclose(D[inner, c, b], torch.full_like(D[inner, c, b], want_D),
                                  rtol=0, atol=1e-11)
            assert torch.allclose(G[inner, c, b], torch.full_like(G[inner, c, b], want_G),
                                  rtol=0, atol=1e-11)


def test_zero_profile_is_the_plain_scheme():
    mesh = _bounded_mesh()
    K = mesh["etov"].shape[0]
    rho, lam, mu = tensors(*random_medium(K, 2))
    P = O.Problem(mesh, 2)
    P.set_source(np.array([0.4, 0.5, 0.6]), 3.0, 0.1, 1.0)
    q = torch.as_tensor(np.random.default_rng(0).standard_normal((K, 9, P.Np)))
    z = torch.zeros(K, 3, P.Np, dtype=torch.float64)
    dt = 1e-3
    qp = O.lserk_step(P, q, 0.0, dt, rho, lam, mu)
    ql, ml = OP.lserk_step(P, q, torch.zeros(K, 18, P.Np, dtype=torch.float64), 0.0,
                           dt, rho, lam, mu, z, z)
    assert torch.equal(qp, ql)
    assert not ml.any()


def test_memory_decays_at_the_shift_rate():
    mesh = _bounded_mesh()
    K = mesh["etov"].shape[0]
    rho, lam, mu = tensors(*random_medium(K, 6))
    P = O.Problem(mesh, 2)
    rng = np.random.default_rng(12)
    m0 = torch.as_tensor(rng.standard_normal((K, 18, P.Np)))
    q0 = torch.zeros(K, 9, P.Np, dtype=torch.float64)
    alpha = 3.0
    z = torch.zeros(K, 3, P.Np, dtype=torch.float64)
    al = torch.full_like(z, alpha)
    T = 0.2
    errs = []
    for n in (10, 20):
        q, m, _ = OP.run(P, q0, rho, lam, mu, z, al, T / n, n, m0=m0.clone())
        errs.append((m - m0 * math.exp(-alpha * T)).abs().max().item())
        # the layer's terms drive the state
        assert q.abs().max() > 1e-3
    rate = math.log2(errs[0] / errs[1])
    assert errs[1] < 1e-7 and rate > 3.7, (errs, rate)


def test_memory_rate_at_rest_is_minus_d_times_the_derivative():
    mesh = _bounded_mesh()
    K = mesh["etov"].shape[0]
    rho, lam, mu = tensors(*random_medium(K, 8))
    P = O.Problem(mesh, 3)
    rng = np.random.default_rng(2)
    q = torch.as_tensor(rng.standard_normal((K, 9, P.Np)))
    d = torch.as_tensor(rng.uniform(0.0, 5.0, (K, 3, P.Np)))
    a = torch.as_tensor(rng.uniform(0.0, 2.0, (K, 3, P.Np)))
    D, G = OP.directional(P, q, rho, lam, mu)
    r = OP.memory_rate(P, q, torch.zeros(K, 18, P.Np, dtype=torch.float64),
                       rho, lam, mu, d, a)
    for c in range(3):
        for b in range(3):
            assert torch.equal(r[:, 3 * c + b], -d[:, b] * D[:, c, b])
            assert torch.equal(r[:, 9 + 3 * c + b], -d[:, b] * G[:, c, b])


# ---- absorption against the sponge ------------------------------------------

H = 0.25            # cell size of the columns (3 x 3 cells across, periodic)
CP, CS, RHO = 2.0, 1.2, 1.0


def _column(nx, ny, N, free_end):
    mesh = W.kuhn_box(nx, ny, 3, nx * H, ny * H, 3 * H, periodic=(False, True, True),
                      free_faces=("x+",) if free_end else ())
    K = mesh["etov"].shape[0]
    P = O.Problem(mesh, N)
    mat = tensors(*W.lame_from_velocities(np.full(K, CP), np.full(K, CS), np.full(K, RHO)))
    return mesh, P, mat


def _pulse(mesh, N, mat, direction, profile):
    """P-wave travelling along `direction`: v = d f, sigma = -(lambda I +
    2 mu d d^T) f / cp with f the given profile of the node coordinates."""
    X = W.lattice_node_coords(mesh, N)
    d = np.asarray(direction, dtype=np.float64)
    lam, mu = float(mat[1][0]), float(mat[2][0])
    S = -(lam * np.eye(3) + 2.0 * mu * np.outer(d, d)) / CP
    f = profile(X)
    q = np.zeros((X.shape[0], 9, X.shape[1]))
    q[:, 0:3] = np.moveaxis(f[..., None] * d, -1, 1)
    for a, (i, j) in enumerate([(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]):
        q[:, 3 + a] = S[i, j] * f
    return torch.as_tensor(q)


def _reflections(direction, profile, ny, n_in, n_ref, T, t_meas, f0, sponges):
    """Reflection amplitude of each absorber: the largest over t in
    [t_meas, T] of sqrt(E_in(q - q_ref) / E_in(q0)), E_in the energy of the
    interior cells x < n_in H.  The absorber (4 cells, width 1) sits between
    the interior and a free surface; q_ref is the run on a column of n_ref
    cells with no absorber, so long that nothing comes back before T.
    Returns ({sigma_max: amplitude}, pml amplitude)."""
    N, nl, dt = 2, 4, 0.02
    nx = n_in + nl
    mR, PR, matR = _column(n_ref, ny, N, False)
    mA, PA, matA = _column(nx, ny, N, True)
    # element of the reference column in the same cell and tetrahedron
    e = np.arange(mA["etov"].shape[0])
    c, p = e // 6, e % 6
    i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
    to_ref = torch.as_tensor(6 * (i + n_ref * (j + ny * k)) + p)
    assert np.allclose(mR["vxyz"][mR["etov"][to_ref.numpy()]], mA["vxyz"][mA["etov"]])
    inner = torch.as_tensor(W.element_centroids(mA)[:, 0] < n_in * H)

    def e_in(dq):
        z = dq.clone()
        z[~inner] = 0
        return O.energy(PA, z, *matA).item()

    nsteps = int(round(T / dt))
    meas = [s for s in range(nsteps) if (s + 1) * dt >= t_meas - 1e-9 and (s + 1) % 5 == 0]
    q = _pulse(mR, N, matR, direction, profile)
    ref = {}
    for s in range(nsteps):
        q = O.lserk_step(PR, q, s * dt, dt, *matR)
        if s in meas:
            ref[s] = q[to_ref]
    q0 = _pulse(mA, N, matA, direction, profile)
    E0 = e_in(q0)
    hi = (nx * H, ny * H, 3 * H)
    cen = W.element_centroids(mA)

    def amplitude(step):
        q, m, worst = q0, None, 0.0
        for s in range(nsteps):
            q, m = step(q, m, s)
            if s in meas:
                worst = max(worst, e_in(q - ref[s]))
        return math.sqrt(worst / E0)

    out = {}
    for sm in sponges:
        PA.sponge = torch.as_tensor(W.sponge_profile(cen, hi=hi, width=nl * H,
                                                     sigma_max=sm, faces=("x+",)))
        out[sm] = amplitude(lambda q, m, s: (O.lserk_step(PA, q, s * dt, dt, *matA), None))
    PA.sponge = None
    _, _, d, a = W.pml_layer(mA, N, hi=hi, width=nl * H, cp_max=CP, reflection=1e-4,
                             f0=f0, faces=("x+",))
    d, a = torch.as_tensor(d), torch.as_tensor(a)
    zero_m = torch.zeros(q0.shape[0], 18, PA.Np, dtype=torch.float64)
    pml = amplitude(lambda q, m, s: OP.lserk_step(PA, q, zero_m if m is None else m,
                                                  s * dt, dt, *matA, d, a))
    return out, pml


def test_pml_reflects_less_than_the_sponge_at_normal_incidence():
    # Ricker pulse of peak frequency 1 (wavelength 2) at x = 1.5; the layer
    # is half a wavelength wide
    f0 = 1.0

    def ricker(X):
        a2 = (math.pi * f0 * (X[..., 0] - 1.5) / CP) ** 2
        return (1.0 - 2.0 * a2) * np.exp(-a2)

    sp, pml = _reflections((1.0, 0.0, 0.0), ricker, ny=3, n_in=12, n_ref=34, T=3.2,
                           t_meas=1.6, f0=f0, sponges=(16.0, 32.0, 64.0))
    # measured: sponge 5.4e-3, 2.3e-3, >= 2.3e-3; layer 8.2e-4
    best = min(sp.values())
    assert best < 0.05 and pml < 0.5 * best, (sp, pml)


def test_pml_reflects_less_than_the_sponge_at_oblique_incidence():
    # wave packet at 45 degrees: wavevector (k, k, 0)/sqrt(2) with k sin 45
    # one period across the 1.5-wide periodic column, Gaussian envelope in x
    ny = 6
    k = (2.0 * math.pi / (ny * H)) / math.sin(math.pi / 4)
    d = np.array([1.0, 1.0, 0.0]) / math.sqrt(2.0)
    w = 1.2 * CP / (math.pi * 2.0)

    def packet(X):
        return np.exp(-((X[..., 0] - 1.0) / w) ** 2) * np.cos(k * (X @ d - d[0]))

    sp, pml = _reflections(d, packet, ny=ny, n_in=8, n_ref=22, T=2.5, t_meas=1.0,
                           f0=2.0, sponges=(16.0, 32.0))
    # measured: sponge 9.9e-2, 1.2e-1; layer 3.0e-3
    assert pml < 0.1 * min(sp.values()), (sp, pml)
