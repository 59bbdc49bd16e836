"""Convolutional perfectly matched layer (C-PML) for the nodal DG scheme.

Oracle (test infrastructure), plain PyTorch CPU in FP64.  The paper (arXiv
2205.11052) does not describe this method; each function states the formula
it implements.

Continuous model (the recursive-convolution PML of Roden and Gedney, 2000,
in the unsplit first-order form of Komatitsch and Martin, Geophysics 72,
2007, with the stretching factor kappa = 1): inside the layer each spatial
derivative d/dx_b is replaced by d/dx_b + (memory variable), the memory
variable of a derivative du/dx_b obeying
    m_t = -(d_b + alpha_b) m - d_b du/dx_b,
with d_b >= 0 the damping profile and alpha_b >= 0 the frequency shift of
axis b (given per element [K, 3] or per node [K, 3, Np]; where d_b = 0 a
memory variable that starts at zero stays zero).  For the velocity-stress system this gives
    rho v_c,t = sum_b (D_cb + phi_cb),
    sigma_t   = lambda tr(G + Psi) I + mu (G + Psi + (G + Psi)^T),
    phi_cb,t  = -(d_b + alpha_b) phi_cb - d_b D_cb,
    psi_cb,t  = -(d_b + alpha_b) psi_cb - d_b G_cb,
where D_cb = d sigma_cb / dx_b (no sum) and G_cb = d v_c / dx_b.

Discrete directional derivatives (the scheme's own, split by axis): with
dT = t* - t- and dV = v* - v- the flux-state changes of the scheme on each
face node and n the outward normal,
    G_cb = sum_r Xinv[r, b] D_r v_c + sum_f Fscale_f LIFT_f (n_b dV_c),
    D_cb = sum_r Xinv[r, b] D_r sigma_cb + sum_f Fscale_f LIFT_f (n_b S_cb),
where S = dT n^T + n dT^T - (n.dT) n n^T is the symmetric stress change whose
traction is dT (S n = dT, since |n| = 1).  Summed over b these reproduce the
scheme's right-hand side exactly: sum_b D_cb = rho (L q)_v_c and
lambda tr(G) I + mu (G + G^T) = (L q)_sigma.  So with d = 0 the layer is
the plain scheme, and the layer adds
    dL_v = (1/rho) sum_b phi_cb,  dL_sigma = lambda tr(Psi) I + mu (Psi + Psi^T)
to L q (isotropic elements only; a sponge set on the problem still acts).

State: q [K, 9, Np] and the memory variables m [K, 18, Np] with
m[:, 3c + b] = phi_cb and m[:, 9 + 3c + b] = psi_cb (c, b = x, y, z).  Both
advance with the same LSERK4 stages as the scheme (res = A_i res +
dt rate(q, m), then q, m += B_i res, the rates taken at the stage input).
"""

import torch

from . import solver as S


def directional(P, q, rho, lam, mu):
    """Directional derivatives (D [K, 3, 3, Np], G [K, 3, 3, Np]) of state q;
    D[:, c, b] = d sigma_cb / dx_b, G[:, c, b] = d v_c / dx_b, volume and face
    parts as in the module docstring."""
    if P.stiffness is not None:
        raise ValueError("the perfectly matched layer is isotropic only")
    dt_ = q.dtype
    K, Nfp = P.K, P.Nfp
    Xinv = P.Xinv.to(dt_)
    ref = torch.stack([q @ P.Dr.to(dt_).T, q @ P.Ds.to(dt_).T, q @ P.Dt.to(dt_).T],
                      dim=2)                                       # [K,9,3,Np]
    grad = torch.einsum("krb,kcrn->kcbn", Xinv, ref)              # [K,9,3,Np]
    # stress component index of sigma_cb (Voigt order xx yy zz yz xz xy)
    voigt = [[S.SXX, S.SXY, S.SXZ], [S.SXY, S.SYY, S.SYZ], [S.SXZ, S.SYZ, S.SZZ]]
    Dv = torch.stack([torch.stack([grad[:, voigt[c][b], b] for b in range(3)], dim=1)
                      for c in range(3)], dim=1)                   # [K,3,3,Np]
    Gv = grad[:, 0:3]                                              # [K,3,3,Np]

    dT, dV, n = S.face_states(P, q, rho, lam, mu)                  # [K,3,4,Nfp]
    nn = n[:, :, :, 0]                                             # [K,3,4]
    ndT = (n * dT).sum(dim=1)                                      # [K,4,Nfp]
    # S_cb = dT_c n_b + n_c dT_b - (n.dT) n_c n_b on every face node
    Sst = (dT[:, :, None] * n[:, None, :] + n[:, :, None] * dT[:, None, :]
           - ndT[:, None, None] * n[:, :, None] * n[:, None, :])   # [K,3,3,4,Nfp]
    fs = P.Fscale.to(dt_)[:, None, None, :, None]                  # [K,1,1,4,1]
    nb = nn[:, None, :, :, None]                                   # n_b [K,1,3,4,1]
    Dface = fs * nb * Sst                                          # [K,3,3,4,Nfp]
    Gface = fs * nb * dV[:, :, None]                               # [K,3,3,4,Nfp]
    LT = P.LIFT.to(dt_).T
    Df = Dface.reshape(K, 3, 3, 4 * Nfp) @ LT
    Gf = Gface.reshape(K, 3, 3, 4 * Nfp) @ LT
    return Dv + Df, Gv + Gf


def layer_terms(m, rho, lam, mu):
    """dL(m) [K, 9, Np]: what the memory variables add to L q."""
    phi = m[:, 0:9].reshape(m.shape[0], 3, 3, -1)
    psi = m[:, 9:18].reshape(m.shape[0], 3, 3, -1)
    r = rho[:, None]
    l = lam[:, None]
    u = mu[:, None]
    tr = psi[:, 0, 0] + psi[:, 1, 1] + psi[:, 2, 2]
    return torch.stack([
        phi[:, 0].sum(dim=1) / r,
        phi[:, 1].sum(dim=1) / r,
        phi[:, 2].sum(dim=1) / r,
        l * tr + 2.0 * u * psi[:, 0, 0],
        l * tr + 2.0 * u * psi[:, 1, 1],
        l * tr + 2.0 * u * psi[:, 2, 2],
        u * (psi[:, 1, 2] + psi[:, 2, 1]),
        u * (psi[:, 0, 2] + psi[:, 2, 0]),
        u * (psi[:, 0, 1] + psi[:, 1, 0]),
    ], dim=1)


def memory_rate(P, q, m, rho, lam, mu, d, alpha):
    """m_t [K, 18, Np] for the damping profile d and shift alpha, per element
    [K, 3] or per node [K, 3, Np]."""
    D, G = directional(P, q, rho, lam, mu)
    # d_b, alpha_b per element [K, 3] or per node [K, 3, Np]
    ex = (lambda a: a[:, None, :, None]) if d.dim() == 2 else (lambda a: a[:, None])
    db = ex(d.to(q.dtype))
    ab = ex(alpha.to(q.dtype))
    K = q.shape[0]
    phi = m[:, 0:9].reshape(K, 3, 3, -1)
    psi = m[:, 9:18].reshape(K, 3, 3, -1)
    rphi = -(db + ab) * phi - db * D
    rpsi = -(db + ab) * psi - db * G
    return torch.cat([rphi.reshape(K, 9, -1), rpsi.reshape(K, 9, -1)], dim=1)


def lserk_step(P, q, m, t, dt, rho, lam, mu, d, alpha):
    """One LSERK4 step of (q, m) from time t; returns the new (q, m)."""
    rq = torch.zeros_like(q)
    rm = torch.zeros_like(m)
    for i in range(5):
        tau = t + S.LSERK_C[i] * dt
        Lq = S.rhs(P, q, rho, lam, mu) + S.source_term(P, tau, q.dtype) \
            + layer_terms(m, rho, lam, mu)
        Lm = memory_rate(P, q, m, rho, lam, mu, d, alpha)
        rq = S.LSERK_A[i] * rq + dt * Lq
        rm = S.LSERK_A[i] * rm + dt * Lm
        q = q + S.LSERK_B[i] * rq
        m = m + S.LSERK_B[i] * rm
    return q, m


def run(P, q0, rho, lam, mu, d, alpha, dt, nsteps, m0=None, t0=0.0, record=False):
    """Advance (q, m) nsteps; returns (q, m, traces [nrec, 3, nsteps] or None)."""
    q = q0
    m = torch.zeros(q0.shape[0], 18, q0.shape[2], dtype=q0.dtype) if m0 is None else m0
    traces = []
    for s in range(nsteps):
        q, m = lserk_step(P, q, m, t0 + s * dt, dt, rho, lam, mu, d, alpha)
        if record:
            traces.append(S.sample_receivers(P, q))
    tr = torch.stack(traces, dim=2) if record and traces else None
    return q, m, tr
