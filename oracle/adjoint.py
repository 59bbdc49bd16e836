"""Discrete adjoint gradient of the receiver misfit.

Oracle (test infrastructure).  The gradient of the fully discrete misfit
J(rho, lambda, mu) = 1/2 dt sum_n sum_r sum_c (trace_{n,r,c} - d_{n,r,c})^2
with respect to the per-element rho, lambda, mu is the exact discrete adjoint
of the forward LSERK4 + nodal-DG map.  Here it is obtained by reverse-mode
differentiation (torch.autograd) of the oracle's own forward code, which is by
definition the transpose of every linear step of the discrete forward map; no
hand-written transpose is involved.

Memory is bounded by checkpointing: the forward pass stores the state every
``ckpt_every`` steps; the reverse pass walks the segments backwards,
recomputes each segment from its checkpoint with the graph recorded, and
back-propagates the adjoint state of the segment's end into its start.
"""

import torch

from . import solver


def forward_misfit(P, rho, lam, mu, q0, dt, nsteps, d_obs):
    """Misfit and receiver traces of a forward run (no gradient)."""
    with torch.no_grad():
        _, tr = solver.run(P, q0, rho, lam, mu, dt, nsteps, record=True)
        return solver.misfit(tr, d_obs, dt), tr


def misfit_gradient(P, rho, lam, mu, q0, dt, nsteps, d_obs, ckpt_every=100):
    """(misfit, g_rho, g_lam, g_mu) by checkpointed reverse mode."""
    ckpts = []
    q = q0
    with torch.no_grad():
        for s in range(nsteps):
            if s % ckpt_every == 0:
                ckpts.append((s, q.clone()))
            q = solver.lserk_step(P, q, s * dt, dt, rho, lam, mu)
    g = [torch.zeros_like(rho), torch.zeros_like(lam), torch.zeros_like(mu)]
    adj_q = torch.zeros_like(q0)
    total = torch.zeros((), dtype=q0.dtype)
    for s0, qs in reversed(ckpts):
        s1 = min(s0 + ckpt_every, nsteps)
        params = [p.detach().clone().requires_grad_(True)
                  for p in (rho, lam, mu)]
        qv = qs.detach().clone().requires_grad_(True)
        q = qv
        seg = torch.zeros((), dtype=q0.dtype)
        for s in range(s0, s1):
            q = solver.lserk_step(P, q, s * dt, dt, *params)
            tr = solver.sample_receivers(P, q)
            seg = seg + 0.5 * dt * torch.sum((tr - d_obs[:, :, s]) ** 2)
        obj = seg + torch.sum(adj_q * q)
        grads = torch.autograd.grad(obj, [qv] + params)
        adj_q = grads[0]
        for i in range(3):
            g[i] = g[i] + grads[1 + i]
        total = total + seg.detach()
    return total, g[0], g[1], g[2]
