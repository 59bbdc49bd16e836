"""Full-waveform inversion loop, written out plainly.

Oracle (test infrastructure; only tests, smoke and the benchmark's CPU
baseline use it).  The objective is the receiver misfit summed over shots,
each shot's misfit and gradient from ``adjoint.misfit_gradient`` (reverse
mode through the oracle's own forward code).  Parameters are relative
perturbations x of a reference model, m = m_ref (1 + x) on the inverted
components.

Optimiser: limited-memory BFGS as in Nocedal and Wright, Numerical
Optimization (2nd ed., 2006):
* search direction d = -H g from the two-loop recursion (Algorithm 7.4),
  the initial matrix gamma I with gamma = s^T y / (y^T y) of the newest
  stored pair (eq. 7.20), identity-free steepest descent when no pair is
  stored;
* backtracking line search (Algorithm 3.1): trial steps alpha, alpha/2,
  ... until f(x + alpha d) <= f(x) + 1e-4 alpha g^T d, at most 20 trials;
  the first trial is alpha = step0 / max|g| when no pair is stored (so the
  largest parameter change is step0) and alpha = 1 otherwise;
* a pair (s, y) is stored only if s^T y > 1e-12 |s| |y|, the oldest one
  dropped beyond ``memory`` pairs; a direction that is not a descent
  direction restarts from steepest descent with no pairs.
"""

import math

import numpy as np
import torch

from . import adjoint
from . import solver as OS


def two_loop(g, pairs):
    """H g for the L-BFGS matrix of the stored (s, y) pairs (oldest first)."""
    q = list(g)
    dot = lambda a, b: math.fsum(u * v for u, v in zip(a, b))
    alphas = []
    for s, y in reversed(pairs):
        rho = 1.0 / dot(y, s)
        a = rho * dot(s, q)
        q = [qi - a * yi for qi, yi in zip(q, y)]
        alphas.append(a)
    alphas.reverse()
    if pairs:
        s, y = pairs[-1]
        gamma = dot(s, y) / dot(y, y)
        q = [gamma * qi for qi in q]
    for (s, y), a in zip(pairs, alphas):
        rho = 1.0 / dot(y, s)
        b = rho * dot(y, q)
        q = [qi + (a - b) * si for qi, si in zip(q, s)]
    return q


def minimise(fg, x0, iterations, memory=5, step0=0.05):
    """fg(x) -> (f, g).  Returns (x, list of f after each iteration, the
    first entry at x0)."""
    dot = lambda a, b: math.fsum(u * v for u, v in zip(a, b))
    x = [float(v) for v in x0]
    f, g = fg(x)
    g = [float(v) for v in g]
    history = [float(f)]
    pairs = []
    for _ in range(iterations):
        gmax = max(abs(v) for v in g)
        if gmax == 0.0:
            break
        if pairs:
            d = [-v for v in two_loop(g, pairs)]
            alpha = 1.0
        else:
            d = [-v for v in g]
            alpha = step0 / gmax
        slope = dot(g, d)
        if slope >= 0.0:
            pairs = []
            d = [-v for v in g]
            slope = -dot(g, g)
            alpha = step0 / gmax
        for _trial in range(20):
            xt = [xi + alpha * di for xi, di in zip(x, d)]
            ft, gt = fg(xt)
            if ft <= f + 1e-4 * alpha * slope:
                break
            alpha *= 0.5
        else:
            break
        gt = [float(v) for v in gt]
        s = [a - b for a, b in zip(xt, x)]
        y = [a - b for a, b in zip(gt, g)]
        ns = math.sqrt(dot(s, s))
        ny = math.sqrt(dot(y, y))
        if dot(s, y) > 1e-12 * ns * ny:
            pairs.append((s, y))
            if len(pairs) > memory:
                pairs.pop(0)
        x, f, g = xt, ft, gt
        history.append(float(f))
    return x, history


def shots_objective(P, shots, d_obs, m_ref, which, dt, nsteps, ckpt_every):
    """fg(x) for the misfit summed over shots.  shots: list of
    (position, f0, t0, amp, moment); d_obs [S][R][3][nsteps]; m_ref the
    reference (rho, lam, mu) [K] arrays; which: indices into (rho, lam, mu)
    of the inverted components."""
    K = len(m_ref[0])
    ref = [np.asarray(a, dtype=np.float64) for a in m_ref]

    def fg(x):
        m = [a.copy() for a in ref]
        for i, c in enumerate(which):
            m[c] = ref[c] * (1.0 + np.asarray(x[i * K:(i + 1) * K]))
        t = [torch.as_tensor(a) for a in m]
        total = 0.0
        grad = [np.zeros(K) for _ in range(3)]
        for s, (pos, f0, t0, amp, moment) in enumerate(shots):
            P.set_source(pos, f0, t0, amp, moment=moment)
            q0 = torch.zeros(K, 9, P.Np, dtype=torch.float64)
            d = torch.as_tensor(np.asarray(d_obs[s], dtype=np.float64))
            J, gr, gl, gm = adjoint.misfit_gradient(P, t[0], t[1], t[2], q0, dt,
                                                    nsteps, d, ckpt_every)
            total += float(J)
            for c, gc in enumerate((gr, gl, gm)):
                grad[c] += gc.detach().numpy()
        g = np.concatenate([ref[c] * grad[c] for c in which])
        return total, list(g)

    return fg


def observed(P, shots, m, dt, nsteps):
    """Receiver traces [S][R][3][nsteps] of every shot in model m, from zero
    fields."""
    t = [torch.as_tensor(np.asarray(a, dtype=np.float64)) for a in m]
    out = []
    for pos, f0, t0, amp, moment in shots:
        P.set_source(pos, f0, t0, amp, moment=moment)
        q0 = torch.zeros(len(m[0]), 9, P.Np, dtype=torch.float64)
        _, tr = OS.run(P, q0, t[0], t[1], t[2], dt, nsteps, record=True)
        out.append(tr.numpy())
    return np.stack(out)
