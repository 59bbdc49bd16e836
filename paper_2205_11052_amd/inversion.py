"""Full-waveform inversion over the batched per-shot gradients.

The objective is the summed receiver misfit of all shots,
J(m) = sum_s 1/2 dt sum_n sum_r sum_c (trace - d_obs)^2, as a function of the
per-element (rho, lambda, mu).  Every forward sweep (with checkpoints) and
every reverse sweep runs in the library (dgw_forward_checkpointed,
dgw_adjoint: one launch per stage over all shots); the host does only the
optimiser's vector arithmetic on the 3K parameters.

Parameters are relative perturbations x of a reference model:
m = m_ref * (1 + x) for the inverted components, the others held at m_ref,
so dJ/dx = m_ref * dJ/dm (summed over shots).

The optimiser is limited-memory BFGS (Nocedal and Wright, Numerical
Optimization, 2nd ed., 2006: the two-loop recursion of Algorithm 7.4 with the
initial matrix gamma I, gamma = s^T y / y^T y of the newest pair, eq. 7.20)
with a backtracking line search on the sufficient-decrease (Armijo)
condition (Algorithm 3.1).  The first direction is steepest descent with
the step scaled so the largest parameter change is ``step0``; later steps
start at alpha = 1.  A pair is kept only when s^T y > 1e-12 |s| |y|.
"""

import numpy as np

COMPONENTS = ("rho", "lam", "mu")


def lbfgs(value, grad, x0, iterations, memory=5, step0=0.05, c1=1e-4,
          shrink=0.5, max_backtracks=20):
    """Minimise with L-BFGS.

    value(x) -> f at x; grad() -> the gradient at the x of the latest
    value() call (so a trial point's forward run serves its gradient).
    Returns (x, history) with history[i] = {"f", "evals", "alpha"} after
    iteration i (entry 0: the start).  Stops early when the gradient
    vanishes or the line search fails.
    """
    x = np.array(x0, dtype=np.float64)
    f = value(x)
    g = np.array(grad(), dtype=np.float64)
    hist = [{"f": float(f), "evals": 1, "alpha": 0.0}]
    S, Y = [], []
    for _ in range(iterations):
        gmax = float(np.max(np.abs(g))) if g.size else 0.0
        if gmax == 0.0:
            break
        # two-loop recursion: d = -H g
        q = g.copy()
        rho_a = []
        for s, y in zip(reversed(S), reversed(Y)):
            r = 1.0 / float(y @ s)
            a = r * float(s @ q)
            q -= a * y
            rho_a.append((r, a))
        if S:
            q *= float(S[-1] @ Y[-1]) / float(Y[-1] @ Y[-1])
        for (s, y), (r, a) in zip(zip(S, Y), reversed(rho_a)):
            b = r * float(y @ q)
            q += (a - b) * s
        d = -q
        alpha = step0 / gmax if not S else 1.0
        slope = float(g @ d)
        if slope >= 0.0:           # not a descent direction: restart
            S, Y = [], []
            d = -g
            slope = -float(g @ g)
            alpha = step0 / gmax
        evals = 0
        accepted = False
        for _ in range(max_backtracks):
            x_new = x + alpha * d
            f_new = value(x_new)
            evals += 1
            if f_new <= f + c1 * alpha * slope:
                accepted = True
                break
            alpha *= shrink
        if not accepted:
            break
        g_new = np.array(grad(), dtype=np.float64)
        s = x_new - x
        y = g_new - g
        if float(s @ y) > 1e-12 * float(np.linalg.norm(s) * np.linalg.norm(y)):
            S.append(s)
            Y.append(y)
            if len(S) > memory:
                S.pop(0)
                Y.pop(0)
        x, f, g = x_new, f_new, g_new
        hist.append({"f": float(f), "evals": evals, "alpha": float(alpha)})
    return x, hist


class MisfitObjective:
    """J(x) of all the solver's shots from zero fields, over the relative
    perturbations x of ``m_ref`` = (rho, lam, mu) in the components
    ``which``; x is laid out component-major, K values each."""

    def __init__(self, solver, d_obs, nsteps, ckpt_every, m_ref,
                 which=COMPONENTS):
        self.solver = solver
        self.d_obs = np.ascontiguousarray(d_obs, dtype=np.float64)
        self.nsteps = int(nsteps)
        self.ckpt = int(ckpt_every)
        self.m_ref = [np.asarray(a, dtype=np.float64) for a in m_ref]
        self.which = [COMPONENTS.index(c) for c in which]
        self.K = self.m_ref[0].shape[0]
        self.evaluations = 0
        self.gradients = 0

    def model(self, x):
        m = [a.copy() for a in self.m_ref]
        for i, c in enumerate(self.which):
            m[c] = self.m_ref[c] * (1.0 + x[i * self.K:(i + 1) * self.K])
        return m

    def value(self, x):
        rho, lam, mu = self.model(x)
        self.solver.set_material(rho, lam, mu)
        self.solver.zero_fields()
        mis = self.solver.forward_checkpointed(self.nsteps, self.ckpt, self.d_obs)
        self.evaluations += 1
        return float(np.sum(mis))

    def grad(self):
        g = self.solver.adjoint()                  # 3 x [nshots][K]
        self.gradients += 1
        out = [self.m_ref[c] * g[c].sum(axis=0) for c in self.which]
        return np.concatenate(out)


def invert(solver, d_obs, nsteps, ckpt_every, m_ref, iterations,
           which=COMPONENTS, memory=5, step0=0.05):
    """L-BFGS inversion from m_ref; returns (model, history, objective)."""
    obj = MisfitObjective(solver, d_obs, nsteps, ckpt_every, m_ref, which)
    x0 = np.zeros(obj.K * len(obj.which))
    x, hist = lbfgs(obj.value, obj.grad, x0, iterations, memory=memory,
                    step0=step0)
    return obj.model(x), hist, obj
