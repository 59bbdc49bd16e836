"""Pin of where the oracle evaluates the point source inside an LSERK4 step.

With the source, the semi-discrete system is the forced linear ODE
q' = L q + s(t) b (b the projected moment-tensor source, s the Ricker
wavelet).  A Runge-Kutta method keeps its classical order on a forced
problem only when stage i evaluates the forcing at the stage time
t_n + c_i dt, with c_i the abscissae of its Butcher tableau; for the
Carpenter-Kennedy 2N-storage scheme these are the C_i of its table.
Evaluating the forcing at t_n in every stage, or at t_n + B_i dt, makes the
method first order in the forcing.

The reference here is independent of the oracle's time stepping: the same
ODE, with L assembled column by column from the oracle's right-hand side,
integrated by scipy's DOP853 at a tolerance far below the errors measured.
From zero fields the oracle's source-driven run must converge to it at
observed order close to 4 under dt, dt/2, dt/4; the planted readings
(t_n, or B_i as stage times) must converge at order below 2.
"""

import math

import numpy as np
import pytest
import torch
from scipy.integrate import solve_ivp

import workloads as W
from oracle import solver as O
from oracle_helpers import assemble_L

F0, T0, T_END = 2.5, 0.2, 0.4
LEVELS = (40, 80, 160)


@pytest.fixture(scope="module")
def forced_problem():
    N = 2
    mesh = W.kuhn_cube(1, 1.0)           # 6 elements, free top, absorbing sides
    P = O.Problem(mesh, N)
    rng = np.random.default_rng(31)
    cp = rng.uniform(1.5, 3.0, P.K)
    rho, lam, mu = (torch.as_tensor(a) for a in
                    W.lame_from_velocities(cp, cp / rng.uniform(1.5, 2.2, P.K),
                                           rng.uniform(1.0, 3.0, P.K)))
    P.set_source([0.37, 0.52, 0.44], F0, T0, 1.0,
                 moment=(1.0, 0.5, -0.7, 0.3, 0.2, -0.4))
    L = assemble_L(P, rho, lam, mu)
    # spatial part of the forcing: the source term at the wavelet's peak,
    # where the Ricker value is its amplitude 1
    b = O.source_term(P, T0, torch.float64).reshape(-1).numpy()
    assert O.ricker(T0, F0, T0) == 1.0
    ode = lambda t, y: L @ y + O.ricker(t, F0, T0) * b
    y0 = np.zeros(L.shape[0])
    fine = solve_ivp(ode, (0.0, T_END), y0, method="DOP853", rtol=1e-13,
                     atol=1e-15).y[:, -1]
    coarse = solve_ivp(ode, (0.0, T_END), y0, method="DOP853", rtol=1e-11,
                       atol=1e-13).y[:, -1]
    # the reference's own error is far below the smallest error measured
    assert np.linalg.norm(fine - coarse) <= 1e-11 * np.linalg.norm(fine)
    return P, rho, lam, mu, fine


def _errors(P, rho, lam, mu, ref):
    errs = []
    for n in LEVELS:
        q0 = torch.zeros(P.K, 9, P.Np, dtype=torch.float64)
        q, _ = O.run(P, q0, rho, lam, mu, T_END / n, n)
        errs.append(np.linalg.norm(q.reshape(-1).numpy() - ref) / np.linalg.norm(ref))
    return errs, [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def test_forced_run_converges_at_fourth_order(forced_problem):
    P, rho, lam, mu, ref = forced_problem
    errs, rates = _errors(P, rho, lam, mu, ref)
    assert min(rates) >= 3.7, (errs, rates)
    assert errs[-1] < 1e-7, errs


@pytest.mark.parametrize("planted", ["t_n", "B_i"])
def test_wrong_stage_times_are_caught(forced_problem, monkeypatch, planted):
    """A planted mistake in the oracle's stage times drops the order."""
    P, rho, lam, mu, ref = forced_problem
    wrong = [0.0] * 5 if planted == "t_n" else list(O.LSERK_B)
    monkeypatch.setattr(O, "LSERK_C", wrong)
    errs, rates = _errors(P, rho, lam, mu, ref)
    assert max(rates) < 2.0, (errs, rates)
