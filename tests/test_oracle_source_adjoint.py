"""Pins of the oracle's source, receivers and discrete adjoint gradient.

* Ricker wavelet: peak value, zero crossings and minima of the closed form;
* the projected point source reproduces point evaluation: for every
  polynomial p of degree <= N, p^T (J M) w = p(x_s) (so it integrates to 1);
* receivers interpolate polynomial fields exactly at the receiver point;
* the reverse-mode gradient equals the complex-step derivative
  Im J(m + i h e_k) / h (h = 1e-30, no subtractive cancellation) for every
  parameter of a small mesh, equals central finite differences, and does not
  depend on the checkpoint interval;
* dot-product test: the reverse-mode transpose of the right-hand side (the
  map the adjoint is built from) satisfies <a, L b> = <L^T a, b> for random
  a, b, with L b from the forward right-hand side and L^T a from one
  vector-Jacobian product, and L^T a equals the transpose of the assembled
  matrix applied to a.
"""

import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint, solver
from oracle_helpers import assemble_L, random_medium, tensors


def test_ricker_closed_form():
    f0, t0 = 1.3, 0.9
    assert solver.ricker(t0, f0, t0, 2.5) == 2.5
    for sgn in (-1, 1):
        tz = t0 + sgn / (math.sqrt(2) * math.pi * f0)
        assert abs(solver.ricker(tz, f0, t0)) < 1e-15
        tm = t0 + sgn * math.sqrt(1.5) / (math.pi * f0)
        assert abs(solver.ricker(tm, f0, t0) + 2 * math.exp(-1.5)) < 1e-15


def _monos(N):
    return [(a, b, c) for a in range(N + 1) for b in range(N + 1)
            for c in range(N + 1) if a + b + c <= N]


@pytest.mark.parametrize("N", [2, 4])
def test_point_source_reproduces_point_values(N):
    mesh = W.kuhn_cube(2, 2.0)
    P = solver.Problem(mesh, N)
    xs = np.array([0.71, 1.23, 0.37])
    P.set_source(xs, 1.0, 1.0)
    k = P.source["k"]
    w = P.source["vec"].numpy()
    JM = P.geo["J"][k] * P.ops["M"]
    x = W.lattice_node_coords(mesh, N)[k]
    for e in _monos(N):
        p = x[:, 0] ** e[0] * x[:, 1] ** e[1] * x[:, 2] ** e[2]
        exact = xs[0] ** e[0] * xs[1] ** e[1] * xs[2] ** e[2]
        assert abs(p @ JM @ w - exact) < 1e-12 * max(1.0, abs(exact))


def test_receivers_interpolate_polynomials():
    N = 3
    mesh = W.kuhn_cube(2, 1.0)
    P = solver.Problem(mesh, N)
    rec = np.array([[0.2, 0.3, 1.0], [0.61, 0.45, 0.5], [0.9, 0.1, 0.05]])
    P.set_receivers(rec)
    x = W.lattice_node_coords(mesh, N)
    f = lambda y: np.stack([y[..., 0] ** 3 - y[..., 1], y[..., 1] * y[..., 2],
                            np.ones(y.shape[:-1]) * 2.0], axis=-1)
    q = np.zeros((P.K, 9, P.Np))
    q[:, 0:3, :] = f(x).transpose(0, 2, 1)
    got = solver.sample_receivers(P, torch.as_tensor(q)).numpy()
    assert np.max(np.abs(got - f(rec))) < 1e-13


def _tiny_problem(N=2, nsteps=20):
    mesh = W.kuhn_cube(1, 1.0)
    P = solver.Problem(mesh, N)
    med = random_medium(P.K, 13)
    P.set_source([0.3, 0.4, 0.5], 5.0, 0.2)
    P.set_receivers([[0.2, 0.2, 1.0], [0.7, 0.5, 1.0], [0.5, 0.5, 0.0]])
    dt = P.suggest_dt(*med, 0.5)
    q0 = torch.zeros(P.K, 9, P.Np, dtype=torch.float64)
    rho, lam, mu = tensors(*med)
    _, tr = solver.run(P, q0, rho, lam, mu, dt, nsteps, record=True)
    d_obs = 0.6 * tr + 1e-4 * torch.sin(torch.arange(tr.numel(),
                                                      dtype=torch.float64)).view_as(tr)
    return P, (rho, lam, mu), q0, dt, nsteps, d_obs


def _misfit(P, params, q0, dt, nsteps, d_obs):
    _, tr = solver.run(P, q0, *params, dt, nsteps, record=True)
    return solver.misfit(tr, d_obs.to(tr.dtype), dt)


def test_gradient_equals_complex_step():
    P, params, q0, dt, nsteps, d_obs = _tiny_problem()
    J, gr, gl, gm = adjoint.misfit_gradient(P, *params, q0, dt, nsteps, d_obs,
                                            ckpt_every=7)
    grads = (gr, gl, gm)
    h = 1e-30
    for i in range(3):
        for k in range(P.K):
            pc = [p.to(torch.complex128) for p in params]
            pc[i] = pc[i].clone()
            pc[i][k] += 1j * h
            Jc = _misfit(P, pc, q0.to(torch.complex128), dt, nsteps, d_obs)
            cs = Jc.imag.item() / h
            assert abs(cs - grads[i][k].item()) <= 1e-12 * abs(cs) + 1e-30
    assert abs(J.item() - _misfit(P, params, q0, dt, nsteps, d_obs).item()) \
        < 1e-15 * J.item()


def test_gradient_matches_central_differences_and_checkpointing():
    P, params, q0, dt, nsteps, d_obs = _tiny_problem(N=1, nsteps=15)
    _, g1r, g1l, g1m = adjoint.misfit_gradient(P, *params, q0, dt, nsteps,
                                               d_obs, ckpt_every=4)
    _, g2r, g2l, g2m = adjoint.misfit_gradient(P, *params, q0, dt, nsteps,
                                               d_obs, ckpt_every=100)
    for a, b in ((g1r, g2r), (g1l, g2l), (g1m, g2m)):
        assert torch.max(torch.abs(a - b)) <= 1e-13 * torch.max(torch.abs(b))
    for i, g in enumerate((g1r, g1l, g1m)):
        k = int(torch.argmax(torch.abs(g)))
        delta = 1e-6 * params[i][k].item()
        vals = []
        for sgn in (1, -1):
            p = [x.clone() for x in params]
            p[i][k] += sgn * delta
            vals.append(_misfit(P, p, q0, dt, nsteps, d_obs).item())
        fd = (vals[0] - vals[1]) / (2 * delta)
        assert abs(fd - g[k].item()) < 1e-6 * abs(fd)


def test_dot_product_transpose_of_rhs():
    for periodic, n, N in ((True, 3, 2), (False, 2, 1), (False, 1, 3)):
        mesh = W.kuhn_cube(n, 1.0, periodic=periodic)
        P = solver.Problem(mesh, N)
        rho, lam, mu = tensors(*random_medium(P.K, 13 + N))
        rng = np.random.default_rng(21 + N)
        a = torch.as_tensor(rng.standard_normal((P.K, 9, P.Np)))
        b = torch.as_tensor(rng.standard_normal((P.K, 9, P.Np)))
        Lb = solver.rhs(P, b, rho, lam, mu)
        x = torch.zeros_like(b).requires_grad_(True)
        (LTa,) = torch.autograd.grad(solver.rhs(P, x, rho, lam, mu), x,
                                     grad_outputs=a)
        lhs, rhs_ = torch.sum(a * Lb).item(), torch.sum(LTa * b).item()
        scale = torch.linalg.norm(a).item() * torch.linalg.norm(Lb).item()
        assert abs(lhs - rhs_) <= 1e-13 * scale
        if periodic:
            continue                      # assembled L too large here
        L = assemble_L(P, rho, lam, mu)
        want = L.T @ a.reshape(-1).numpy()
        assert np.abs(LTa.reshape(-1).numpy() - want).max() \
            <= 1e-13 * np.abs(want).max()
