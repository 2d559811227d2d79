"""Pins of the oracle's damping rule, power method, Armijo search and NGD step (CPU only)."""
import dataclasses

import numpy as np

import workloads as wl
from oracle import linalg, mlp, ngd


def test_damping_rule():
    assert ngd.damping(2.0, 0.5, 2.0 ** -23) == max(10 * 2.0 ** -23 * 2.0, 1e-4 * 0.25)
    assert ngd.damping(1e6, 1e-6, 2.0 ** -52) == 10 * 2.0 ** -52 * 1e6


def test_power_method_bounds():
    """Rayleigh quotients of a PSD matrix lie below the top eigenvalue and approach it."""
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((50, 50)))
    ev = np.logspace(-6, 2, 50)
    A = Q @ np.diag(ev) @ Q.T
    v0 = rng.standard_normal(50)
    l4 = ngd.power_method(lambda v: A @ v, v0, 4)
    l40 = ngd.power_method(lambda v: A @ v, v0, 40)
    assert l4 <= ev.max() * (1 + 1e-12) and l40 <= ev.max() * (1 + 1e-12)
    assert l40 >= l4 * (1 - 1e-12) and l40 > 0.99 * ev.max()


def test_armijo_sufficient_decrease():
    f = lambda x: float(x @ x)
    x = np.array([3.0, -1.0])
    g = 2 * x
    alpha, Lt = ngd.armijo(f, x, 4 * x, g, f(x))     # full step overshoots to -3x
    assert 0 < alpha < 1 and Lt <= f(x) - 1e-4 * alpha * (g @ (4 * x))
    assert ngd.armijo(f, x, -x, g, f(x)) == (0.0, f(x))   # ascent direction: rejected


def _teacher(seed=0):
    prob = wl.small_problem(widths=(2, 6, 6, 1), n_interior=40, n_boundary=12, seed=seed, lam=1e-9)
    theta_star = wl.glorot_theta(prob.widths, seed + 100)
    u, _, lap, _, _ = mlp.taylor_forward(theta_star, prob.widths, prob.X, prob.pde)
    inner = prob.kind == wl.KIND_INTERIOR
    prob = dataclasses.replace(prob, f=np.where(inner, -lap, 0.0), g=np.where(inner, 0.0, u))
    return prob, theta_star


def test_gauss_newton_from_perturbed_teacher():
    """Zero-residual problem: the damped Gauss-Newton (NGD) step from theta* + delta reduces the loss
    by orders of magnitude (fast local convergence), and the loss at theta* is exactly zero."""
    prob, theta_star = _teacher()
    assert mlp.loss(theta_star, prob) < 1e-28
    theta = theta_star + 1e-3 * np.random.default_rng(1).standard_normal(theta_star.size)
    L0 = mlp.loss(theta, prob)
    r, J = mlp.residual_and_jacobian(theta, prob)
    d = linalg.solve_svd(J, r, prob.lam)
    L1 = mlp.loss(theta - d, prob)
    assert L1 < 1e-3 * L0


def test_nystrom_and_plain_cg_steps_agree():
    """Both solvers target (G + mu I) d = g, so the directions agree to the solve tolerance."""
    prob = wl.small_problem(widths=(2, 8, 8, 1), n_interior=30, n_boundary=10, seed=2, lam=1e-4)
    theta = wl.glorot_theta(prob.widths, 2)
    P = theta.size
    Om = wl.gaussian_omega(P, 20, seed=3)
    th1, i1 = ngd.ngd_step(theta, prob, solver="nystrom", Omega=Om, rtol=1e-10)
    th2, i2 = ngd.ngd_step(theta, prob, solver="cg", power_v0=np.ones(P), rtol=1e-10, maxit=5 * P)
    assert i1.cg.converged and i2.cg.converged and i1.cg.iters < i2.cg.iters
    r, J = mlp.residual_and_jacobian(theta, prob)
    dstar = linalg.solve_svd(J, r, prob.lam)
    for info in (i1, i2):
        assert np.linalg.norm(info.direction - dstar) <= 1e-6 * np.linalg.norm(dstar)
        assert info.loss_new <= info.loss


def test_gain_ratio_is_one_for_a_linear_residual():
    """For a linear residual r(theta) = A theta - b the Gauss-Newton model of the loss is exact, so any
    step has gain ratio 1 and the Levenberg-Marquardt rule halves mu (Section 5.1.3)."""
    rng = np.random.default_rng(3)
    A, b, th = rng.standard_normal((9, 4)), rng.standard_normal(9), rng.standard_normal(4)
    L = lambda t: 0.5 * float(np.sum((A @ t - b) ** 2))
    g = A.T @ (A @ th - b)
    G = A.T @ A
    d = np.linalg.solve(G + 0.3 * np.eye(4), g)
    for alpha in (1.0, 0.5, 0.125):
        rho = ngd.gain_ratio(L(th), L(th - alpha * d), alpha, g @ d, d @ G @ d)
        assert abs(rho - 1.0) < 1e-12
        assert ngd.lm_update(0.3, rho) == 0.15


def test_gain_ratio_of_a_poor_step_and_no_step():
    """Hand-worked cases: a step of alpha = 1/2 along d with g^T d = d^T G d = 1 predicts a decrease of
    1/2 - 1/8 = 3/8; an actual decrease of 0.05 gives rho = 2/15 (mu grows 4x), one of 0.3 gives 4/5
    (mu halves), one of 0.15 gives 2/5 (kept); alpha = 0 counts as a poor step; the floor holds."""
    assert abs(ngd.gain_ratio(1.0, 0.95, 0.5, 1.0, 1.0) - 2.0 / 15.0) < 1e-15
    assert ngd.lm_update(1.0, ngd.gain_ratio(1.0, 0.95, 0.5, 1.0, 1.0)) == 4.0
    assert ngd.lm_update(1.0, ngd.gain_ratio(1.0, 0.7, 0.5, 1.0, 1.0)) == 0.5
    assert ngd.lm_update(1.0, ngd.gain_ratio(1.0, 0.85, 0.5, 1.0, 1.0)) == 1.0
    assert ngd.gain_ratio(1.0, 1.0, 0.0, 1.0, 1.0) == -1.0
    assert ngd.gain_ratio(1.0, 0.9, 1.0, 1.0, 4.0) == -1.0  # the model predicts an increase
    assert ngd.lm_update(1.0, -1.0) == 4.0
    assert ngd.lm_update(1e-9, 0.9, floor=1e-8) == 1e-8
