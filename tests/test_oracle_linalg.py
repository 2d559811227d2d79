"""Pins of the oracle's Gramian and direct solves (CPU only)."""
import numpy as np

import workloads as wl
from oracle import linalg, mlp


def _jac(seed=0, widths=(2, 8, 8, 1), n_int=20, n_bdry=8):
    prob = wl.small_problem(widths=widths, n_interior=n_int, n_boundary=n_bdry, seed=seed)
    theta = wl.glorot_theta(prob.widths, seed)
    r, J = mlp.residual_and_jacobian(theta, prob)
    return r, J


def test_gramian_symmetric_psd_low_rank():
    """G = J^T W J is symmetric, PSD and of rank at most min(N, P) (eq. G_matrixfree; here N < P)."""
    r, J = _jac()
    G = linalg.gramian(J)
    assert np.max(np.abs(G - G.T)) <= 1e-14 * np.max(np.abs(G))
    ev = np.linalg.eigvalsh(G)
    assert ev.min() >= -1e-13 * ev.max()
    assert np.linalg.matrix_rank(G) <= min(J.shape)
    v = np.random.default_rng(0).standard_normal(J.shape[1])
    np.testing.assert_allclose(G @ v, J.T @ (J @ v), rtol=1e-12, atol=1e-14 * np.abs(G).max())


def test_direct_solves_agree():
    """Alg. 2 (Cholesky of G + lambda I) = SVD closed form = push-through form."""
    r, J = _jac(seed=1)
    lam = 1e-3
    G = linalg.gramian(J)
    g = J.T @ r
    d1 = linalg.solve_cholesky(G, g, lam)
    d2 = linalg.solve_svd(J, r, lam)
    d3 = linalg.solve_pushthrough(J, r, lam)
    kappa = (np.linalg.eigvalsh(G).max() + lam) / lam
    tol = 1e-15 * kappa * 10
    np.testing.assert_allclose(d1, d2, rtol=0, atol=tol * np.linalg.norm(d2))
    np.testing.assert_allclose(d3, d2, rtol=0, atol=tol * np.linalg.norm(d2))
    assert linalg.true_relative_residual(G, lam, g, d2) < 1e-10


def test_error_bound_from_residual():
    """With N < P the smallest eigenvalue of G + lambda I is lambda, so ||d - d*|| <= ||res|| / lambda."""
    r, J = _jac(seed=2)
    lam = 1e-2
    G = linalg.gramian(J)
    g = J.T @ r
    dstar = linalg.solve_svd(J, r, lam)
    ev = np.linalg.eigvalsh(G + lam * np.eye(G.shape[0]))
    assert abs(ev.min() - lam) <= 1e-10 * ev.max()
    d = dstar + 1e-3 * np.random.default_rng(0).standard_normal(dstar.size)
    res = g - G @ d - lam * d
    assert np.linalg.norm(d - dstar) <= np.linalg.norm(res) / lam * (1 + 1e-8)
