"""Pins of the oracle's randomized Nystrom approximation and preconditioner (CPU only)."""
import numpy as np

import workloads as wl
from oracle import cg, linalg, mlp, nystrom


def _problem(n_int, n_bdry, widths=(2, 10, 10, 1), seed=0):
    prob = wl.small_problem(widths=widths, n_interior=n_int, n_boundary=n_bdry, seed=seed)
    theta = wl.glorot_theta(prob.widths, seed)
    r, J = mlp.residual_and_jacobian(theta, prob)
    return r, J, linalg.gramian(J)


def test_exact_when_rank_at_most_ell():
    """rank(G) <= N < ell: the Nystrom approximation reproduces G and its nonzero eigenvalues."""
    r, J, G = _problem(8, 4)          # N = 12 rows, P = 151
    ell = 20
    Om = wl.gaussian_omega(G.shape[0], ell, seed=1)
    U, lam, nu = nystrom.nystrom_alg6(lambda V: G @ V, Om)
    Gn = U @ np.diag(lam) @ U.T
    assert np.linalg.norm(Gn - G) <= 1e-10 * np.linalg.norm(G)
    ev = np.sort(np.linalg.eigvalsh(G))[::-1][:12]
    np.testing.assert_allclose(lam[:12], ev, rtol=0, atol=1e-10 * ev[0])
    assert np.all(lam[12:] <= 1e-10 * ev[0])


def test_bounds_and_invariance():
    """0 <= G_nys <= G, lam_hat >= 0, G_nys invariant under Omega -> Omega R, Alg. 6 = definition."""
    r, J, G = _problem(30, 10)        # N = 40 > ell
    ell = 15
    Om = wl.gaussian_omega(G.shape[0], ell, seed=2)
    U, lam, _ = nystrom.nystrom_alg6(lambda V: G @ V, Om)
    Gn = U @ np.diag(lam) @ U.T
    assert np.all(lam >= 0) and np.all(np.diff(lam) <= 0)
    scale = np.linalg.eigvalsh(G).max()
    assert np.linalg.eigvalsh(Gn).min() >= -1e-12 * scale
    assert np.linalg.eigvalsh(G - Gn).min() >= -1e-12 * scale
    R = np.random.default_rng(3).standard_normal((ell, ell)) + 3 * np.eye(ell)
    U2, lam2, _ = nystrom.nystrom_alg6(lambda V: G @ V, Om @ R)
    assert np.linalg.norm(U2 @ np.diag(lam2) @ U2.T - Gn) <= 1e-8 * np.linalg.norm(Gn)
    Gd = nystrom.nystrom_definition(G, Om)
    assert np.linalg.norm(Gd - Gn) <= 1e-8 * np.linalg.norm(Gn)
    # orthonormal eigenvectors
    np.testing.assert_allclose(U.T @ U, np.eye(ell), atol=1e-10)


def test_structured_sketch_equals_alg6():
    """Because G = J^T J, (G Omega)(Omega^T G Omega)^+(G Omega)^T = J^T P_Z J with Z = J Omega."""
    r, J, G = _problem(30, 10, seed=4)
    ell = 12
    Om = wl.gaussian_omega(G.shape[0], ell, seed=5)
    U, lam, _ = nystrom.nystrom_alg6(lambda V: J.T @ (J @ V), Om)
    Z = J @ Om
    Q, _ = np.linalg.qr(Z)
    Gs = J.T @ Q @ Q.T @ J
    assert np.linalg.norm(Gs - U @ np.diag(lam) @ U.T) <= 1e-9 * np.linalg.norm(Gs)


def test_preconditioner_spectrum():
    """eq. nystrom_inverse: P^{-1} u_i = u_i / (lam_i + mu); P^{-1} v = v / (lam_ell + mu) for v _|_ U."""
    rng = np.random.default_rng(6)
    P, ell, mu = 40, 6, 0.1
    U, _ = np.linalg.qr(rng.standard_normal((P, ell)))
    lam = np.sort(rng.uniform(1, 10, ell))[::-1]
    for i in range(ell):
        np.testing.assert_allclose(nystrom.precond_apply(U, lam, mu, U[:, i]), U[:, i] / (lam[i] + mu), atol=1e-14)
    v = rng.standard_normal(P)
    v -= U @ (U.T @ v)
    np.testing.assert_allclose(nystrom.precond_apply(U, lam, mu, v), v / (lam[-1] + mu), atol=1e-13)
    Pm = nystrom.precond_matrix(U, lam, mu)
    assert np.allclose(Pm, Pm.T) and np.linalg.eigvalsh(Pm).min() > 0


def test_exact_nystrom_pcg_converges_in_two_steps():
    """With an exact Nystrom factorisation the preconditioned operator has the eigenvalues 1 and
    mu / (lam_ell + mu), so PCG terminates in at most two iterations (one if lam_ell = 0)."""
    r, J, G = _problem(8, 4, seed=7)
    g = J.T @ r
    mu = 1e-4
    for ell, max_it in [(20, 1), (12, 2)]:
        Om = wl.gaussian_omega(G.shape[0], ell, seed=8)
        U, lam, _ = nystrom.nystrom_alg6(lambda V: G @ V, Om)
        res = cg.pcg(lambda v: G @ v + mu * v, g, 1e-8, 50, lambda v: nystrom.precond_apply(U, lam, mu, v))
        assert res.converged and res.iters <= max_it
