"""Pins of the oracle's adaptive sketch-size rule (Alg. 4), its accuracy measure (relative L2 / H1
errors, Section 5) and the paper's 3D Poisson workload (CPU only)."""

import numpy as np
import pytest

import workloads as wl
from oracle import mlp, ngd


# ---- Alg. 4: the next sketch size ----

def test_next_rank_grows_while_smallest_estimate_exceeds_ten_mu():
    # lam_hat_3 = 2 > 10 mu = 1: grow by dell, capped at ell_max
    assert ngd.next_rank([10.0, 5.0, 2.0], 0.1, 3, 500, 20) == 23
    assert ngd.next_rank([10.0, 5.0, 2.0], 0.1, 3, 10, 20) == 10


def test_next_rank_shrinks_to_first_index_below_threshold_plus_offset():
    # 1-based first index with lam_hat_i < 1 is 3; plus the offset 1
    assert ngd.next_rank([10.0, 5.0, 0.5, 0.1], 0.1, 4, 500, 20) == 4
    assert ngd.next_rank([10.0, 5.0, 0.5, 0.1, 0.0, 0.0], 0.1, 6, 500, 20) == 4
    assert ngd.next_rank([0.5, 0.1, 0.0], 0.1, 3, 500, 20) == 2
    assert ngd.next_rank([10.0, 5.0, 0.5, 0.1], 0.1, 4, 500, 20, offset=2) == 5
    # the shrunk rank never exceeds ell_max
    assert ngd.next_rank([10.0, 5.0, 2.0, 0.5], 0.1, 4, 4, 20) == 4


def test_next_rank_boundary_of_the_threshold():
    # lam_hat_ell equal to 10 mu does not grow the rank, and no estimate lies strictly below: keep ell
    assert ngd.next_rank([5.0, 1.0], 0.1, 2, 500, 20) == 2
    # just above the threshold grows it
    assert ngd.next_rank([5.0, 1.0 + 1e-12], 0.1, 2, 500, 20) == 22


# ---- accuracy measure: relative L2 and H1 errors ----

def _glorot(widths, seed):
    return wl.glorot_theta(widths, seed) + 0.1 * np.random.default_rng(seed).standard_normal(wl.num_params(widths))


def test_solution_error_sums_linear_network_closed_form():
    """widths (d, 1): u = w . x + b exactly, grad u = w."""
    rng = np.random.default_rng(1)
    d, n = 3, 50
    w, b = rng.standard_normal(d), 0.7
    theta = np.concatenate([w, [b]])
    X = rng.uniform(0, 1, (n, d))
    u_ref, g_ref = rng.standard_normal(n), rng.standard_normal((n, d))
    s = mlp.solution_error_sums(theta, (d, 1), X, u_ref, g_ref)
    u = X @ w + b
    want = [np.sum((u - u_ref) ** 2), np.sum((w[None, :] - g_ref) ** 2), np.sum(u_ref ** 2), np.sum(g_ref ** 2)]
    np.testing.assert_allclose(s, want, rtol=1e-13)


def test_solution_error_sums_constant_network():
    """All weights zero: u is the output bias everywhere and its gradient vanishes."""
    widths = (2, 5, 4, 1)
    theta = np.zeros(wl.num_params(widths))
    theta[-1] = -1.25
    rng = np.random.default_rng(2)
    X = rng.uniform(0, 1, (20, 2))
    u_ref, g_ref = rng.standard_normal(20), rng.standard_normal((20, 2))
    s = mlp.solution_error_sums(theta, widths, X, u_ref, g_ref)
    np.testing.assert_allclose(s, [np.sum((-1.25 - u_ref) ** 2), np.sum(g_ref ** 2), np.sum(u_ref ** 2),
                                   np.sum(g_ref ** 2)], rtol=1e-14)


def test_solution_error_gradient_matches_finite_differences():
    """The gradient term uses grad_x u; compare with central differences of u (error O(h^2))."""
    widths = (3, 12, 9, 1)
    theta = _glorot(widths, 3)
    rng = np.random.default_rng(3)
    X = rng.uniform(0, 1, (15, 3))
    h = 1e-5
    fd = np.stack([(mlp.taylor_forward(theta, widths, X + h * e, wl.PDE_POISSON)[0]
                    - mlp.taylor_forward(theta, widths, X - h * e, wl.PDE_POISSON)[0]) / (2 * h)
                   for e in np.eye(3)], axis=1)
    zeros = np.zeros(15)
    s = mlp.solution_error_sums(theta, widths, X, zeros, np.zeros((15, 3)))
    assert abs(s[1] - np.sum(fd ** 2)) <= 1e-8 * np.sum(fd ** 2)
    # against the exact gradient itself the gradient term vanishes up to the FD error
    s2 = mlp.solution_error_sums(theta, widths, X, zeros, fd)
    assert s2[1] <= 1e-16 * np.sum(fd ** 2) + 1e-18


def test_relative_errors_and_empty_set():
    assert mlp.relative_errors([1.0, 3.0, 4.0, 12.0]) == (0.5, 0.5)
    np.testing.assert_array_equal(mlp.solution_error_sums(np.zeros(4), (2, 1), np.zeros((0, 2)), [], np.zeros((0, 2))),
                                  np.zeros(4))


# ---- the paper's 3D Poisson setup ----

def test_paper3d_workload_shape():
    p = wl.config("paper3d")
    assert p.widths == (3, 64, 64, 64, 1) and p.n_params == 8641  # the paper's p
    assert (p.kind == wl.KIND_INTERIOR).sum() == 10000 and (p.kind == wl.KIND_BOUNDARY).sum() == 1000
    assert p.dtype == "f64" and p.ell_max == 500 and p.dell == 20 and p.maxit == 20 and p.ell == 20
    X, u, g = wl.evaluation_set(p, 1000)
    assert X.shape == (1000, 3) and np.all((X >= 0) & (X <= 1))


@pytest.mark.parametrize("solution,d", [("sinprod", 3), ("sinsum", 5), ("heat", 3)])
def test_exact_solution_gradients(solution, d):
    X = np.random.default_rng(4).uniform(0, 1, (6, d))
    u, g = wl.exact_solution(solution, X)
    h = 1e-6
    fd = np.stack([(wl.exact_solution(solution, X + h * e)[0] - wl.exact_solution(solution, X - h * e)[0]) / (2 * h)
                   for e in np.eye(d)], axis=1)
    np.testing.assert_allclose(g, fd, atol=1e-8)


def test_exact_solution_special_points():
    u, g = wl.exact_solution("sinprod", np.full((1, 3), 0.5))
    assert abs(u[0] - 1.0) < 1e-15 and np.abs(g).max() < 1e-15
    u, g = wl.exact_solution("sinsum", np.zeros((1, 5)))
    assert u[0] == 0.0 and np.allclose(g, np.pi)


# ---- Gramian diagonal, pivot sampling, sampling test matrix ----

def test_gram_diagonal_is_diag_of_product():
    from oracle import sampling
    J = np.random.default_rng(5).standard_normal((30, 12))
    np.testing.assert_allclose(sampling.gram_diagonal(J), np.diag(J.T @ J), rtol=1e-14)


def test_sample_pivots_frequencies_follow_weights():
    """s ~ d: empirical frequencies within 5 standard deviations of d_j / sum d; zero and negative
    weights are never drawn."""
    from oracle import sampling
    w = np.array([0.0, 1.0, 0.0, 3.0, -1.0, 0.0, 6.0, 0.5])
    n = 200_000
    s = sampling.sample_pivots(w, n, seed=3, counter=1)
    p = np.maximum(w, 0) / np.maximum(w, 0).sum()
    freq = np.bincount(s, minlength=w.size) / n
    assert np.all(freq[p == 0] == 0)
    assert np.all(np.abs(freq - p) <= 5 * np.sqrt(p * (1 - p) / n) + 1e-12)


def test_sample_pivots_special_cases():
    from oracle import sampling
    w = np.zeros(9)
    assert sampling.sample_pivots(w, 5, 1, 0).size == 0
    w[4] = 2.5
    assert np.all(sampling.sample_pivots(w, 50, 1, 0) == 4)
    u = sampling.sample_uniforms(1000, 7, 2, 3)
    assert np.all((u > 0) & (u < 1))
    # substreams and counters give different draws
    assert not np.array_equal(u, sampling.sample_uniforms(1000, 7, 2, 4))
    assert not np.array_equal(u, sampling.sample_uniforms(1000, 7, 3, 3))
    s = sampling.sample_pivots(np.arange(1.0, 31.0), 40, 1, 0, unique=True)
    assert np.all(np.diff(s) > 0)


def test_column_test_matrix_nystrom_is_column_form():
    """With Omega = I[:, S] the Nystrom approximation is G[:, S] G[S, S]^+ G[S, :]; it is exact once the
    sampled columns span range(G)."""
    from oracle import nystrom, sampling
    rng = np.random.default_rng(6)
    B = rng.standard_normal((5, 14))
    G = B.T @ B  # rank 5
    S = np.array([0, 3, 7, 9])
    Om = sampling.column_test_matrix(14, S)
    Gn = nystrom.nystrom_definition(G, Om)
    np.testing.assert_allclose(Gn, G[:, S] @ np.linalg.pinv(G[np.ix_(S, S)]) @ G[S, :], atol=1e-10)
    S6 = np.array([0, 2, 3, 7, 9, 11])
    np.testing.assert_allclose(nystrom.nystrom_definition(G, sampling.column_test_matrix(14, S6)), G, atol=1e-9)
    # Alg. 6 with the column test matrix agrees with the definition
    U, lam, _ = nystrom.nystrom_alg6(lambda V: G @ V, Om)
    np.testing.assert_allclose(U @ np.diag(lam) @ U.T, Gn, atol=1e-9 * np.abs(G).max())


def test_shifted_nystrom_limits_and_order():
    """nu -> 0 recovers eq. nystrom_approx (well-conditioned core); a positive shift lowers the
    approximation in the PSD order, by at most nu-scaled terms."""
    from oracle import nystrom
    rng = np.random.default_rng(8)
    B = rng.standard_normal((9, 20))
    G = B.T @ B
    Om = rng.standard_normal((20, 6))
    G0 = nystrom.nystrom_definition(G, Om)
    np.testing.assert_allclose(nystrom.nystrom_shifted(G, Om, 0.0), G0, atol=1e-10)
    Gs = nystrom.nystrom_shifted(G, Om, 1e-3)
    ev = np.linalg.eigvalsh(G0 - Gs)
    assert ev.min() >= -1e-10 and ev.max() > 0
    assert np.linalg.norm(G0 - nystrom.nystrom_shifted(G, Om, 1e-9)) <= 1e-6 * np.linalg.norm(G0)


# ---- block RPCholesky and its preconditioner ----

def _psd(rank, p, seed):
    B = np.random.default_rng(seed).standard_normal((rank, p)) * np.logspace(0, -3, rank)[:, None]
    return B.T @ B


def test_rpcholesky_exact_for_low_rank_and_trace_identity():
    from oracle import sampling
    G = _psd(7, 30, 1)
    F, piv, tr = sampling.block_rpcholesky(lambda S: G[:, S], np.diag(G).copy(), 20, 4, seed=1, counter=0,
                                           eps=1e-12 * np.trace(G))
    assert F.shape[1] <= 20
    np.testing.assert_allclose(F @ F.T, G, atol=1e-9 * np.abs(G).max())
    assert abs(tr - np.trace(G - F @ F.T)) <= 1e-12 * np.trace(G)


def test_rpcholesky_interpolates_pivot_columns_and_stops_on_trace():
    from oracle import sampling
    G = _psd(25, 40, 2)
    eps = 0.05 * np.trace(G)
    F, piv, tr = sampling.block_rpcholesky(lambda S: G[:, S], np.diag(G).copy(), 24, 5, seed=3, counter=2, eps=eps)
    # partial Cholesky reproduces the selected columns exactly and leaves a PSD residual
    np.testing.assert_allclose((F @ F.T)[:, piv], G[:, piv], atol=1e-10 * np.abs(G).max())
    assert np.linalg.eigvalsh(G - F @ F.T).min() >= -1e-10 * np.abs(G).max()
    assert abs(tr - np.trace(G - F @ F.T)) <= 1e-10 * np.trace(G)
    # it stopped at the first round whose residual trace fell below eps (or ran out of room)
    assert tr < eps or F.shape[1] + 1 > 24


def test_rpchol_preconditioner_is_the_inverse_of_FFt_plus_mu():
    from oracle import sampling
    rng = np.random.default_rng(4)
    F = rng.standard_normal((25, 6))
    mu = 0.3
    V = rng.standard_normal((25, 3))
    want = np.linalg.solve(F @ F.T + mu * np.eye(25), V)
    np.testing.assert_allclose(sampling.rpchol_precond_apply(F, mu, V), want, rtol=1e-12, atol=1e-12)
    # the SVD form of the same inverse
    U, s, _ = np.linalg.svd(F, full_matrices=False)
    svd_form = U @ ((U.T @ V) / (s[:, None] ** 2 + mu)) + (V - U @ (U.T @ V)) / mu
    np.testing.assert_allclose(svd_form, want, rtol=1e-12, atol=1e-12)


def test_paper_heat_workload_and_source():
    """The heat 3+1D setup: shapes, and f = u_t - Laplace u of the exact solution (central differences)."""
    p = wl.config("paper_heat")
    assert p.widths == (4, 64, 64, 64, 1) and p.n_params == 8705 and p.pde == wl.PDE_HEAT
    n_i = int((p.kind == wl.KIND_INTERIOR).sum())
    assert n_i == 10000 and p.n_rows == 11000 and (p.kind == wl.KIND_INITIAL).sum() == 143
    assert np.all(p.X[p.kind == wl.KIND_INITIAL, 3] == 0)
    lat = p.X[p.kind == wl.KIND_BOUNDARY, :3]
    assert np.all(np.any((lat == 0) | (lat == 1), axis=1))
    X = p.X[:20][p.kind[:20] == wl.KIND_INTERIOR]
    h = 1e-4
    u = lambda Y: wl.exact_solution("heatcos", Y)[0]
    E = np.eye(4)
    lap = sum((u(X + h * E[j]) - 2 * u(X) + u(X - h * E[j])) / h ** 2 for j in range(3))
    ut = (u(X + h * E[3]) - u(X - h * E[3])) / (2 * h)
    np.testing.assert_allclose(p.f[:20][p.kind[:20] == wl.KIND_INTERIOR], ut - lap, rtol=1e-5, atol=1e-6)
    g0 = p.g[p.kind == wl.KIND_INITIAL]
    np.testing.assert_allclose(g0, u(p.X[p.kind == wl.KIND_INITIAL]), rtol=1e-14)
    # the oracle's residual at the exact solution's values: u - g vanishes on boundary rows by construction
    _, grad = wl.exact_solution("heatcos", X)
    fd = np.stack([(u(X + 1e-6 * e) - u(X - 1e-6 * e)) / 2e-6 for e in E], axis=1)
    np.testing.assert_allclose(grad, fd, atol=1e-7)
