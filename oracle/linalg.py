"""Gramian, damped matvec and direct solves (FP64).

Test infrastructure (see the package docstring); imports nothing from the GPU path.

Theorem thm:matfree (eq. G_matrixfree): with quadrature weights folded into the rows of J_w,
G = J_w^T J_w. The damped operator of eq. regularized_ng is G + lambda I.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def gramian(J: np.ndarray) -> np.ndarray:
    """Explicit P x P Gramian G = J_w^T J_w (eq. G_matrixfree)."""
    return J.T @ J


def damped_matvec(G: np.ndarray, V: np.ndarray, lam: float) -> np.ndarray:
    """(G + lambda I) V by definition, from the explicit Gramian."""
    return G @ V + lam * V


def solve_cholesky(G: np.ndarray, g: np.ndarray, lam: float) -> np.ndarray:
    """Alg. 2: Cholesky G + lambda I = R^T R, then forward and backward substitution."""
    R = sla.cholesky(G + lam * np.eye(G.shape[0]), lower=False)
    y = sla.solve_triangular(R, g, trans="T", lower=False)
    return sla.solve_triangular(R, y, lower=False)


def solve_svd(J: np.ndarray, r: np.ndarray, lam: float) -> np.ndarray:
    """Closed form of (J^T J + lambda I)^{-1} J^T r through the thin SVD J = U S V^T:
    d = V diag(s / (s^2 + lambda)) U^T r."""
    U, s, Vt = np.linalg.svd(J, full_matrices=False)
    return Vt.T @ ((s / (s * s + lam)) * (U.T @ r))


def solve_pushthrough(J: np.ndarray, r: np.ndarray, lam: float) -> np.ndarray:
    """(J^T J + lambda I)^{-1} J^T r = J^T (J J^T + lambda I)^{-1} r: the N x N form that the paper
    recalls for few points (Section 4, remark on Woodbury when q << p)."""
    N = J.shape[0]
    c = sla.cho_factor(J @ J.T + lam * np.eye(N))
    return J.T @ sla.cho_solve(c, r)


def true_relative_residual(G: np.ndarray, lam: float, g: np.ndarray, d: np.ndarray) -> float:
    """||g - (G + lambda I) d|| / ||g||."""
    return float(np.linalg.norm(g - G @ d - lam * d) / np.linalg.norm(g))
