"""Randomized Nystrom approximation and preconditioner (FP64).

Test infrastructure (see the package docstring); imports nothing from the GPU path.

* `nystrom_alg6` follows Alg. 6 (the stable randomized Nystrom of the appendix) step by step.
  MATLAB notation is read as: qr(., 0) = thin QR; eps(x) = spacing of doubles at x; chol = upper
  factor C with C^T C = M; Y / C = right triangular solve; svd(., 0) = thin SVD, singular values
  descending. The core matrix is symmetrised before chol (finite precision).
* `nystrom_definition` is eq. nystrom_approx written out: (G Omega)(Omega^T G Omega)^+ (G Omega)^T.
* `precond_apply` is eq. nystrom_inverse.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def nystrom_alg6(G_fun, Omega: np.ndarray):
    """Alg. 6. Returns (U, lam_hat, nu): G_nys = U diag(lam_hat) U^T with lam_hat descending."""
    Omega, _ = np.linalg.qr(Omega, mode="reduced")             # thin QR
    Y = G_fun(Omega)                                             # ell matvecs with G
    nu = float(np.spacing(np.linalg.norm(Y, "fro")))             # shift
    Y_nu = Y + nu * Omega
    M = Omega.T @ Y_nu
    M = 0.5 * (M + M.T)
    C = sla.cholesky(M, lower=False)                             # C^T C = Omega^T Y_nu
    B = sla.solve_triangular(C, Y_nu.T, trans="T", lower=False).T  # B = Y_nu C^{-1}
    U, S, _ = np.linalg.svd(B, full_matrices=False)
    lam_hat = np.maximum(0.0, S * S - nu)                        # remove shift
    return U, lam_hat, nu


def nystrom_definition(G: np.ndarray, Omega: np.ndarray) -> np.ndarray:
    """eq. nystrom_approx: (G Omega)(Omega^T G Omega)^+ (G Omega)^T with an SVD pseudo-inverse."""
    Y = G @ Omega
    core = Omega.T @ Y
    core = 0.5 * (core + core.T)
    return Y @ np.linalg.pinv(core, rcond=1e-13, hermitian=True) @ Y.T


def nystrom_shifted(G: np.ndarray, Omega: np.ndarray, nu: float) -> np.ndarray:
    """The Nystrom approximation with its core shifted and the shift kept: (G Omega)(Omega^T G Omega +
    nu I)^{-1} (G Omega)^T. It tends to eq. nystrom_approx as nu -> 0 and lies below it in the PSD
    order; Alg. 6 shifts the core in the same way for stability and then subtracts nu from the
    eigenvalues."""
    Y = G @ Omega
    core = Omega.T @ Y
    core = 0.5 * (core + core.T) + nu * np.eye(core.shape[0])
    out = Y @ np.linalg.solve(core, Y.T)
    return 0.5 * (out + out.T)


def precond_apply(U: np.ndarray, lam_hat: np.ndarray, mu: float, V: np.ndarray) -> np.ndarray:
    """eq. nystrom_inverse: P^{-1} v = U (Lambda + mu I)^{-1} U^T v + (lam_ell + mu)^{-1} (v - U U^T v),
    with lam_ell the smallest of the ell Nystrom eigenvalues."""
    Ut_v = U.T @ V
    lam_ell = float(lam_hat[-1])
    scale = 1.0 / (lam_hat + mu)
    if V.ndim == 1:
        return U @ (scale * Ut_v) + (V - U @ Ut_v) / (lam_ell + mu)
    return U @ (scale[:, None] * Ut_v) + (V - U @ Ut_v) / (lam_ell + mu)


def precond_matrix(U, lam_hat, mu) -> np.ndarray:
    """The preconditioner inverse of eq. nystrom_inverse as an explicit P x P matrix."""
    return precond_apply(U, lam_hat, mu, np.eye(U.shape[0]))
