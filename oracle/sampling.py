"""Gramian diagonal, pivot sampling and column test matrices (FP64).

Test infrastructure (see the package docstring); imports nothing from the GPU path.

* diag(G) for G = J_w^T J_w (eq. gram_diagonal, the quadrature weights folded into J_w): the squared
  column norms of J_w.
* Sampling s ~ d (Section 4.2.2: P(s = j) = d_j / sum_k d_k), used by RPCholesky and by the sampling
  test matrix of the experiments (Section 5). Readings: negative entries (rounding in a downdated
  diagonal) weigh 0; sample k of substream q takes its uniform u from Philox4x32-10 at counter
  (k, 2^31 + q, counter_lo, counter_hi), key (seed_lo, seed_hi), as u = ((x0 >> 5) 2^26 + (x1 >> 6) +
  1/2) 2^-53; the index is the inverse of the cumulative distribution at u, i.e. the first j with
  d_0 + ... + d_j > u * sum(d).
* The sampling test matrix Omega = [e_{s_1}, ..., e_{s_ell}] (columns of the identity).
"""
from __future__ import annotations

import numpy as np

from .philox import _u53, philox4x32_10


def gram_diagonal(J: np.ndarray) -> np.ndarray:
    """diag(J^T J) as the sum over rows of the squared entries."""
    J = np.asarray(J, dtype=np.float64)
    return np.einsum("ij,ij->j", J, J)


def sample_uniforms(n: int, seed: int, counter: int, substream: int) -> np.ndarray:
    k = np.arange(n, dtype=np.uint64)
    x = philox4x32_10(k & np.uint64(0xFFFFFFFF), np.full(n, 0x80000000 | int(substream), dtype=np.uint64),
                      np.full(n, int(counter) & 0xFFFFFFFF, dtype=np.uint64),
                      np.full(n, (int(counter) >> 32) & 0xFFFFFFFF, dtype=np.uint64),
                      int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF)
    return _u53(x[0], x[1])


def sample_pivots(weights, n: int, seed: int, counter: int, substream: int = 0, unique: bool = False):
    """n indices drawn with probability proportional to max(weights, 0), by the inverse of the running sum.
    Returns the (sorted, distinct when `unique`) index array; empty when every weight is <= 0."""
    w = np.maximum(np.asarray(weights, dtype=np.float64), 0.0)
    cum = np.cumsum(w)
    total = cum[-1] if w.size else 0.0
    if n == 0 or not total > 0.0:
        return np.zeros(0, dtype=np.int64)
    u = sample_uniforms(n, seed, counter, substream)
    idx = np.searchsorted(cum, u * total, side="right").astype(np.int64)
    idx = np.minimum(idx, w.size - 1)
    return np.unique(idx) if unique else idx


def column_test_matrix(p: int, cols) -> np.ndarray:
    """Omega (p x len(cols)) whose columns are the identity's columns at `cols`."""
    cols = np.asarray(cols, dtype=np.int64)
    Om = np.zeros((p, cols.size))
    Om[cols, np.arange(cols.size)] = 1.0
    return Om


def block_rpcholesky(G_cols, d0, ell_max: int, block: int, seed: int, counter: int, eps: float):
    """Block RPCholesky (Section 4.2.2, the block algorithm of the appendix) on a PSD matrix given by
    column access G_cols(S) -> G[:, S] and its diagonal d0. Round i draws `block` pivots ~ d (substream
    i, sorted, repeats dropped), forms C = G[:, S'] - F F[S', :]^T, factors C[S', S'] = R^T R and
    appends C R^{-1} to F, downdates d by the squared rows and stops once sum(d) < eps or F is full.
    Reading: a pivot whose residual diagonal in the block's elimination is not above 1e-13 of the
    block's largest is dropped with its column (a direction F already holds).
    Returns (F (p x r), pivots kept, trace sum(d))."""
    d = np.array(d0, dtype=np.float64)
    p = d.size
    F = np.zeros((p, ell_max))
    r = 0
    kept_all = []
    rounds = -(-ell_max // block)
    done = False
    for i in range(rounds):
        if done:
            break
        S = sample_pivots(d, block, seed, counter, substream=i, unique=True)
        if S.size == 0:
            break
        C = G_cols(S) - F[:, :r] @ F[S, :r].T
        A = C[S, :].T.copy()  # the pivot block (symmetric up to rounding); lower part used
        dmax = max(float(np.max(np.diag(A))), 0.0)
        keep = []
        for j in range(S.size):  # right-looking elimination deciding which pivots stay
            pj = A[j, j]
            if not (pj > 1e-13 * dmax) or r + len(keep) >= ell_max:
                continue
            rj = np.sqrt(pj)
            A[j, j] = rj
            A[j + 1:, j] /= rj
            for m in range(j + 1, S.size):
                A[m, j + 1:m + 1] -= A[m, j] * A[j + 1:m + 1, j]
            keep.append(j)
        if keep:
            k = np.array(keep)
            Lk = A[np.ix_(k, k)]
            Lk = np.tril(Lk)
            Fn = np.linalg.solve(Lk, C[:, k].T).T  # C[:, k] R^{-1} with R = Lk^T
            F[:, r:r + k.size] = Fn
            d -= np.sum(Fn * Fn, axis=1)
            r += k.size
            kept_all.extend(S[k].tolist())
        tr = float(np.sum(d))
        if tr < eps or r + 1 > ell_max:
            done = True
    return F[:, :r], np.array(kept_all, dtype=np.int64), float(np.sum(d))


def rpchol_precond_apply(F: np.ndarray, mu: float, V: np.ndarray) -> np.ndarray:
    """eq. rpchol_precond: P^{-1} v = mu^{-1} (v - F R^{-1} R^{-T} F^T v) with R^T R = F^T F + mu I."""
    R = np.linalg.cholesky(F.T @ F + mu * np.eye(F.shape[1])).T
    W = np.linalg.solve(R, np.linalg.solve(R.T, F.T @ V))
    return (V - F @ W) / mu
