"""Shared helpers of the GPU parity tests: build a problem on both sides from the same seeded data."""
import numpy as np

import workloads as wl


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rowwise_rel(A, B):
    """max over rows of ||A_r - B_r|| / ||B_r|| (rows with zero norm use the global scale)."""
    A, B = np.asarray(A, np.float64), np.asarray(B, np.float64)
    nb = np.linalg.norm(B, axis=1)
    scale = np.where(nb > 0, nb, np.linalg.norm(B) / np.sqrt(B.shape[0]))
    return float(np.max(np.linalg.norm(A - B, axis=1) / scale))


def rounded_theta(theta, dtype):
    return theta.astype(np.float32).astype(np.float64) if dtype == "f32" else theta


def make(prob, seed=0):
    """(oracle-side problem promoted from the working precision, theta64 rounded likewise)."""
    theta = wl.glorot_theta(prob.widths, seed)
    theta = theta + 0.05 * np.random.default_rng(seed + 1).standard_normal(theta.size)
    th = rounded_theta(theta, prob.dtype)
    return prob.cast(prob.dtype), th
