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


U32 = 2.0 ** -24


def jt_mul(J32, V, chunk=2048):
    """FP64 J^T (J V) with J a host copy of an FP32 Jacobian, in row chunks (V a vector or a block)."""
    out = np.zeros((J32.shape[1],) + np.shape(V)[1:])
    for s in range(0, J32.shape[0], chunk):
        Jc = J32[s:s + chunk].astype(np.float64)
        out += Jc.T @ (Jc @ V)
    return out


def check_fp32_solve(J32, g, d, mu, rtol):
    """True residual of a solve on an FP32 Jacobian promoted to FP64, against the PCG tolerance plus the
    rounding bound of the FP32 operator the solver applies (a sqrt(P) u dot-product bound)."""
    absd = np.zeros(J32.shape[1])
    for s in range(0, J32.shape[0], 2048):
        Jc = np.abs(J32[s:s + 2048].astype(np.float64))
        absd += Jc.T @ (Jc @ np.abs(d))
    res = np.linalg.norm(g - jt_mul(J32, d) - mu * d) / np.linalg.norm(g)
    bound = 10 * rtol + np.sqrt(J32.shape[1]) * U32 * np.linalg.norm(absd) / np.linalg.norm(g)
    assert res <= bound, (res, bound)
    return res
