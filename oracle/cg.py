"""Preconditioned conjugate gradients, the `pCG` of Alg. 3 (FP64).

Test infrastructure (see the package docstring); imports nothing from the GPU path.

The paper names pCG without printing it; this is the textbook recurrence with x_0 = 0. It stops when
the 2-norm of the recursively updated residual is at most rtol * ||b||, or after maxit iterations.
With M_fun = None it is plain CG.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class CGResult:
    x: np.ndarray
    iters: int
    rel_res: float          # recursive residual / ||b||
    converged: bool
    breakdown: bool
    history: list


def pcg(A_fun, b: np.ndarray, rtol: float, maxit: int, M_fun=None) -> CGResult:
    M = (lambda v: v) if M_fun is None else M_fun
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b)
    r = b.copy()
    hist = [1.0]
    if bnorm == 0.0:
        return CGResult(x, 0, 0.0, True, False, hist)
    z = M(r)
    p = z.copy()
    rz = float(r @ z)
    k = 0
    while k < maxit:
        q = A_fun(p)
        pq = float(p @ q)
        if not pq > 0.0:
            return CGResult(x, k, hist[-1], False, True, hist)
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        k += 1
        rel = float(np.linalg.norm(r)) / bnorm
        hist.append(rel)
        if rel <= rtol:
            return CGResult(x, k, rel, True, False, hist)
        z = M(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return CGResult(x, k, hist[-1], hist[-1] <= rtol, False, hist)
