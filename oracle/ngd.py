"""One natural-gradient step: damping rule, power method, Armijo, Alg. 1 with Alg. 3 + Alg. 4 (FP64).

Test infrastructure (see the package docstring); imports nothing from the GPU path.

Readings of points the paper leaves open:
* damping (Section 4.3 and the general setup of Section 5): mu = max(gamma eps lam1_hat, 1e-4 L^2)
  with gamma = 10, L the loss value 1/2 sum w res^2 and eps the unit roundoff of the working precision
  (2^-52 for FP64 runs, 2^-23 for FP32 runs); a fixed mu is used when the workload prescribes one.
* Nystrom NGD takes lam1_hat from the Nystrom eigenvalues; plain CG from 4 power iterations
  (Rayleigh quotient of the last normalised iterate) started from a given vector.
* Armijo (Section 4.4): alpha_0 = 1, halve until L(theta - alpha d) <= L(theta) - c1 alpha g^T d,
  c1 = 1e-4, at most 30 halvings; alpha = 0 if none is accepted.
* adaptive sketch size (Alg. 4, Section 4.3, experimental setup of Section 5): the next rank from
  lam_hat_ell / mu against 10, growing by dell = 20 up to ell_max = 500, shrinking to the first index
  below the threshold plus an offset of 1; the initial rank is not stated and is taken as dell.
* Levenberg-Marquardt damping (the Navier-Stokes experiment, Section 5.1.3): the first step takes mu
  from the rule above, later steps from the gain ratio of the previous step (gain_ratio, lm_update),
  never below the rule's roundoff term gamma eps lam1_hat.
* the sketch is of the undamped Gramian (Alg. 4 sketches G_fun and forms mu afterwards); the CG
  operator is G + mu I and the preconditioner uses the same mu (Alg. 3, Alg. 4).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import cg as _cg
from . import mlp, nystrom

EPS = {"f64": 2.0 ** -52, "f32": 2.0 ** -23}


def damping(lam1_hat: float, loss_value: float, eps: float, gamma: float = 10.0,
            c: float = 1e-4) -> float:
    """mu = max(gamma * eps * lam1_hat, c * L^2)."""
    return max(gamma * eps * lam1_hat, c * loss_value ** 2)


def next_rank(lam_hat, mu: float, ell: int, ell_max: int, dell: int, offset: int = 1) -> int:
    """Sketch size for the next NGD step (Alg. 4, after the preconditioner is built; Section 4.3).

    lam_hat holds the ell Nystrom eigenvalues in descending order. If the smallest, lam_hat_ell, is
    above 10 mu the rank grows by dell (capped at ell_max). Otherwise it becomes the first (1-based)
    index i with lam_hat_i < 10 mu plus `offset`, capped at ell_max. When no eigenvalue lies strictly
    below 10 mu (lam_hat_ell equal to 10 mu) the rank is kept."""
    lam = np.asarray(lam_hat, dtype=np.float64)[:ell]
    thresh = 10.0 * mu
    if lam[ell - 1] > thresh:
        return min(ell + dell, ell_max)
    below = np.nonzero(lam < thresh)[0]
    if below.size == 0:
        return min(ell, ell_max)
    return min(int(below[0]) + 1 + offset, ell_max)


def gain_ratio(loss0: float, loss1: float, alpha: float, gd: float, dGd: float) -> float:
    """Actual over predicted decrease of the step theta - alpha d, the prediction from the Gauss-Newton
    model of the loss, L(theta - s) ~ L - g^T s + s^T G s / 2: rho = (L0 - L1) / (alpha g^T d -
    alpha^2 d^T G d / 2); -1 when no step was taken or the model predicts no decrease."""
    pred = alpha * gd - 0.5 * alpha * alpha * dGd
    if alpha <= 0.0 or pred <= 0.0:
        return -1.0
    return (loss0 - loss1) / pred


def lm_update(mu: float, rho: float, floor: float = 0.0) -> float:
    """Levenberg-Marquardt damping update (the heuristic of Section 5.1.3; the factors of the trust-region
    radius rule of Nocedal and Wright, with the damping moving opposite to the radius): 4 mu for a poor
    step (rho < 1/4), mu / 2 for a good one (rho > 3/4), else unchanged, and never below `floor`."""
    m = 4.0 * mu if rho < 0.25 else (0.5 * mu if rho > 0.75 else mu)
    return max(m, floor)


def power_method(G_fun, v0: np.ndarray, iters: int = 4) -> float:
    """Estimate of the largest eigenvalue of a PSD operator: v <- G v / ||G v||, Rayleigh quotient."""
    v = v0 / np.linalg.norm(v0)
    lam = 0.0
    for _ in range(iters):
        w = G_fun(v)
        lam = float(v @ w)
        v = w / np.linalg.norm(w)
    return lam


def armijo(loss_fn, theta, d, g, L0, c1=1e-4, max_halvings=30):
    """Backtracking along theta - alpha d; returns (alpha, L(theta - alpha d))."""
    slope = float(g @ d)
    alpha = 1.0
    for _ in range(max_halvings + 1):
        Lt = loss_fn(theta - alpha * d)
        if Lt <= L0 - c1 * alpha * slope:
            return alpha, Lt
        alpha *= 0.5
    return 0.0, L0


@dataclasses.dataclass
class StepInfo:
    loss: float
    mu: float
    lam_hat: Optional[np.ndarray]
    lam1: float
    cg: _cg.CGResult
    alpha: float
    loss_new: float
    direction: np.ndarray


def ngd_step(theta, prob, *, solver="nystrom", Omega=None, rtol=1e-6, maxit=None, eps=None,
             power_v0=None, power_iters=4) -> tuple:
    """theta_{k+1} = theta_k - alpha_k d_k (Alg. 1), d from matrix-free pCG (Alg. 3) with the Nystrom
    builder of Alg. 4 at a fixed sketch size (solver="nystrom") or without preconditioner ("cg")."""
    eps = EPS[prob.dtype] if eps is None else eps
    r, J = mlp.residual_and_jacobian(theta, prob)
    L0 = 0.5 * float(r @ r)
    g = J.T @ r
    G_fun = lambda V: J.T @ (J @ V)
    P = theta.size
    if solver == "nystrom":
        U, lam_hat, _ = nystrom.nystrom_alg6(G_fun, Omega)
        lam1 = float(lam_hat[0])
    else:
        U = lam_hat = None
        lam1 = power_method(G_fun, power_v0, power_iters)
    mu = prob.lam if prob.lam is not None else damping(lam1, L0, eps)
    A_fun = lambda v: G_fun(v) + mu * v
    M_fun = None if U is None else (lambda v: nystrom.precond_apply(U, lam_hat, mu, v))
    res = _cg.pcg(A_fun, g, rtol, maxit if maxit is not None else (1000 if U is not None else P), M_fun)
    alpha, L1 = armijo(lambda th: mlp.loss(th, prob), theta, res.x, g, L0)
    info = StepInfo(L0, mu, lam_hat, lam1, res, alpha, L1, res.x)
    return theta - alpha * res.x, info
