"""Steady incompressible Navier-Stokes rows (the Kovasznay flow of Section 5.1.3): residuals, loss and
their exact parameter Jacobian, in FP64.

Test infrastructure (see the package docstring); imports nothing from the GPU path.

Two tanh MLPs (Section 2.3): the velocity network (u_1, u_2) = u_{theta_1}(x, y) with two outputs and
the pressure network p = p_{theta_2}(x, y) with one, theta = [theta_1, theta_2] (Section 5.1.3). The
residual of eq. navier_residual, split into rows:

* momentum k (k = 1, 2):  -nu Laplace u_k + u_1 d_x u_k + u_2 d_y u_k + d_k p - f_k
* continuity:             d_x u_1 + d_y u_2
* boundary, component k:  u_k - g_k

each multiplied by sqrt(w_r) so that 1/2 sum_r w_r res_r^2 is the quadrature of eq. navier_loss. The
Gauss-Newton metric of the section is J_w^T J_w, J_w = d r_w / d theta the Jacobian of the (nonlinear)
weighted residual rows.

The networks' value, gradient and Laplacian come from the Taylor-mode forward sweep of `mlp` (same
recurrences, several outputs); the Jacobian is the reverse sweep of those channels seeded, per row, with
the derivative of the row's residual with respect to the output channels (the linearisation of the
convective term puts point-dependent seeds on the value and gradient channels).
"""
from __future__ import annotations

import numpy as np

from workloads import (KIND_NS_BOUNDARY_U, KIND_NS_BOUNDARY_V, KIND_NS_CONTINUITY, KIND_NS_MOMENTUM_X,
                       KIND_NS_MOMENTUM_Y, num_params, pressure_widths)

from .mlp import unpack


def split_theta(theta: np.ndarray, widths) -> tuple:
    """(theta_1, theta_2): the velocity network's parameters, then the pressure network's."""
    n1 = num_params(widths)
    assert theta.size == n1 + num_params(pressure_widths(widths))
    return theta[:n1], theta[n1:]


def forward(theta_net: np.ndarray, widths, X: np.ndarray):
    """Value (N, k), gradient (N, k, 2) with [., o, j] = d out_o / d x_j, and Laplacian (N, k) of every
    output of one tanh MLP with inputs (x, y), by the Taylor-mode recurrences of `mlp` (value h,
    gradient G, Laplacian L; z = W h + b, Gz = W G, Lz = W L, then h' = a, G' = s1 Gz,
    L' = s1 Lz + s2 |Gz|^2 with a = tanh z, s1 = 1 - a^2, s2 = -2 a s1). Also returns the cache of
    every layer's inputs and pre-activation channels for the reverse sweep."""
    params = unpack(theta_net, widths)
    N = X.shape[0]
    h = np.asarray(X, dtype=np.float64).copy()
    G = np.zeros((N, 2, 2))
    G[:, 0, 0] = 1.0
    G[:, 1, 1] = 1.0
    L = np.zeros((N, 2))
    cache = []
    for W, b in params[:-1]:
        z = h @ W.T + b
        Gz = np.einsum("oi,nij->noj", W, G)
        Lz = L @ W.T
        cache.append(((h, G, L), (z, Gz, Lz)))
        a = np.tanh(z)
        s1 = 1.0 - a * a
        s2 = -2.0 * a * s1
        h = a
        G = s1[:, :, None] * Gz
        L = s1 * Lz + s2 * np.sum(Gz * Gz, axis=2)
    W, b = params[-1]
    val = h @ W.T + b
    grad = np.einsum("ki,nij->nkj", W, G)
    lap = L @ W.T
    cache.append(((h, G, L), None))
    return val, grad, lap, cache


def rows_from_channels(kind, U, gradU, lapU, gradP, f, g, nu):
    """Unweighted residual of every row from the velocity (N, 2), its gradient (N, 2, 2), its Laplacian
    (N, 2) and the pressure gradient (N, 2) at the row's point (eq. navier_residual)."""
    conv = np.einsum("nj,nkj->nk", U, gradU)  # (u . grad) u_k
    mom = -nu * lapU + conv + gradP
    res = np.zeros(len(kind))
    res = np.where(kind == KIND_NS_MOMENTUM_X, mom[:, 0] - f, res)
    res = np.where(kind == KIND_NS_MOMENTUM_Y, mom[:, 1] - f, res)
    res = np.where(kind == KIND_NS_CONTINUITY, gradU[:, 0, 0] + gradU[:, 1, 1], res)
    res = np.where(kind == KIND_NS_BOUNDARY_U, U[:, 0] - g, res)
    res = np.where(kind == KIND_NS_BOUNDARY_V, U[:, 1] - g, res)
    return res


def _channels(theta, prob, X):
    t1, t2 = split_theta(theta, prob.widths)
    U, gU, lU, c1 = forward(t1, prob.widths, X)
    P, gP, _, c2 = forward(t2, pressure_widths(prob.widths), X)
    return U, gU, lU, gP[:, 0, :], (t1, c1), (t2, c2)


def residual(theta, prob):
    U, gU, lU, gP, _, _ = _channels(theta, prob, prob.X)
    return rows_from_channels(prob.kind, U, gU, lU, gP, prob.f, prob.g, prob.nu)


def weighted_residual(theta, prob):
    """r_w = sqrt(w) * res."""
    return np.sqrt(prob.w) * residual(theta, prob)


def loss(theta, prob) -> float:
    """1/2 sum_r w_r res_r^2 (the quadrature of eq. navier_loss)."""
    r = weighted_residual(theta, prob)
    return 0.5 * float(r @ r)


def seeds(kind, U, gradU, nu, sw):
    """d r_w / d(output channels) per row (the Gauss-Newton linearisation of eq. navier_residual):
    velocity (value (N, 2), gradient (N, 2, 2), Laplacian (N, 2)) and pressure (value (N, 1), gradient
    (N, 1, 2), Laplacian (N, 1))."""
    N = len(kind)
    av, ag, aL = np.zeros((N, 2)), np.zeros((N, 2, 2)), np.zeros((N, 2))
    pv, pg, pL = np.zeros((N, 1)), np.zeros((N, 1, 2)), np.zeros((N, 1))
    for k, kk in ((0, KIND_NS_MOMENTUM_X), (1, KIND_NS_MOMENTUM_Y)):
        m = kind == kk
        # -nu Laplace u_k + sum_j u_j d_j u_k + d_k p: d/du_j = d_j u_k, d/d(d_j u_k) = u_j
        av[m, 0] = gradU[m, k, 0]
        av[m, 1] = gradU[m, k, 1]
        ag[m, k, 0] = U[m, 0]
        ag[m, k, 1] = U[m, 1]
        aL[m, k] = -nu
        pg[m, 0, k] = 1.0
    m = kind == KIND_NS_CONTINUITY
    ag[m, 0, 0] = 1.0
    ag[m, 1, 1] = 1.0
    av[kind == KIND_NS_BOUNDARY_U, 0] = 1.0
    av[kind == KIND_NS_BOUNDARY_V, 1] = 1.0
    s = sw[:, None]
    return (av * s, ag * s[:, :, None], aL * s), (pv * s, pg * s[:, :, None], pL * s)


def _reverse(theta_net, widths, cache, av_o, ag_o, aL_o):
    """Parameter derivatives of sum_o (av_o out_o + ag_o . grad out_o + aL_o Laplace out_o) per row by
    the reverse sweep of the Taylor channels (N x p_net)."""
    params = unpack(theta_net, widths)
    N = av_o.shape[0]
    blocks = []
    (h, G, L), _ = cache[-1]
    W, _ = params[-1]
    dW = (av_o[:, :, None] * h[:, None, :] + np.einsum("nkj,nij->nki", ag_o, G) + aL_o[:, :, None] * L[:, None, :])
    blocks.append((dW, av_o))
    av = av_o @ W
    aG = np.einsum("nkj,ki->nij", ag_o, W)
    aL = aL_o @ W
    for li in range(len(params) - 2, -1, -1):
        W, _ = params[li]
        (h_in, G_in, L_in), (z, Gz, Lz) = cache[li]
        a = np.tanh(z)
        s1 = 1.0 - a * a
        s2 = -2.0 * a * s1
        s3 = -2.0 * s1 * (s1 - 2.0 * a * a)
        gsq = np.sum(Gz * Gz, axis=2)
        zG = s1[:, :, None] * aG + 2.0 * (s2 * aL)[:, :, None] * Gz
        zL = s1 * aL
        zv = s1 * av + s2 * np.sum(Gz * aG, axis=2) + (s2 * Lz + s3 * gsq) * aL
        dW = (np.einsum("no,ni->noi", zv, h_in) + np.einsum("noj,nij->noi", zG, G_in)
              + np.einsum("no,ni->noi", zL, L_in))
        blocks.append((dW, zv))
        av = zv @ W
        aG = np.einsum("noj,oi->nij", zG, W)
        aL = zL @ W
    cols = []
    for dW, db in reversed(blocks):
        cols.append(dW.reshape(N, -1))
        cols.append(db.reshape(N, -1))
    return np.concatenate(cols, axis=1)


def jacobian(theta, prob, rows=None) -> np.ndarray:
    """Exact J_w = d r_w / d theta (N x p): the velocity network's columns, then the pressure
    network's."""
    sel = np.arange(prob.n_rows) if rows is None else np.asarray(rows)
    X = prob.X[sel]
    U, gU, lU, gP, (t1, c1), (t2, c2) = _channels(theta, prob, X)
    (av, ag, aL), (pv, pg, pL) = seeds(prob.kind[sel], U, gU, prob.nu, np.sqrt(prob.w[sel]))
    J1 = _reverse(t1, prob.widths, c1, av, ag, aL)
    J2 = _reverse(t2, pressure_widths(prob.widths), c2, pv, pg, pL)
    return np.concatenate([J1, J2], axis=1)


def residual_and_jacobian(theta, prob, chunk=2048):
    """(r_w, J_w), the Jacobian assembled in row chunks to bound memory."""
    r = weighted_residual(theta, prob)
    N = prob.n_rows
    J = np.empty((N, theta.size))
    for s in range(0, N, chunk):
        rows = np.arange(s, min(N, s + chunk))
        J[rows] = jacobian(theta, prob, rows)
    return r, J


def velocity_error_sums(theta, widths, X, u_ref, grad_ref) -> np.ndarray:
    """The four sums behind the relative L2 and H1 errors of the velocity against a reference on
    evaluation points X (the accuracy measure of Section 5.1.3, Monte Carlo over uniform points):
    [sum |u - u_ref|^2, sum |grad u - grad u_ref|^2, sum |u_ref|^2, sum |grad u_ref|^2], the gradient
    over both inputs of both components."""
    X = np.asarray(X, dtype=np.float64)
    if X.shape[0] == 0:
        return np.zeros(4)
    t1 = theta[:num_params(widths)]
    U, gU, _, _ = forward(t1, widths, X)
    return np.array([np.sum((U - u_ref) ** 2), np.sum((gU - grad_ref) ** 2), np.sum(u_ref ** 2),
                     np.sum(grad_ref ** 2)])
