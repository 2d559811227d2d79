"""tanh MLP, Taylor-mode Laplacian, PINN residuals and their exact parameter Jacobian (FP64).

Test infrastructure (see the package docstring); imports nothing from the GPU path.

Network (Section 2.3): x_0 = x, x_l = tanh(W_l x_{l-1} + b_l) for hidden layers, u = W_{L+1} x_L +
b_{L+1}; theta = [W_1, b_1, ..., W_{L+1}, b_{L+1}] with each W stored row-major (out x in).

Residuals (one per collocation point r, weighted by the square root of its quadrature weight so that
the loss is 1/2 sum_r w_r res_r^2 and G = J_w^T J_w is the Gramian of eq. G_matrixfree):

* Poisson interior (eq. energy_poisson): res = Laplace(u) + f.
* heat interior (eq. heat_energy):       res = u_t - Laplace_x(u) - f.
* boundary / initial rows:              res = u - g.

The Laplacian is obtained by propagating, through every layer, the value h, the gradient G with
respect to the Laplacian coordinates S, the Laplacian L and (heat) the time derivative T:
z = W h + b, Gz = W G, Lz = W L, Tz = W T and, with a = tanh z, s1 = 1 - a^2, s2 = -2 a s1,
h' = a, G' = s1 Gz, L' = s1 Lz + s2 sum_k Gz_k^2, T' = s1 Tz. This is the chain rule written out;
the paper obtains the same derivatives by automatic differentiation (Section 3.2, Section 4.1.1).
"""
from __future__ import annotations

import numpy as np

from workloads import KIND_INTERIOR, PDE_HEAT, PDE_POISSON, num_params


def unpack(theta: np.ndarray, widths) -> list:
    """Split theta into [(W_1, b_1), ..., (W_{L+1}, b_{L+1})] (Section 2.3)."""
    out, off = [], 0
    for n_in, n_out in zip(widths[:-1], widths[1:]):
        W = theta[off:off + n_out * n_in].reshape(n_out, n_in)
        off += n_out * n_in
        b = theta[off:off + n_out]
        off += n_out
        out.append((W, b))
    assert off == theta.size == num_params(widths)
    return out


def derivative_dims(pde: int, d: int):
    """(Laplacian coordinates S, time coordinate or None)."""
    if pde == PDE_POISSON:
        return list(range(d)), None
    if pde == PDE_HEAT:
        return list(range(d - 1)), d - 1
    raise ValueError(pde)


def _input_channels(X, S, t):
    N, d = X.shape
    G = np.zeros((N, d, len(S)))
    for k, s in enumerate(S):
        G[:, s, k] = 1.0
    T = np.zeros((N, d))
    if t is not None:
        T[:, t] = 1.0
    return X.astype(np.float64).copy(), G, np.zeros((N, d)), T


def taylor_forward(theta, widths, X, pde):
    """Value u, gradient grad_S u, Laplacian Laplace_S u and time derivative u_t at every point.

    Returns (u, grad (N,|S|), lap, ut, cache) where cache holds per-layer inputs and pre-activations
    for the reverse sweep."""
    params = unpack(theta, widths)
    S, t = derivative_dims(pde, X.shape[1])
    h, G, L, T = _input_channels(X, S, t)
    cache = []
    for W, b in params[:-1]:
        z = h @ W.T + b
        Gz = np.einsum("oi,nik->nok", W, G)
        Lz = L @ W.T
        Tz = T @ W.T
        cache.append(((h, G, L, T), (z, Gz, Lz, Tz)))
        a = np.tanh(z)
        s1 = 1.0 - a * a
        s2 = -2.0 * a * s1
        h = a
        G = s1[:, :, None] * Gz
        L = s1 * Lz + s2 * np.sum(Gz * Gz, axis=2)
        T = s1 * Tz
    W, b = params[-1]
    u = h @ W[0] + b[0]
    grad = np.einsum("i,nik->nk", W[0], G)
    lap = L @ W[0]
    ut = T @ W[0]
    cache.append(((h, G, L, T), None))
    return u, grad, lap, ut, cache


def residual(theta, prob, X=None):
    """Unweighted residual res_r for every row (see the module docstring)."""
    X = prob.X if X is None else X
    u, _, lap, ut, _ = taylor_forward(theta, prob.widths, X, prob.pde)
    interior = prob.kind == KIND_INTERIOR
    if prob.pde == PDE_POISSON:
        pde_res = lap + prob.f
    else:
        pde_res = ut - lap - prob.f
    return np.where(interior, pde_res, u - prob.g)


def weighted_residual(theta, prob):
    """r_w = sqrt(w) * res."""
    return np.sqrt(prob.w) * residual(theta, prob)


def loss(theta, prob) -> float:
    """L(theta) = 1/2 sum_r w_r res_r^2 (discrete eq. energy_poisson / heat_energy)."""
    r = weighted_residual(theta, prob)
    return 0.5 * float(r @ r)


def _output_adjoint(prob):
    """d r_w / d(u, Laplace u, u_t) per row: the seed of the reverse sweep."""
    sw = np.sqrt(prob.w)
    interior = prob.kind == KIND_INTERIOR
    a_v = np.where(interior, 0.0, sw)
    if prob.pde == PDE_POISSON:
        a_L = np.where(interior, sw, 0.0)
        a_T = np.zeros_like(sw)
    else:
        a_L = np.where(interior, -sw, 0.0)
        a_T = np.where(interior, sw, 0.0)
    return a_v, a_L, a_T


def jacobian(theta, prob, rows=None) -> np.ndarray:
    """Exact J_w = d r_w / d theta by reverse mode through the Taylor-mode forward (N x p).

    For a layer z = W h + b with channels c (value, gradient k, Laplacian, time), the parameter
    derivative is d/dW[o,i] = sum_c zbar_c[o] h_c[i] and d/db[o] = zbar_value[o]."""
    X = prob.X if rows is None else prob.X[rows]
    sub = prob if rows is None else _subproblem(prob, rows)
    params = unpack(theta, prob.widths)
    _, _, _, _, cache = taylor_forward(theta, prob.widths, X, prob.pde)
    N = X.shape[0]
    a_v, a_L, a_T = _output_adjoint(sub)
    blocks = []
    # output layer (linear): u = W h + b, lap = W L, ut = W T, grad = W G
    (h, G, L, T), _ = cache[-1]
    W, _ = params[-1]
    blocks.append(((a_v[:, None] * h + a_L[:, None] * L + a_T[:, None] * T)[:, None, :], a_v[:, None]))
    # adjoints of the last hidden layer's outputs
    av = a_v[:, None] * W[0][None, :]
    aG = np.zeros_like(G)
    aL = a_L[:, None] * W[0][None, :]
    aT = a_T[:, None] * W[0][None, :]
    for li in range(len(params) - 2, -1, -1):
        W, _ = params[li]
        (h_in, G_in, L_in, T_in), (z, Gz, Lz, Tz) = cache[li]
        a = np.tanh(z)
        s1 = 1.0 - a * a
        s2 = -2.0 * a * s1
        s3 = -2.0 * s1 * (s1 - 2.0 * a * a)
        gsq = np.sum(Gz * Gz, axis=2)
        zG = s1[:, :, None] * aG + 2.0 * (s2 * aL)[:, :, None] * Gz
        zL = s1 * aL
        zT = s1 * aT
        zv = s1 * av + s2 * np.sum(Gz * aG, axis=2) + (s2 * Lz + s3 * gsq) * aL + s2 * Tz * aT
        dW = (np.einsum("no,ni->noi", zv, h_in) + np.einsum("nok,nik->noi", zG, G_in)
              + np.einsum("no,ni->noi", zL, L_in) + np.einsum("no,ni->noi", zT, T_in))
        blocks.append((dW, zv))
        av = zv @ W
        aG = np.einsum("nok,oi->nik", zG, W)
        aL = zL @ W
        aT = zT @ W
    cols = []
    for dW, db in reversed(blocks):
        cols.append(dW.reshape(N, -1))
        cols.append(db.reshape(N, -1))
    return np.concatenate(cols, axis=1)


def _subproblem(prob, rows):
    import dataclasses
    return dataclasses.replace(prob, X=prob.X[rows], kind=prob.kind[rows], w=prob.w[rows],
                               f=prob.f[rows], g=prob.g[rows])


def residual_and_jacobian(theta, prob, chunk=2048):
    """(r_w, J_w), the Jacobian assembled in row chunks to bound memory."""
    r = weighted_residual(theta, prob)
    N = prob.n_rows
    J = np.empty((N, num_params(prob.widths)))
    for s in range(0, N, chunk):
        rows = np.arange(s, min(N, s + chunk))
        J[rows] = jacobian(theta, prob, rows)
    return r, J


def gradient(theta, prob) -> np.ndarray:
    """Euclidean gradient of the loss: grad L = J_w^T r_w (Alg. 1, first step)."""
    r, J = residual_and_jacobian(theta, prob)
    return J.T @ r


def solution_error_sums(theta, widths, X, u_ref, grad_ref) -> np.ndarray:
    """The four sums behind the relative L2 and H1 errors of u_theta against a reference solution on
    evaluation points X (n x d), the accuracy measure of the experiments of Section 5 (Monte Carlo over
    uniform random points): [sum (u - u_ref)^2, sum |grad u - grad u_ref|^2, sum u_ref^2,
    sum |grad u_ref|^2], with grad over all d inputs."""
    X = np.asarray(X, dtype=np.float64)
    if X.shape[0] == 0:
        return np.zeros(4)
    # with every input a Laplacian coordinate, the forward sweep's gradient channel is grad_x u
    u, grad, _, _, _ = taylor_forward(theta, widths, X, PDE_POISSON)
    u_ref = np.asarray(u_ref, dtype=np.float64)
    grad_ref = np.asarray(grad_ref, dtype=np.float64)
    return np.array([np.sum((u - u_ref) ** 2), np.sum((grad - grad_ref) ** 2), np.sum(u_ref ** 2),
                     np.sum(grad_ref ** 2)])


def relative_errors(sums) -> tuple:
    """(relative L2 error, relative H1 error) from the four sums of solution_error_sums."""
    s = np.asarray(sums, dtype=np.float64)
    return float(np.sqrt(s[0] / s[2])), float(np.sqrt((s[0] + s[1]) / (s[2] + s[3])))
