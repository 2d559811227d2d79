"""Pins of the oracle's Navier-Stokes rows (the Kovasznay flow of Section 5.1.3), CPU only.

The residual rows are checked on the exact Kovasznay solution (closed-form derivatives typed here), the
network channels against finite differences in space, and the Gauss-Newton Jacobian against central
differences in theta and against torch CPU automatic differentiation of an independent torch
implementation of the rows."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import navier_stokes as ns


def _small(n_interior=5, n_boundary=4, widths=(2, 5, 4, 2), seed=2):
    return wl.kovasznay(widths=widths, n_interior=n_interior, n_boundary=n_boundary, seed=seed)


def _theta(prob, seed):
    th = wl.ns_glorot_theta(prob.widths, seed)
    return th + 0.1 * np.random.default_rng(seed + 11).standard_normal(th.size)  # nonzero biases


def test_parameter_count_section_5_1_3():
    # two networks with three hidden layers of 45: (2*45+45) + 2*(45*45+45) + (45*2+2) = 4,367 for the
    # velocity, (2*45+45) + 2*(45*45+45) + (45+1) = 4,321 for the pressure
    assert wl.num_params((2, 45, 45, 45, 2)) == 4367
    assert wl.num_params((2, 45, 45, 45, 1)) == 4321
    assert wl.ns_num_params((2, 45, 45, 45, 2)) == 8688
    prob = wl.config("paper_ns")
    assert prob.n_params == 8688 and prob.n_rows == 3 * 10000 + 2 * 1000


def test_exact_kovasznay_flow_has_zero_residual():
    """eq. navier_residual on the exact solution (f = 0, g = the exact velocity) vanishes: Laplacians
    and the pressure gradient from their closed forms, lambda from its definition."""
    nu = 1.0 / 40.0
    prob = wl.kovasznay(n_interior=50, n_boundary=30, nu=nu, seed=4)
    U, gU, _ = wl.kovasznay_solution(prob.X, nu)
    lam = 1.0 / (2 * nu) - math.sqrt(1.0 / (4 * nu * nu) + 4 * math.pi ** 2)
    x, y = prob.X[:, 0], prob.X[:, 1]
    e = np.exp(lam * x)
    k2 = lam * lam - 4 * math.pi ** 2
    lapU = np.stack([-e * np.cos(2 * math.pi * y) * k2, lam / (2 * math.pi) * e * np.sin(2 * math.pi * y) * k2], 1)
    gradP = np.stack([-lam * np.exp(2 * lam * x), np.zeros_like(x)], 1)
    res = ns.rows_from_channels(prob.kind, U, gU, lapU, gradP, prob.f, prob.g, nu)
    assert np.max(np.abs(res)) < 1e-11
    # each term matters: a dropped convective term, pressure gradient or viscous term leaves O(1) rows
    mom = (prob.kind == wl.KIND_NS_MOMENTUM_X) | (prob.kind == wl.KIND_NS_MOMENTUM_Y)
    for bad in (dict(gradP=0 * gradP), dict(lapU=0 * lapU), dict(U=0 * U)):
        args = dict(U=U, gU=gU, lapU=lapU, gradP=gradP)
        args.update(bad)
        r = ns.rows_from_channels(prob.kind, args["U"], args["gU"], args["lapU"], args["gradP"], prob.f, prob.g, nu)
        assert np.max(np.abs(r[mom])) > 1e-2


def test_exact_solution_gradient_and_mean_pressure():
    """The workload's exact gradient against central differences; the pressure has mean zero over the
    box (midpoint rule on a fine grid)."""
    X = np.random.default_rng(1).uniform([-0.5, -0.5], [1.0, 1.5], size=(20, 2))
    _, g, _ = wl.kovasznay_solution(X)
    h = 1e-6
    for j in range(2):
        e = np.zeros(2)
        e[j] = h
        fd = (wl.kovasznay_solution(X + e)[0] - wl.kovasznay_solution(X - e)[0]) / (2 * h)
        np.testing.assert_allclose(g[:, :, j], fd, atol=1e-7)
    n = 2000
    xs = -0.5 + 1.5 * (np.arange(n) + 0.5) / n
    Xg = np.stack([xs, np.zeros(n)], 1)
    assert abs(np.mean(wl.kovasznay_solution(Xg)[2])) < 1e-6


def test_network_channels_match_spatial_differences():
    prob = _small()
    t1, _ = ns.split_theta(_theta(prob, 3), prob.widths)
    X = prob.X[:8]
    val, grad, lap, _ = ns.forward(t1, prob.widths, X)
    h = 1e-4
    fd_g, fd_lap = np.zeros_like(grad), np.zeros_like(lap)
    for j in range(2):
        e = np.zeros(2)
        e[j] = h
        up, um = ns.forward(t1, prob.widths, X + e)[0], ns.forward(t1, prob.widths, X - e)[0]
        fd_g[:, :, j] = (up - um) / (2 * h)
        fd_lap += (up - 2 * val + um) / h ** 2
    np.testing.assert_allclose(grad, fd_g, atol=1e-8)
    np.testing.assert_allclose(lap, fd_lap, atol=2e-5)


def test_jacobian_matches_central_differences():
    prob = _small(seed=5)
    theta = _theta(prob, 5)
    J = ns.jacobian(theta, prob)
    h = 1e-6
    Jfd = np.empty_like(J)
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        Jfd[:, k] = (ns.weighted_residual(theta + e, prob) - ns.weighted_residual(theta - e, prob)) / (2 * h)
    assert np.max(np.abs(J - Jfd)) <= 1e-7 * np.max(np.abs(J))
    # the pressure columns vanish on the continuity and boundary rows
    n1 = wl.num_params(prob.widths)
    quiet = (prob.kind != wl.KIND_NS_MOMENTUM_X) & (prob.kind != wl.KIND_NS_MOMENTUM_Y)
    assert np.all(J[quiet, n1:] == 0.0)


def test_jacobian_matches_torch_cpu_autodiff():
    torch = pytest.importorskip("torch")
    prob = _small(n_interior=3, n_boundary=2, widths=(2, 4, 3, 2), seed=6)
    theta = _theta(prob, 6)
    pw = wl.pressure_widths(prob.widths)
    n1 = wl.num_params(prob.widths)

    def net(th, widths, x):
        h, off = x, 0
        for li, (a, b) in enumerate(zip(widths[:-1], widths[1:])):
            W = th[off:off + a * b].reshape(b, a)
            off += a * b
            c = th[off:off + b]
            off += b
            h = W @ h + c
            if li < len(widths) - 2:
                h = torch.tanh(h)
        return h

    def res_w(th):
        out = []
        for r in range(prob.n_rows):
            x = torch.tensor(prob.X[r])
            uv = lambda z: net(th[:n1], prob.widths, z)
            pp = lambda z: net(th[n1:], pw, z)[0]
            U = uv(x)
            gU = torch.autograd.functional.jacobian(uv, x, create_graph=True)  # [k, j]
            gP = torch.autograd.functional.jacobian(pp, x, create_graph=True)
            lap = torch.stack([torch.diagonal(torch.autograd.functional.hessian(
                lambda z, k=k: uv(z)[k], x, create_graph=True)).sum() for k in range(2)])
            k = int(prob.kind[r])
            if k in (wl.KIND_NS_MOMENTUM_X, wl.KIND_NS_MOMENTUM_Y):
                c = 0 if k == wl.KIND_NS_MOMENTUM_X else 1
                v = -prob.nu * lap[c] + U[0] * gU[c, 0] + U[1] * gU[c, 1] + gP[c] - prob.f[r]
            elif k == wl.KIND_NS_CONTINUITY:
                v = gU[0, 0] + gU[1, 1]
            else:
                v = U[0 if k == wl.KIND_NS_BOUNDARY_U else 1] - prob.g[r]
            out.append(math.sqrt(prob.w[r]) * v)
        return torch.stack(out)

    Jt = torch.autograd.functional.jacobian(res_w, torch.tensor(theta)).numpy()
    J = ns.jacobian(theta, prob)
    np.testing.assert_allclose(J, Jt, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(ns.weighted_residual(theta, prob), res_w(torch.tensor(theta)).detach().numpy(),
                               rtol=1e-12, atol=1e-14)


def test_loss_gradient_matches_differences():
    """J_w^T r_w is the gradient of the loss (Alg. 1, first step) for the Navier-Stokes rows too."""
    prob = _small(seed=8)
    theta = _theta(prob, 8)
    r, J = ns.residual_and_jacobian(theta, prob, chunk=7)
    g = J.T @ r
    rng = np.random.default_rng(0)
    v = rng.standard_normal(theta.size)
    h = 1e-6
    fd = (ns.loss(theta + h * v, prob) - ns.loss(theta - h * v, prob)) / (2 * h)
    assert abs(fd - g @ v) <= 1e-7 * max(1.0, abs(fd))


def test_velocity_error_sums_of_exact_velocity_network():
    """A velocity equal to the reference gives zero error sums; the reference sums are the plain sums."""
    prob = _small()
    theta = _theta(prob, 9)
    X = prob.X[:10]
    t1 = theta[:wl.num_params(prob.widths)]
    U, gU, _, _ = ns.forward(t1, prob.widths, X)
    s = ns.velocity_error_sums(theta, prob.widths, X, U, gU)
    assert s[0] == 0.0 and s[1] == 0.0
    np.testing.assert_allclose(s[2:], [np.sum(U ** 2), np.sum(gU ** 2)])
