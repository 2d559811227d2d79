"""Pins of the oracle's network, residuals and Jacobian (CPU only).

Each check compares the oracle with something computed another way: finite differences, closed forms
of a one-unit network, torch CPU automatic differentiation, and the manufactured solutions."""
import numpy as np
import pytest

import workloads as wl
from oracle import mlp


def _fd_jacobian(theta, prob, h=1e-6):
    J = np.empty((prob.n_rows, theta.size))
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        J[:, k] = (mlp.weighted_residual(theta + e, prob) - mlp.weighted_residual(theta - e, prob)) / (2 * h)
    return J


CASES = [
    dict(pde=wl.PDE_POISSON, d=2, widths=(2, 6, 5, 1)),
    dict(pde=wl.PDE_POISSON, d=3, widths=(3, 5, 4, 4, 1)),
    dict(pde=wl.PDE_HEAT, d=3, widths=(3, 5, 6, 1)),
]


def test_param_count_section_2_3():
    # hand-counted: sum_l n_l n_{l-1} + n_l
    assert wl.num_params((2, 32, 32, 1)) == 64 + 32 + 1024 + 32 + 32 + 1 == 1185
    assert wl.num_params((2, 64, 64, 64, 1)) == 8577
    assert wl.num_params((5, 128, 128, 128, 1)) == 33921
    assert wl.num_params((3, 64, 64, 64, 64, 1)) == 12801


@pytest.mark.parametrize("case", CASES)
def test_jacobian_matches_central_differences(case):
    prob = wl.small_problem(**case, n_interior=10, n_boundary=6, seed=3)
    theta = wl.glorot_theta(prob.widths, 3)
    theta = theta + 0.1 * np.random.default_rng(0).standard_normal(theta.size)  # nonzero biases
    J = mlp.jacobian(theta, prob)
    Jfd = _fd_jacobian(theta, prob)
    assert np.max(np.abs(J - Jfd)) <= 1e-7 * np.max(np.abs(J))


def _fd_derivatives(theta, widths, X, pde, h=1e-4):
    u0 = mlp.taylor_forward(theta, widths, X, pde)[0]
    d = X.shape[1]
    grad, second = np.empty((X.shape[0], d)), np.empty((X.shape[0], d))
    for k in range(d):
        e = np.zeros(d)
        e[k] = h
        up = mlp.taylor_forward(theta, widths, X + e, pde)[0]
        um = mlp.taylor_forward(theta, widths, X - e, pde)[0]
        grad[:, k] = (up - um) / (2 * h)
        second[:, k] = (up - 2 * u0 + um) / h ** 2
    return grad, second


@pytest.mark.parametrize("case", CASES)
def test_taylor_forward_matches_spatial_differences(case):
    prob = wl.small_problem(**case, n_interior=8, n_boundary=4, seed=5)
    theta = wl.glorot_theta(prob.widths, 5)
    u, grad, lap, ut, _ = mlp.taylor_forward(theta, prob.widths, prob.X, prob.pde)
    fd_grad, fd_second = _fd_derivatives(theta, prob.widths, prob.X, prob.pde)
    S, t = mlp.derivative_dims(prob.pde, prob.d)
    np.testing.assert_allclose(grad, fd_grad[:, S], atol=1e-8)
    np.testing.assert_allclose(lap, fd_second[:, S].sum(1), atol=2e-5)
    if t is not None:
        np.testing.assert_allclose(ut, fd_grad[:, t], atol=1e-8)


def test_one_unit_network_closed_form():
    """u = a tanh(v.x + c) + b: Laplace u = a s2(z) |v|^2 and the Jacobian columns in closed form."""
    rng = np.random.default_rng(7)
    prob = wl.small_problem(pde=wl.PDE_POISSON, d=2, widths=(2, 1, 1), n_interior=5, n_boundary=3, seed=7)
    v, c, a, b = rng.standard_normal(2), 0.3, 1.7, -0.4
    theta = np.concatenate([v, [c], [a], [b]])
    X = prob.X
    z = X @ v + c
    th = np.tanh(z)
    s1 = 1 - th ** 2
    s2 = -2 * th * s1
    s3 = -2 * s1 * (1 - 3 * th ** 2)
    vv = v @ v
    u, _, lap, _, _ = mlp.taylor_forward(theta, prob.widths, X, prob.pde)
    np.testing.assert_allclose(u, a * th + b, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(lap, a * s2 * vv, rtol=1e-13, atol=1e-14)
    sw = np.sqrt(prob.w)
    inner = prob.kind == wl.KIND_INTERIOR
    Jc = np.empty((prob.n_rows, 5))
    # interior: r = sw (a s2(z) |v|^2 + f)
    Jc[:, 0:2] = np.where(inner[:, None], (a * (s3 * vv)[:, None] * X + a * s2[:, None] * 2 * v) * sw[:, None],
                          (a * s1)[:, None] * X * sw[:, None])
    Jc[:, 2] = np.where(inner, a * s3 * vv, a * s1) * sw
    Jc[:, 3] = np.where(inner, s2 * vv, th) * sw
    Jc[:, 4] = np.where(inner, 0.0, 1.0) * sw
    np.testing.assert_allclose(mlp.jacobian(theta, prob), Jc, rtol=1e-12, atol=1e-14)


def test_output_bias_and_weight_columns():
    """Last-layer bias column: 0 on interior rows, sqrt(w) on boundary rows (Laplacian of a constant
    vanishes); last-layer weight columns on boundary rows are sqrt(w) times the last hidden layer."""
    prob = wl.small_problem(pde=wl.PDE_POISSON, d=2, widths=(2, 7, 6, 1), n_interior=9, n_boundary=5, seed=2)
    theta = wl.glorot_theta(prob.widths, 2)
    J = mlp.jacobian(theta, prob)
    sw = np.sqrt(prob.w)
    inner = prob.kind == wl.KIND_INTERIOR
    np.testing.assert_allclose(J[:, -1], np.where(inner, 0.0, sw), atol=1e-15)
    params = mlp.unpack(theta, prob.widths)
    h = prob.X
    for W, b in params[:-1]:
        h = np.tanh(h @ W.T + b)
    np.testing.assert_allclose(J[~inner, -7:-1], sw[~inner, None] * h[~inner], rtol=1e-13)


def test_gradient_matches_loss_differences():
    prob = wl.small_problem(pde=wl.PDE_HEAT, d=3, widths=(3, 6, 6, 1), n_interior=12, n_boundary=6, seed=4)
    theta = wl.glorot_theta(prob.widths, 4)
    g = mlp.gradient(theta, prob)
    h = 1e-6
    for k in range(0, theta.size, 7):
        e = np.zeros_like(theta)
        e[k] = h
        fd = (mlp.loss(theta + e, prob) - mlp.loss(theta - e, prob)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, np.abs(g).max())


@pytest.mark.parametrize("case", CASES)
def test_jacobian_matches_torch_cpu_autodiff(case):
    torch = pytest.importorskip("torch")
    prob = wl.small_problem(**case, n_interior=6, n_boundary=4, seed=9)
    theta = wl.glorot_theta(prob.widths, 9)
    S, t = mlp.derivative_dims(prob.pde, prob.d)
    X = torch.tensor(prob.X)
    inner = torch.tensor(prob.kind == wl.KIND_INTERIOR)

    def res_w(th):
        out, off = [], 0
        layers = []
        for n_in, n_out in zip(prob.widths[:-1], prob.widths[1:]):
            W = th[off:off + n_in * n_out].reshape(n_out, n_in)
            off += n_in * n_out
            b = th[off:off + n_out]
            off += n_out
            layers.append((W, b))

        def net(x):
            h = x
            for W, b in layers[:-1]:
                h = torch.tanh(W @ h + b)
            W, b = layers[-1]
            return (W @ h + b)[0]

        for r in range(X.shape[0]):
            x = X[r]
            if bool(inner[r]):
                H = torch.autograd.functional.hessian(net, x, create_graph=True)
                lap = sum(H[s, s] for s in S)
                if prob.pde == wl.PDE_POISSON:
                    val = lap + prob.f[r]
                else:
                    gr = torch.autograd.functional.jacobian(net, x, create_graph=True)
                    val = gr[t] - lap - prob.f[r]
            else:
                val = net(x) - prob.g[r]
            out.append(np.sqrt(prob.w[r]) * val)
        return torch.stack(out)

    Jt = torch.autograd.functional.jacobian(res_w, torch.tensor(theta)).numpy()
    np.testing.assert_allclose(mlp.jacobian(theta, prob), Jt, rtol=1e-10, atol=1e-12)


def test_manufactured_solutions_solve_their_pdes():
    """-Laplace u* = f (Poisson) and u*_t = Laplace u* (heat) for the workload data, by differences."""
    h = 1e-4
    for prob, u in [
        (wl.poisson_random(d=2, n_interior=20, n_boundary=8, seed=1), lambda X: np.prod(np.sin(np.pi * X), 1)),
        (wl.poisson_random(d=5, widths=(5, 4, 1), n_interior=20, n_boundary=8, seed=1, solution="sinsum"),
         lambda X: np.sum(np.sin(np.pi * X), 1)),
    ]:
        Xi = prob.X[prob.kind == wl.KIND_INTERIOR]
        lap = sum((u(Xi + h * e) - 2 * u(Xi) + u(Xi - h * e)) / h ** 2 for e in np.eye(prob.d))
        np.testing.assert_allclose(-lap, prob.f[prob.kind == wl.KIND_INTERIOR], rtol=1e-5, atol=1e-5)
        Xb = prob.X[prob.kind == wl.KIND_BOUNDARY]
        np.testing.assert_allclose(u(Xb), prob.g[prob.kind == wl.KIND_BOUNDARY], atol=1e-14)
    heat = wl.heat2d(widths=(3, 4, 1), n_interior=20, n_lateral=6, n_initial=6, seed=1)
    us = lambda X: np.exp(-2 * np.pi ** 2 * X[:, 2]) * np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1])
    Xi = heat.X[heat.kind == wl.KIND_INTERIOR]
    ex, ey, et = np.eye(3)
    ut = (us(Xi + h * et) - us(Xi - h * et)) / (2 * h)
    lap = sum((us(Xi + h * e) - 2 * us(Xi) + us(Xi - h * e)) / h ** 2 for e in (ex, ey))
    np.testing.assert_allclose(ut, lap, rtol=1e-5, atol=1e-5)
    X0 = heat.X[heat.kind == wl.KIND_INITIAL]
    np.testing.assert_allclose(us(X0), heat.g[heat.kind == wl.KIND_INITIAL], atol=1e-14)


def test_teacher_network_has_zero_residual():
    """Data generated by a network itself (f = -Laplace u_teacher by differences, g = u_teacher) gives
    a residual at the level of the difference error only."""
    import dataclasses
    prob = wl.small_problem(pde=wl.PDE_POISSON, d=2, widths=(2, 6, 6, 1), n_interior=10, n_boundary=6, seed=11)
    theta = wl.glorot_theta(prob.widths, 11)
    _, second = _fd_derivatives(theta, prob.widths, prob.X, prob.pde)
    u = mlp.taylor_forward(theta, prob.widths, prob.X, prob.pde)[0]
    inner = prob.kind == wl.KIND_INTERIOR
    teacher = dataclasses.replace(prob, f=np.where(inner, -second.sum(1), 0.0), g=np.where(inner, 0.0, u))
    assert np.max(np.abs(mlp.residual(theta, teacher))) < 1e-5
