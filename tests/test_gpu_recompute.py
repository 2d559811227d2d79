"""Recompute mode (J_w never stored): the forward-tangent (JVP) and adjoint (VJP) kernels, the
autograd.Function built on them, and every entry point driven by them, against the FP64 oracle's
explicit Jacobian and against the stored-Jacobian path (MI355X).

Tolerances (relative): 1e-10 in FP64, 1e-5 in FP32 (oracle on the FP32-rounded inputs); the JVP is
also checked against central differences of the library's own residuals (h = 1e-6, FP64)."""
import numpy as np
import pytest

import workloads as wl
from gpu_helpers import make, rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from oracle import linalg, mlp  # noqa: E402
from paper_2505_11638_amd.api import Problem, Recompute  # noqa: E402
from paper_2505_11638_amd.autograd import residual  # noqa: E402
from paper_2505_11638_amd.driver import NGD  # noqa: E402

TOL = {"f64": 1e-10, "f32": 1e-5}

CASES = {
    "poisson2d_f64": lambda: wl.small_problem(widths=(2, 32, 32, 1), n_interior=61, n_boundary=22, seed=11, ell=24,
                                              lam=1e-6),
    "heat_f64": lambda: wl.small_problem(pde=wl.PDE_HEAT, widths=(3, 24, 20, 16, 1), n_interior=45, n_boundary=18,
                                         seed=12, ell=20, lam=1e-6),
    "heat_f32": lambda: wl.small_problem(pde=wl.PDE_HEAT, widths=(3, 64, 64, 64, 64, 1), n_interior=150,
                                         n_boundary=41, seed=13, dtype="f32", ell=40, lam=1e-4),
    "poisson5d_f32": lambda: wl.small_problem(d=5, widths=(5, 48, 40, 1), n_interior=53, n_boundary=20, seed=14,
                                              dtype="f32", ell=32, lam=1e-4),
}


def _setup(name):
    prob, th = make(CASES[name]())
    gp = Problem(prob, dtype=prob.dtype, max_ell=prob.ell)
    J_o = mlp.jacobian(th, prob)
    return prob, th, gp, J_o


@pytest.mark.parametrize("name", list(CASES))
def test_jvp_vjp_match_oracle_jacobian(name):
    prob, th, gp, J_o = _setup(name)
    tol = TOL[prob.dtype]
    rng = np.random.default_rng(5)
    U = rng.standard_normal((3, gp.P))
    if prob.dtype == "f32":
        U = U.astype(np.float32).astype(np.float64)
    theta = gp.theta(th)
    Ut = torch.zeros((3, gp.ld), dtype=gp.tdtype, device="cuda")
    Ut[:, :gp.P] = torch.as_tensor(U, dtype=gp.tdtype)
    Y = gp.jvp(theta, Ut).cpu().numpy()
    for j in range(3):
        assert rel(Y[j], J_o @ U[j]) <= tol, j
    wv = rng.standard_normal(gp.N)
    if prob.dtype == "f32":
        wv = wv.astype(np.float32).astype(np.float64)
    g = gp.vjp(theta, torch.as_tensor(wv, dtype=gp.tdtype, device="cuda")).cpu().numpy()
    assert rel(g, J_o.T @ wv) <= tol
    gp.close()


@pytest.mark.parametrize("name", ["poisson2d_f64", "heat_f64"])
def test_jvp_central_differences(name):
    """J_w u against (r_w(theta + h u) - r_w(theta - h u)) / 2h from the library's residuals."""
    prob, th, gp, _ = _setup(name)
    u = np.random.default_rng(7).standard_normal(gp.P)
    h = 1e-6
    rp, _, _, _ = gp.residual_jacobian(gp.theta(th + h * u), None, want_grad=False, want_loss=False)
    rm, _, _, _ = gp.residual_jacobian(gp.theta(th - h * u), None, want_grad=False, want_loss=False)
    fd = (rp - rm).cpu().numpy() / (2 * h)
    jv = gp.jvp(gp.theta(th), torch.as_tensor(u, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert rel(jv, fd) <= 1e-7
    gp.close()


@pytest.mark.parametrize("name", ["poisson2d_f64", "heat_f64", "heat_f32"])
def test_autograd_function(name):
    prob, th, gp, J_o = _setup(name)
    tol = TOL[prob.dtype]
    theta = gp.theta(th).requires_grad_(True)
    r = residual(theta, gp)
    r_o = mlp.weighted_residual(th, prob)
    assert rel(r.detach().cpu().numpy(), r_o) <= tol
    # reverse mode: d(0.5 ||r||^2)/dtheta = J^T r
    loss = 0.5 * (r.double() ** 2).sum()
    (g,) = torch.autograd.grad(loss, theta)
    assert rel(g.cpu().numpy(), J_o.T @ r_o) <= max(tol, 1e-6 if prob.dtype == "f32" else tol)
    # forward mode: J u
    u = np.random.default_rng(3).standard_normal(gp.P)
    if prob.dtype == "f32":
        u = u.astype(np.float32).astype(np.float64)
    import torch.autograd.forward_ad as fwAD
    with fwAD.dual_level():
        dual = fwAD.make_dual(theta.detach(), torch.as_tensor(u, dtype=gp.tdtype, device="cuda"))
        out = residual(dual, gp)
        tangent = fwAD.unpack_dual(out).tangent
    assert rel(tangent.cpu().numpy(), J_o @ u) <= tol
    gp.close()


@pytest.mark.parametrize("name", list(CASES))
def test_recompute_entry_points_match_stored(name):
    """Gradient, damped matvec, plain CG and Nystrom sketch + PCG with J recomputed vs stored J_w."""
    prob, th, gp, J_o = _setup(name)
    tol = TOL[prob.dtype]
    theta = gp.theta(th)
    J = gp.new_jacobian()
    _, J, grad_s, loss_s = gp.residual_jacobian(theta, J)
    r_r, _, grad_r, loss_r = gp.residual_jacobian(theta, None)
    torch.cuda.synchronize()
    r_o = mlp.weighted_residual(th, prob)
    assert rel(grad_r.cpu().numpy(), J_o.T @ r_o) <= tol
    assert abs(loss_r.item() - loss_s.item()) <= tol * loss_s.item()
    op = Recompute(theta)
    lam = prob.lam
    v = torch.as_tensor(np.random.default_rng(9).standard_normal(gp.P), dtype=gp.tdtype, device="cuda")
    y_r = gp.gramian_matvec(op, v, lam).cpu().numpy().astype(np.float64)
    G_o = linalg.gramian(J_o)
    y_o = linalg.damped_matvec(G_o, v.cpu().numpy().astype(np.float64), lam)
    assert rel(y_r, y_o) <= tol * 10
    # plain CG converges as on the stored path; the error to the direct solve obeys the bound
    # ||d - d*|| <= ||g - (G + lam I) d|| / lam (lam is the smallest eigenvalue of G + lam I when N < P)
    g = grad_s
    rtol = 1e-8 if prob.dtype == "f64" else 1e-5
    out_s = gp.pcg_solve(J, g, lam, rtol=rtol, maxit=4 * gp.P)
    out_r = gp.pcg_solve(op, g, lam, rtol=rtol, maxit=4 * gp.P)
    assert out_s.converged and out_r.converged
    gn = g.cpu().numpy()
    d_star = linalg.solve_cholesky(G_o, gn, lam)
    d_r = out_r.d.cpu().numpy()
    res = linalg.true_relative_residual(G_o, lam, gn, d_r)
    assert res <= 10 * rtol
    assert np.linalg.norm(d_r - d_star) <= 1.01 * res * np.linalg.norm(gn) / lam + 1e-12 * np.linalg.norm(d_star)
    # Nystrom sketch with the same Omega: eigenvalues agree with the stored path
    omega = gp.gaussian_omega(seed=3, counter=1, ell=prob.ell)
    pc_s = gp.nystrom_sketch(J, prob.ell, omega=omega)
    pc_r = gp.nystrom_sketch(op, prob.ell, omega=omega)
    lam_s, lam_r = pc_s.lam_hat.cpu().numpy(), pc_r.lam_hat.cpu().numpy()
    top = lam_s >= 1e-6 * lam_s[0]
    assert np.max(np.abs(lam_r[top] - lam_s[top])) <= (1e-4 if prob.dtype == "f32" else 1e-9) * lam_s[0]
    out_p = gp.pcg_solve(op, g, lam, precond=pc_r, rtol=rtol, maxit=1000)
    assert out_p.converged and out_p.iters <= out_r.iters
    gp.close()


def test_ngd_step_recompute_matches_stored():
    prob, th = make(wl.small_problem(pde=wl.PDE_HEAT, widths=(3, 32, 32, 1), n_interior=120, n_boundary=40,
                                     seed=21, dtype="f32", ell=30, lam=None))
    a = NGD(prob, th, solver="nystrom", recompute=False, seed=1)
    b = NGD(prob, th, solver="nystrom", recompute=True, seed=1)
    for _ in range(2):
        ra, rb = a.step(), b.step()
        assert rb.converged
        assert abs(ra.loss - rb.loss) <= 1e-4 * ra.loss
        assert rb.loss_new <= rb.loss
    a.gp.close()
    b.gp.close()
