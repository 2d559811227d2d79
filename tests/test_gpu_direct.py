"""NGD with the full Gramian (Alg. 2) on the GPU against the oracle's Cholesky solve, through the C ABI
(MI355X): small problems in FP64 and FP32 (stored and recompute mode), the 2D FP64 workload in full
and the benchmark's FP32 workload (P = 8,577: 68 panels of the blocked factorisation, a ragged last one).

FP32 problems are compared with the oracle run on the GPU's own FP32 Jacobian promoted to FP64 (the
Gramian is formed in FP64 on both sides). The solution is checked through the bound
||d - d*|| <= ||g - (G + lambda I) d|| / lambda (lambda_min(G + lambda I) >= lambda) and against d*."""
import numpy as np
import pytest

import workloads as wl
from gpu_helpers import make

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from oracle import linalg, mlp  # noqa: E402
from paper_2505_11638_amd.api import Problem, Recompute  # noqa: E402

SMALL = {
    "poisson2d_f64": lambda: wl.small_problem(widths=(2, 32, 32, 1), n_interior=61, n_boundary=22, seed=1, lam=1e-6),
    "poisson2d_f32": lambda: wl.small_problem(widths=(2, 64, 64, 64, 1), n_interior=97, n_boundary=30, seed=2,
                                              dtype="f32", lam=1e-4),
    "heat_f64": lambda: wl.small_problem(pde=wl.PDE_HEAT, widths=(3, 24, 20, 16, 1), n_interior=45, n_boundary=18,
                                         seed=4, lam=1e-6),
}


def _check(G, g, lam, d, tol):
    d_star = linalg.solve_cholesky(G, g, lam)
    res = linalg.true_relative_residual(G, lam, g, d)
    err = np.linalg.norm(d - d_star) / np.linalg.norm(d_star)
    print(f"  true relative residual {res:.2e}, ||d - d*|| / ||d*|| = {err:.2e}", flush=True)
    assert res <= tol
    assert np.linalg.norm(d - d_star) <= 1.01 * res * np.linalg.norm(g) / lam + tol * np.linalg.norm(d_star)
    return err


@pytest.mark.parametrize("name", list(SMALL))
def test_direct_solve_small(name):
    prob, th = make(SMALL[name]())
    gp = Problem(prob, dtype=prob.dtype, max_ell=8)
    theta = gp.theta(th)
    J = gp.new_jacobian()
    _, J, grad, _ = gp.residual_jacobian(theta, J)
    print(f"direct solve {name}: N={gp.N} P={gp.P}", flush=True)
    d = gp.direct_solve(J, grad, prob.lam).cpu().numpy()
    Jg = J.cpu().numpy().astype(np.float64)[:, :gp.P]
    G = linalg.gramian(Jg)
    g = grad.cpu().numpy()
    _check(G, g, prob.lam, d, 1e-8)
    if prob.dtype == "f64":  # the oracle's own Jacobian as well (it differs from the GPU's at rounding level)
        _check(linalg.gramian(mlp.jacobian(th, prob)), g, prob.lam, d, 1e-7)
    # recompute mode: the Gramian summed over row blocks of J_w formed from theta
    dr = gp.direct_solve(Recompute(theta), grad, prob.lam).cpu().numpy()
    _check(G, g, prob.lam, dr, 1e-8)
    # the output may alias the right-hand side
    g2 = grad.clone()
    gp.direct_solve(J, g2, prob.lam, out=g2)
    assert np.array_equal(g2.cpu().numpy(), d)
    gp.close()


@pytest.mark.parametrize("cfg, lam", [("c1", 1e-6), ("c2", 1e-4)])
def test_direct_solve_full_size(cfg, lam):
    prob = wl.config(cfg)
    theta = wl.glorot_theta(prob.widths, 0)
    p64 = prob.cast(prob.dtype)
    gp = Problem(p64, dtype=prob.dtype, max_ell=8)
    th = gp.theta(theta)
    J = gp.new_jacobian()
    _, J, grad, _ = gp.residual_jacobian(th, J)
    print(f"direct solve {cfg}: N={gp.N} P={gp.P} lambda={lam}", flush=True)
    d = gp.direct_solve(J, grad, lam).cpu().numpy()
    Jg = J.cpu().numpy().astype(np.float64)[:, :gp.P]
    _check(linalg.gramian(Jg), grad.cpu().numpy(), lam, d, 1e-8)
    gp.close()


def test_direct_solve_refuses_bad_arguments():
    prob, th = make(SMALL["poisson2d_f64"]())
    gp = Problem(prob, dtype="f64", max_ell=8)
    J = gp.new_jacobian()
    _, J, grad, _ = gp.residual_jacobian(gp.theta(th), J)
    from paper_2505_11638_amd._lib import NgdError
    for lam in (0.0, -1.0, float("nan")):
        with pytest.raises(NgdError):
            gp.direct_solve(J, grad, lam)
    d = gp.direct_solve(J, grad, 1e-3)  # the handle keeps working
    assert torch.isfinite(d).all()
    gp.close()
