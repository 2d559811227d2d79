"""Parity of every libngd entry point with the FP64 oracle on the same seeded inputs (MI355X).

Tolerances (relative): 1e-10 in FP64, 1e-5 in FP32, 2e-2 for BF16 sketches; FP32 results are
compared with the oracle run on the FP32-rounded inputs."""
import numpy as np
import pytest

import workloads as wl
from gpu_helpers import make, rel, rowwise_rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from oracle import cg, linalg, mlp, ngd, nystrom, philox  # noqa: E402
from paper_2505_11638_amd.api import Problem  # noqa: E402

TOL = {"f64": 1e-10, "f32": 1e-5}

# (name, problem factory) -- ragged row counts (not multiples of the residual tile)
SMALL = {
    "poisson2d_f64": lambda: wl.small_problem(widths=(2, 32, 32, 1), n_interior=61, n_boundary=22, seed=1, ell=24,
                                              lam=1e-6),
    "poisson2d_f32": lambda: wl.small_problem(widths=(2, 64, 64, 64, 1), n_interior=97, n_boundary=30, seed=2,
                                              dtype="f32", ell=40, lam=1e-4),
    "poisson5d_f32": lambda: wl.small_problem(d=5, widths=(5, 48, 40, 1), n_interior=53, n_boundary=20, seed=3,
                                              dtype="f32", ell=32, lam=1e-4),
    "heat_f64": lambda: wl.small_problem(pde=wl.PDE_HEAT, widths=(3, 24, 20, 16, 1), n_interior=45, n_boundary=18,
                                         seed=4, ell=20, lam=1e-6),
    "heat_f32": lambda: wl.small_problem(pde=wl.PDE_HEAT, widths=(3, 64, 64, 1), n_interior=70, n_boundary=26,
                                         seed=5, dtype="f32", ell=30, lam=1e-4),
}


def _setup(name):
    prob64, th = make(SMALL[name]())
    gp = Problem(prob64, dtype=prob64.dtype, max_ell=prob64.ell)
    return prob64, th, gp


@pytest.mark.parametrize("name", list(SMALL))
def test_residual_jacobian_gradient_loss(name):
    prob, th, gp = _setup(name)
    tol = TOL[prob.dtype]
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r, J, grad, loss = gp.residual_jacobian(theta, J)
    torch.cuda.synchronize()
    r_o, J_o = mlp.residual_and_jacobian(th, prob)
    Jg = J.cpu().numpy().astype(np.float64)
    assert rel(r.cpu().numpy(), r_o) <= tol
    assert rowwise_rel(Jg[:, :gp.P], J_o) <= tol
    assert np.all(Jg[:, gp.P:] == 0)
    assert rel(grad.cpu().numpy(), J_o.T @ r_o) <= tol
    assert abs(loss.item() - 0.5 * r_o @ r_o) <= tol * 0.5 * (r_o @ r_o)
    # forward-only call: same residuals
    r2, _, _, loss2 = gp.residual_jacobian(theta, None, want_grad=False)
    torch.cuda.synchronize()
    assert torch.equal(r2, r) and loss2.item() == loss.item()


@pytest.mark.parametrize("name", ["poisson2d_f64", "poisson2d_f32", "heat_f32"])
def test_gramian_matvec_single_and_block(name):
    prob, th, gp = _setup(name)
    tol = TOL[prob.dtype]
    theta = gp.theta(th)
    J = gp.new_jacobian()
    gp.residual_jacobian(theta, J)
    Jg = J.cpu().numpy().astype(np.float64)[:, :gp.P]
    G = Jg.T @ Jg  # operator of the GPU's own (rounded) Jacobian
    rng = np.random.default_rng(7)
    lam = 1e-3
    v = rng.standard_normal(gp.P)
    y = gp.gramian_matvec(J, gp.theta(v), lam).cpu().numpy()
    vr = v.astype(np.float32).astype(np.float64) if prob.dtype == "f32" else v
    ref = G @ vr + lam * vr
    scale = np.linalg.norm(G, 2) * np.linalg.norm(vr)
    assert np.linalg.norm(y - ref) <= tol * scale
    k = 7
    V = np.zeros((k, gp.ld))
    V[:, :gp.P] = rng.standard_normal((k, gp.P))
    Y = gp.gramian_matvec(J, gp.theta(V), lam).cpu().numpy()[:, :gp.P]
    Vr = V[:, :gp.P].astype(np.float32).astype(np.float64) if prob.dtype == "f32" else V[:, :gp.P]
    refY = (G @ Vr.T + lam * Vr.T).T
    assert np.linalg.norm(Y - refY) <= tol * np.linalg.norm(G, 2) * np.linalg.norm(Vr) * 10


def test_gaussian_omega_matches_philox_oracle():
    prob, th, gp = _setup("poisson2d_f64")
    Om = gp.gaussian_omega(seed=1234567890123, counter=17, ell=9).cpu().numpy()
    ref = philox.gaussian_omega(gp.P, 9, seed=1234567890123, counter=17)
    np.testing.assert_allclose(Om[:, :gp.P], ref.T, rtol=1e-13, atol=1e-13)


def _nystrom_compare(prob, th, gp, sketch_dtype=None, tol=None):
    tol = tol or TOL[prob.dtype]
    theta = gp.theta(th)
    J = gp.new_jacobian()
    gp.residual_jacobian(theta, J)
    Jg = J.cpu().numpy().astype(np.float64)[:, :gp.P]
    ell = prob.ell
    Om = wl.gaussian_omega(gp.P, ell, seed=11)
    om_dev = torch.zeros((ell, gp.ld), dtype=gp.tdtype, device="cuda")
    om_dev[:, :gp.P] = torch.as_tensor(Om.T, dtype=gp.tdtype)
    res = gp.nystrom_sketch(J, ell, omega=om_dev, sketch_dtype=sketch_dtype)
    U = res.U.cpu().numpy().astype(np.float64)[:, :gp.P]
    lam = res.lam_hat.cpu().numpy()
    Omr = om_dev.cpu().numpy().astype(np.float64)[:, :gp.P].T
    Uo, lo, _ = nystrom.nystrom_alg6(lambda V: Jg.T @ (Jg @ V), Omr)
    assert np.all(np.diff(lam) <= 0) and np.all(lam >= 0)
    assert np.max(np.abs(lam - lo)) <= tol * lo[0]
    keep = lam > 0
    Uk = U[keep]
    # orthonormality: exact to the working precision on the well-separated top of the spectrum, and
    # within eps * sqrt(lam_1 / lam_i)-type errors near the drop threshold (cross-product SVD)
    top = lam >= 1e-6 * lam[0]
    assert np.max(np.abs(U[top] @ U[top].T - np.eye(top.sum()))) <= max(tol, 1e-10) * 100
    assert np.max(np.abs(Uk @ Uk.T - np.eye(keep.sum()))) <= max(tol, 1e-6)
    X = wl.probe_vectors(gp.P, 5, seed=3)
    Gg = Uk.T @ (lam[keep][:, None] * (Uk @ X))
    Go = Uo @ (lo[:, None] * (Uo.T @ X))
    assert np.linalg.norm(Gg - Go) <= tol * lo[0] * np.linalg.norm(X)
    return res, J, Jg


@pytest.mark.parametrize("name", ["poisson2d_f64", "heat_f64", "poisson2d_f32", "heat_f32"])
def test_nystrom_sketch_matches_alg6(name):
    prob, th, gp = _setup(name)
    _nystrom_compare(prob, th, gp)


@pytest.mark.parametrize("ell", [1, 2, 3, 5])
def test_nystrom_sketch_small_ell(ell):
    prob, th, gp = _setup("poisson2d_f64")
    import dataclasses
    _nystrom_compare(dataclasses.replace(prob, ell=ell), th, gp)


def test_nystrom_exact_when_rank_below_ell():
    """N = 14 rows < ell = 24: the sketch captures range(G) and G_nys = G (eq. nystrom_approx)."""
    prob, th = make(wl.small_problem(widths=(2, 16, 16, 1), n_interior=9, n_boundary=5, seed=8, ell=24, lam=1e-6))
    gp = Problem(prob, dtype="f64", max_ell=24)
    theta = gp.theta(th)
    J = gp.new_jacobian()
    gp.residual_jacobian(theta, J)
    Jg = J.cpu().numpy()[:, :gp.P]
    G = Jg.T @ Jg
    res = gp.nystrom_sketch(J, 24, seed=3)
    U = res.U.cpu().numpy()[:, :gp.P]
    lam = res.lam_hat.cpu().numpy()
    assert np.linalg.norm(U.T @ (lam[:, None] * U) - G) <= 1e-10 * np.linalg.norm(G)
    assert res.info["rank"] <= 14 and res.info["rank_z"] <= 14
    ev = np.sort(np.linalg.eigvalsh(G))[::-1]
    np.testing.assert_allclose(lam[:14], ev[:14], rtol=0, atol=1e-10 * ev[0])


def test_nystrom_sketch_bf16_before_refinement():
    prob, th, gp = _setup("poisson2d_f32")
    _nystrom_compare(prob, th, gp, sketch_dtype="bf16", tol=2e-2)


@pytest.mark.parametrize("name", ["poisson2d_f64", "poisson2d_f32", "heat_f32"])
@pytest.mark.parametrize("precond", [True, False])
def test_pcg_solve_matches_direct_solve(name, precond):
    prob, th, gp = _setup(name)
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r, J, grad, loss = gp.residual_jacobian(theta, J)
    Jg = J.cpu().numpy().astype(np.float64)[:, :gp.P]
    g = grad.cpu().numpy()
    lam = prob.lam
    rtol = 1e-8 if prob.dtype == "f64" else 1e-6
    pc = gp.nystrom_sketch(J, prob.ell, seed=5) if precond else None
    out = gp.pcg_solve(J, grad, lam, precond=pc, rtol=rtol, maxit=20 * gp.P)
    assert out.converged and not out.breakdown
    d = out.d.cpu().numpy()
    G = Jg.T @ Jg
    true_res = np.linalg.norm(g - G @ d - lam * d)
    assert true_res <= 10 * rtol * np.linalg.norm(g)
    dstar = linalg.solve_cholesky(G, g, lam)
    assert np.linalg.norm(d - dstar) <= true_res / lam * (1 + 1e-6) + 1e-12 * np.linalg.norm(dstar)
    # same recurrence in the oracle: iteration counts agree closely
    if precond:
        U = pc.U.cpu().numpy().astype(np.float64)[:, :gp.P].T
        lh = pc.lam_hat.cpu().numpy()
        M = lambda v: nystrom.precond_apply(U, lh, lam, v)
    else:
        M = None
    ref = cg.pcg(lambda v: Jg.T @ (Jg @ v) + lam * v, g, rtol, 20 * gp.P, M)
    assert ref.converged
    if precond:
        # well-conditioned preconditioned system: the counts of the two recurrences agree closely
        assert abs(out.iters - ref.iters) <= max(3, 0.25 * ref.iters)
    else:
        # plain CG on an ill-conditioned system: counts depend on rounding (FP32 matvec vs FP64)
        assert out.iters <= 3 * ref.iters + 10


@pytest.mark.parametrize("name", ["poisson2d_f64", "poisson2d_f32"])
def test_pcg_solve_damped_matches_host_damping(name):
    """The damping rule of Section 4.3 taken on the device (after a sketch that returns no summary)
    gives the lambda the host rule gives from the same lambda_hat_1 and loss, and then the same solve
    bit for bit; the rule's two branches are both exercised."""
    prob, th, gp = _setup(name)
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r, J, grad, loss = gp.residual_jacobian(theta, J)
    pc = gp.nystrom_sketch(J, prob.ell, seed=5, want_info=False)
    lam1 = float(pc.lam_hat[0].item())
    L0 = float(loss.item())
    for c_lam, c_loss in [(1e-3, 1e-4), (1e-12, 1.0)]:
        mu = max(c_lam * lam1, c_loss * (L0 * L0))
        ref = gp.pcg_solve(J, grad, mu, precond=pc, rtol=1e-6, maxit=1000)
        out = gp.pcg_solve(J, grad, None, precond=pc, rtol=1e-6, maxit=1000, damping=(c_lam, c_loss, loss))
        assert out.mu == mu
        assert out.iters == ref.iters and out.converged == ref.converged
        assert torch.equal(out.d, ref.d)
    with pytest.raises(ValueError):
        gp.pcg_solve(J, grad, None, precond=None, damping=(1e-3, 1e-4, loss))


def test_pcg_edge_cases():
    prob, th, gp = _setup("poisson2d_f64")
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r, J, grad, loss = gp.residual_jacobian(theta, J)
    zero = torch.zeros_like(grad)
    out = gp.pcg_solve(J, zero, 1e-3)
    assert out.converged and out.iters == 0 and not out.d.any()
    out = gp.pcg_solve(J, grad, 1e-3, rtol=1e-14, maxit=3)
    assert not out.converged and out.iters == 3
    out = gp.pcg_solve(J, grad, 1e-3, maxit=0)
    assert not out.converged and out.iters == 0


def test_power_method_matches_oracle():
    prob, th, gp = _setup("poisson2d_f64")
    theta = gp.theta(th)
    J = gp.new_jacobian()
    gp.residual_jacobian(theta, J)
    Jg = J.cpu().numpy()[:, :gp.P]
    v0 = np.random.default_rng(2).standard_normal(gp.P)
    lam = gp.power_lambda_max(J, torch.as_tensor(v0, device="cuda"), 4)
    ref = ngd.power_method(lambda v: Jg.T @ (Jg @ v), v0, 4)
    assert abs(lam - ref) <= 1e-10 * ref


@pytest.mark.parametrize("name", ["poisson2d_f64", "poisson2d_f32"])
def test_line_search_matches_oracle(name):
    prob, th, gp = _setup(name)
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r, J, grad, loss = gp.residual_jacobian(theta, J)
    out = gp.pcg_solve(J, grad, prob.lam, rtol=1e-8, maxit=20 * gp.P)
    for scale in (1.0, 40.0):   # the second direction overshoots: several halvings
        d = out.d * scale
        th_new, alpha, lnew = gp.line_search(theta, d, grad, loss.item())
        a_ref, l_ref = ngd.armijo(lambda t: mlp.loss(t, prob), th, d.cpu().numpy(), grad.cpu().numpy(), loss.item())
        assert alpha == a_ref
        assert abs(lnew - l_ref) <= TOL[prob.dtype] * max(l_ref, 1e-30) * 10
        exp = th - alpha * d.cpu().numpy()
        assert rel(th_new.cpu().numpy(), exp) <= (1e-15 if prob.dtype == "f64" else 1e-7)
