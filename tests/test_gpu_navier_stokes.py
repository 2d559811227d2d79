"""The Navier-Stokes rows (the Kovasznay flow of Section 5.1.3) on the GPU against the FP64 oracle (MI355X).

Tolerances (relative): 1e-10 in FP64, 1e-5 in FP32 (the Jacobian row by row); FP32 results are compared
with the oracle on the FP32-rounded inputs. Row counts are ragged against the kernel's rounds of one row
per wave; the paper's size (32,000 rows, P = 8,688, FP64) is checked on sampled rows."""
import numpy as np
import pytest

import workloads as wl
from gpu_helpers import rel, rounded_theta, rowwise_rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from oracle import navier_stokes as ns  # noqa: E402
from oracle import ngd as ongd  # noqa: E402
from paper_2505_11638_amd import _lib as L  # noqa: E402
from paper_2505_11638_amd.api import Batch, Problem  # noqa: E402
from paper_2505_11638_amd.driver import NGD  # noqa: E402

TOL = {"f64": 1e-10, "f32": 1e-5}

CASES = {
    "small_f64": dict(dtype="f64", widths=(2, 24, 20, 2), n_interior=37, n_boundary=13, seed=3),
    "small_f32": dict(dtype="f32", widths=(2, 24, 20, 2), n_interior=37, n_boundary=13, seed=4),
    "paper_nets_f64": dict(dtype="f64", widths=(2, 45, 45, 45, 2), n_interior=613, n_boundary=101, seed=5),
    "paper_nets_f32": dict(dtype="f32", widths=(2, 45, 45, 45, 2), n_interior=613, n_boundary=101, seed=6),
    "wide_deep_f64": dict(dtype="f64", widths=(2, 64, 33, 17, 64, 2), n_interior=29, n_boundary=7, seed=7),
}


def _make(dtype, widths, n_interior, n_boundary, seed):
    prob = wl.kovasznay(widths=widths, n_interior=n_interior, n_boundary=n_boundary, seed=seed, dtype=dtype, ell=24)
    th = wl.ns_glorot_theta(widths, seed)
    th = th + 0.05 * np.random.default_rng(seed + 1).standard_normal(th.size)  # nonzero biases
    return prob.cast(dtype), rounded_theta(th, dtype)


@pytest.mark.parametrize("name", list(CASES))
def test_ns_residual_jacobian_gradient_loss(name):
    print(f"navier-stokes residual/Jacobian case {name}", flush=True)
    prob, th = _make(**CASES[name])
    tol = TOL[prob.dtype]
    gp = Problem(prob, dtype=prob.dtype, max_ell=prob.ell)
    assert gp.P == wl.ns_num_params(prob.widths)
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r, J, grad, loss = gp.residual_jacobian(theta, J)
    torch.cuda.synchronize()
    r_o, J_o = ns.residual_and_jacobian(th, prob)
    Jg = J.cpu().numpy().astype(np.float64)
    assert rel(r.cpu().numpy(), r_o) <= tol
    assert rowwise_rel(Jg[:, :gp.P], J_o) <= tol
    assert np.all(Jg[:, gp.P:] == 0)
    # the pressure network's columns are exactly zero on the continuity and boundary rows
    quiet = (prob.kind != wl.KIND_NS_MOMENTUM_X) & (prob.kind != wl.KIND_NS_MOMENTUM_Y)
    assert np.all(Jg[quiet, wl.num_params(prob.widths):gp.P] == 0)
    assert rel(grad.cpu().numpy(), J_o.T @ r_o) <= tol
    assert abs(loss.item() - 0.5 * r_o @ r_o) <= tol * 0.5 * (r_o @ r_o)
    # forward-only call: the same residuals and, summed in the same groups, the same loss
    r2, _, _, loss2 = gp.residual_jacobian(theta, None, want_grad=False)
    torch.cuda.synchronize()
    assert torch.equal(r2, r) and loss2.item() == loss.item()


def test_ns_paper_size_sampled_rows():
    """The paper's Kovasznay setup (10,000 + 1,000 points, 32,000 rows, P = 8,688, FP64) in the launch
    configuration the benchmark uses: every residual and the loss against the oracle, the Jacobian on
    sampled rows of every kind (first and last rows included)."""
    prob = wl.config("paper_ns")
    print("navier-stokes paper size, N =", prob.n_rows, flush=True)
    th = wl.ns_glorot_theta(prob.widths, 0)
    gp = Problem(prob, dtype="f64", max_ell=20)
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r, J, grad, loss = gp.residual_jacobian(theta, J)
    torch.cuda.synchronize()
    r_o = ns.weighted_residual(th, prob)
    assert rel(r.cpu().numpy(), r_o) <= 1e-10
    assert abs(loss.item() - 0.5 * r_o @ r_o) <= 1e-10 * 0.5 * (r_o @ r_o)
    rng = np.random.default_rng(11)
    rows = [0, prob.n_rows - 1] + [int(np.nonzero(prob.kind == k)[0][0]) for k in range(3, 8)]
    rows = np.unique(np.concatenate([rows, rng.choice(prob.n_rows, 48, replace=False)]))
    J_o = ns.jacobian(th, prob, rows)
    Jg = J[torch.as_tensor(rows, device=J.device)].cpu().numpy()
    assert rowwise_rel(Jg[:, :gp.P], J_o) <= 1e-10
    assert np.all(Jg[:, gp.P:] == 0)
    # the gradient through J_w^T r_w on the GPU's own J, against FP64 on the host
    Jh = J.cpu().numpy()[:, :gp.P]
    assert rel(grad.cpu().numpy(), Jh.T @ r.cpu().numpy()) <= 1e-12
    del J, Jh
    gp.close()


def test_ns_line_search_and_lm_damping():
    """Armijo on the Navier-Stokes loss (the same alpha as the oracle's backtracking) and the
    Levenberg-Marquardt update of mu (Section 5.1.3) against the oracle's gain ratio and rule."""
    prob, th = _make(**CASES["small_f64"])
    gp = Problem(prob, dtype="f64", max_ell=prob.ell)
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r, J, grad, loss = gp.residual_jacobian(theta, J)
    torch.cuda.synchronize()
    r_o, J_o = ns.residual_and_jacobian(th, prob)
    g = J_o.T @ r_o
    L0 = 0.5 * float(r_o @ r_o)
    G = J_o.T @ J_o
    for mu in (1e-2, 1e-6):
        d = np.linalg.solve(G + mu * np.eye(G.shape[0]), g)
        a_o, L1_o = ongd.armijo(lambda t: ns.loss(t, prob), th, d, g, L0)
        dd = torch.as_tensor(d, device=theta.device)
        gg = torch.as_tensor(g, device=theta.device)
        tout = torch.empty_like(theta)
        _, alpha, L1 = gp.line_search(theta, dd, gg, L0, theta_out=tout)
        assert alpha == a_o
        assert abs(L1 - L1_o) <= 1e-10 * L0
        mu_next, rho = gp.lm_damping(J, dd, gg, alpha, L0, L1, mu, 1e-14)
        rho_o = ongd.gain_ratio(L0, L1_o, a_o, float(g @ d), float(d @ G @ d))
        assert abs(rho - rho_o) <= 1e-8 * max(1.0, abs(rho_o))
        assert mu_next == ongd.lm_update(mu, rho_o, 1e-14)


def test_ns_ngd_steps():
    """NGD with the Nystrom preconditioner and Levenberg-Marquardt damping on a small Kovasznay problem:
    each PCG direction within its residual bound of the direct solve on the oracle's Gramian, the loss
    never rises and falls overall, mu follows the oracle's rule."""
    prob, th = _make(**CASES["small_f64"])
    ngd = NGD(prob, th, solver="nystrom", rtol=1e-10, ell=20, ell_max=40, seed=2)
    assert ngd.damping == "lm"
    theta = th.copy()
    losses = []
    mu_prev_next = None
    for k in range(6):
        rep = ngd.step()
        r_o, J_o = ns.residual_and_jacobian(theta, prob)
        g = J_o.T @ r_o
        G = J_o.T @ J_o
        assert abs(rep.loss - 0.5 * r_o @ r_o) <= 1e-10 * rep.loss
        if mu_prev_next is not None:
            assert rep.mu == mu_prev_next
        d_star = np.linalg.solve(G + rep.mu * np.eye(G.shape[0]), g)
        d = ngd.d.cpu().numpy()
        bound = rep.rel_res * np.linalg.norm(g) / rep.mu
        assert np.linalg.norm(d - d_star) <= 1.01 * bound + 1e-9 * np.linalg.norm(d_star)
        rho_o = ongd.gain_ratio(rep.loss, rep.loss_new, rep.alpha, float(g @ d), float(d @ G @ d))
        mu_prev_next = ongd.lm_update(rep.mu, rho_o, ngd.gamma * ngd.eps * rep.lam1) if abs(rho_o - 0.25) > 1e-6 \
            and abs(rho_o - 0.75) > 1e-6 else None
        assert rep.loss_new <= rep.loss
        losses.append(rep.loss)
        theta = theta - rep.alpha * d
        np.testing.assert_allclose(ngd.theta.cpu().numpy(), theta, rtol=0, atol=1e-12 * np.max(np.abs(theta)))
        theta = ngd.theta.cpu().numpy()
    assert losses[-1] < 0.5 * losses[0]


def test_ns_velocity_error():
    prob, th = _make(**CASES["paper_nets_f64"])
    gp = Problem(prob, dtype="f64", max_ell=prob.ell)
    Xe, ue, ge = wl.kovasznay_evaluation_set(prob.nu, 3001, seed=1)
    l2, h1, sums = gp.solution_error(gp.theta(th), Xe, ue, ge)
    s_o = ns.velocity_error_sums(th, prob.widths, Xe, ue, ge)
    assert rel(sums.cpu().numpy(), s_o) <= 1e-12
    assert abs(h1 - np.sqrt((s_o[0] + s_o[1]) / (s_o[2] + s_o[3]))) <= 1e-10
    _, _, sums0 = gp.solution_error(gp.theta(th), Xe[:0], ue[:0], ge[:0])
    assert np.all(sums0.cpu().numpy() == 0)


def test_ns_refuses_the_recompute_mode_and_batches():
    prob, th = _make(**CASES["small_f64"])
    gp = Problem(prob, dtype="f64", max_ell=prob.ell)
    theta = gp.theta(th)
    with pytest.raises(L.NgdError, match="Navier-Stokes"):
        gp.jvp(theta, theta)
    with pytest.raises(L.NgdError, match="Navier-Stokes"):
        gp.residual_jacobian(theta, None, want_grad=True)
    with pytest.raises(L.NgdError):
        Batch([prob])
    # the handle keeps working
    J = gp.new_jacobian()
    r, _, _, _ = gp.residual_jacobian(theta, J)
    torch.cuda.synchronize()
    assert rel(r.cpu().numpy(), ns.weighted_residual(th, prob)) <= 1e-10


@pytest.mark.parametrize("variant", ["rpchol", "sampling"])
def test_ns_rpchol_and_sampling_ngd_steps(variant):
    """The paper's other preconditioners on the Navier-Stokes rows (Section 5.1.3 runs both): RPCholNGD with
    the Woodbury-Cholesky preconditioner and Nystrom NGD with a sampling test matrix, Levenberg-Marquardt
    damping; every PCG direction within the residual bound of the direct solve on the oracle's Gramian and
    the loss falling."""
    prob, th = _make(**CASES["small_f64"])
    if variant == "rpchol":
        ngd = NGD(prob, th, solver="rpchol", rtol=1e-10, ell_max=40, seed=4)
    else:
        ngd = NGD(prob, th, solver="nystrom", test_matrix="sampling", rtol=1e-10, ell=30, ell_max=60, seed=4)
    theta = th.copy()
    losses = []
    for k in range(5):
        rep = ngd.step()
        r_o, J_o = ns.residual_and_jacobian(theta, prob)
        g = J_o.T @ r_o
        G = J_o.T @ J_o
        d_star = np.linalg.solve(G + rep.mu * np.eye(G.shape[0]), g)
        d = ngd.d.cpu().numpy()
        bound = max(rep.rel_res, 1e-10) * np.linalg.norm(g) / rep.mu
        assert np.linalg.norm(d - d_star) <= 1.01 * bound + 1e-9 * np.linalg.norm(d_star)
        assert rep.loss_new <= rep.loss
        losses.append(rep.loss)
        theta = ngd.theta.cpu().numpy()
    assert losses[-1] < 0.5 * losses[0]
