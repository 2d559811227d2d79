"""Parity at the benchmark's full sizes, in the launch configurations bench.py times (MI355X).

The oracle computes what it can at these sizes (sampled Jacobian rows, all residuals, the Alg. 6 sketch and
solves in FP64 on the GPU's own FP32-rounded Jacobian for the 2D workload); elsewhere results are checked
against FP64 products with the GPU's own Jacobian and against properties that hold at any size.
"""
import numpy as np
import pytest

import workloads as wl
from gpu_helpers import rel, rowwise_rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from oracle import linalg, mlp, nystrom  # noqa: E402
from paper_2505_11638_amd.api import Problem, Recompute  # noqa: E402
from paper_2505_11638_amd.driver import EPS  # noqa: E402

U32 = 2.0 ** -24


def _setup(cfg):
    prob = wl.config(cfg)
    theta = wl.glorot_theta(prob.widths, 0)
    theta = theta + 0.05 * np.random.default_rng(1).standard_normal(theta.size)
    p64 = prob.cast(prob.dtype)
    th = theta.astype(np.float32).astype(np.float64) if prob.dtype == "f32" else theta
    gp = Problem(p64, dtype=prob.dtype, max_ell=prob.ell)
    return p64, th, gp


def _sample_rows(prob, n=12, seed=0):
    """Rows spread over the point set, including boundary (and initial) rows."""
    rng = np.random.default_rng(seed)
    interior = np.flatnonzero(prob.kind == wl.KIND_INTERIOR)
    other = np.flatnonzero(prob.kind != wl.KIND_INTERIOR)
    rows = np.concatenate([rng.choice(interior, n - n // 3, replace=False), rng.choice(other, n // 3, replace=False),
                           [0, prob.n_rows - 1]])
    return np.unique(rows)


def _jt_mul(J32, v, chunk=2048):
    """FP64 J^T (J v) with J the GPU's FP32 Jacobian (host copy), in row chunks."""
    out = np.zeros(J32.shape[1])
    for s in range(0, J32.shape[0], chunk):
        Jc = J32[s:s + chunk].astype(np.float64)
        out += Jc.T @ (Jc @ v)
    return out


def _abs_mul(J32, d, chunk=2048):
    """|| |J|^T (|J| |d|) ||: the scale of the rounding error of an FP32 product J^T J d."""
    out = np.zeros(J32.shape[1])
    for s in range(0, J32.shape[0], chunk):
        Jc = np.abs(J32[s:s + chunk].astype(np.float64))
        out += Jc.T @ (Jc @ np.abs(d))
    return float(np.linalg.norm(out))


def _check_solve(J32, g, d, mu, rtol):
    """True residual of the solve on the GPU's FP32 Jacobian promoted to FP64, against the PCG tolerance
    plus the rounding bound of the FP32 operator the solver applies (a sqrt(P) * u dot-product bound)."""
    res = np.linalg.norm(g - _jt_mul(J32, d) - mu * d) / np.linalg.norm(g)
    bound = 10 * rtol + np.sqrt(J32.shape[1]) * U32 * _abs_mul(J32, d) / np.linalg.norm(g)
    assert res <= bound, (res, bound)


def test_c1_full_fp64():
    """The 2D FP64 workload in full: J, gradient, Alg. 6 sketch and PCG at rtol 1e-8 against the oracle."""
    prob, th, gp = _setup("c1")
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r, J, grad, loss = gp.residual_jacobian(theta, J)
    r_o, J_o = mlp.residual_and_jacobian(th, prob)
    Jg = J.cpu().numpy()[:, :gp.P]
    assert rowwise_rel(Jg, J_o) <= 1e-10
    assert rel(r.cpu().numpy(), r_o) <= 1e-10
    assert rel(grad.cpu().numpy(), J_o.T @ r_o) <= 1e-10
    omega = gp.gaussian_omega(seed=0, counter=0, ell=prob.ell)
    pc = gp.nystrom_sketch(J, prob.ell, omega=omega)
    G = linalg.gramian(J_o)
    _, lam_o, _ = nystrom.nystrom_alg6(lambda V: G @ V, omega.cpu().numpy()[:, :gp.P].T)
    lam = pc.lam_hat.cpu().numpy()
    assert np.max(np.abs(lam - lam_o[:lam.size])) <= 1e-10 * lam_o[0]
    g = grad
    out = gp.pcg_solve(J, g, prob.lam, precond=pc, rtol=1e-8, maxit=1000)
    assert out.converged
    d_star = linalg.solve_cholesky(G, g.cpu().numpy(), prob.lam)
    res = linalg.true_relative_residual(G, prob.lam, g.cpu().numpy(), out.d.cpu().numpy())
    assert res <= 1e-7
    assert np.linalg.norm(out.d.cpu().numpy() - d_star) <= 1.01 * res * np.linalg.norm(g.cpu().numpy()) / prob.lam \
        + 1e-9 * np.linalg.norm(d_star)
    gp.close()


def test_c2_full_fp32():
    """The benchmark workload: sampled Jacobian rows and all residuals against the oracle; the matvec, the
    gradient, the Alg. 6 eigenvalues and the PCG solution in FP64 on the GPU's own Jacobian."""
    prob, th, gp = _setup("c2")
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r, J, grad, loss = gp.residual_jacobian(theta, J)
    rows = _sample_rows(prob)
    J32 = J.cpu().numpy()[:, :gp.P]
    assert rowwise_rel(J32[rows], mlp.jacobian(th, prob, rows)) <= 1e-5
    r_o = mlp.weighted_residual(th, prob)
    assert rel(r.cpu().numpy(), r_o) <= 1e-5
    r32 = r.cpu().numpy().astype(np.float64)
    assert rel(grad.cpu().numpy(), J32.astype(np.float64).T @ r32) <= 1e-5
    # one-pass matvec at full size
    v = np.random.default_rng(2).standard_normal(gp.P).astype(np.float32)
    lam = 1e-4
    y = gp.gramian_matvec(J, torch.as_tensor(v, device="cuda"), lam).cpu().numpy()
    y_ref = _jt_mul(J32, v.astype(np.float64)) + lam * v
    assert rel(y, y_ref) <= 1e-5
    # Alg. 6 on the same (FP32-rounded) Jacobian and Omega, FP64
    omega = gp.gaussian_omega(seed=0, counter=3, ell=prob.ell)
    pc = gp.nystrom_sketch(J, prob.ell, omega=omega, sketch_dtype="f32")
    J64 = J32.astype(np.float64)
    _, lam_o, _ = nystrom.nystrom_alg6(lambda V: J64.T @ (J64 @ V), omega.cpu().numpy()[:, :gp.P].T.astype(np.float64))
    lam_g = pc.lam_hat.cpu().numpy()
    top = lam_o[:lam_g.size] >= 1e-6 * lam_o[0]
    assert np.max(np.abs(lam_g[top] - lam_o[:lam_g.size][top])) <= 1e-5 * lam_o[0]
    # PCG at rtol 1e-6 with the solver's damping rule (Section 4.3): true residual on the FP32 operator
    mu = max(10 * EPS["f32"] * lam_g[0], 1e-4 * loss.item() ** 2)
    out = gp.pcg_solve(J, grad, mu, precond=pc, rtol=1e-6, maxit=1000)
    assert out.converged
    _check_solve(J32, grad.cpu().numpy(), out.d.cpu().numpy(), mu, 1e-6)
    gp.close()


def _gnys_frobenius_rel(Ua, a, Ub, b):
    """||Ua diag(a) Ua^T - Ub diag(b) Ub^T||_F / ||Ub diag(b) Ub^T||_F without forming the P x P matrices:
    with [Ua Ub] = Q R (thin QR), the difference is Q (Ra diag(a) Ra^T - Rb diag(b) Rb^T) Q^T."""
    ka = Ua.shape[1]
    _, R = np.linalg.qr(np.concatenate([Ua, Ub], axis=1), mode="reduced")
    Ra, Rb = R[:, :ka], R[:, ka:]
    Bm = (Rb * b) @ Rb.T
    return float(np.linalg.norm((Ra * a) @ Ra.T - Bm) / np.linalg.norm(Bm))


def _j64_mul(J32, V, chunk=2048):
    """FP64 J^T (J V) for a block V with J the GPU's FP32 Jacobian (host copy), in row chunks."""
    out = np.zeros((J32.shape[1], V.shape[1]))
    for s in range(0, J32.shape[0], chunk):
        Jc = J32[s:s + chunk].astype(np.float64)
        out += Jc.T @ (Jc @ V)
    return out


@pytest.mark.timeout(900)
def test_c3_full_bf16_sketch():
    """The 5D workload (N = 18,432, P = 33,921, ell = 800): sampled Jacobian rows against the oracle; the
    gradient in FP64 on the GPU's Jacobian; the BF16 and the FP32 sketch against Alg. 6 run in FP64 on the
    GPU's own FP32 Jacobian with the same Omega: eigenvalues lam_i >= 0.1 lam_1 and G_nys in the Frobenius
    norm, relative (BF16 before refinement <= 2e-2, FP32 <= 1e-5); U orthonormal; the refined solve's
    true residual."""
    prob, th, gp = _setup("c3")
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r, J, grad, loss = gp.residual_jacobian(theta, J)
    rows = _sample_rows(prob, n=9)
    Jr = J[torch.as_tensor(rows, device="cuda")].cpu().numpy()[:, :gp.P]
    assert rowwise_rel(Jr, mlp.jacobian(th, prob, rows)) <= 1e-5
    J32 = J.cpu().numpy()[:, :gp.P]
    r32 = r.cpu().numpy().astype(np.float64)
    g_ref = np.zeros(gp.P)
    for s in range(0, J32.shape[0], 2048):
        g_ref += J32[s:s + 2048].astype(np.float64).T @ r32[s:s + 2048]
    assert rel(grad.cpu().numpy(), g_ref) <= 1e-5
    omega = gp.gaussian_omega(seed=0, counter=0, ell=prob.ell)
    pb = gp.nystrom_sketch(J, prob.ell, omega=omega, sketch_dtype="bf16")
    pf = gp.nystrom_sketch(J, prob.ell, omega=omega, sketch_dtype="f32")
    torch.cuda.synchronize()
    Om = omega.cpu().numpy()[:, :gp.P].T.astype(np.float64)
    Uo, lo, _ = nystrom.nystrom_alg6(lambda V: _j64_mul(J32, V), Om)
    big = lo >= 0.1 * lo[0]
    for name, pc, tol in (("bf16", pb, 2e-2), ("f32", pf, 1e-5)):
        lam = pc.lam_hat.cpu().numpy()
        U = pc.U.cpu().numpy()[:, :gp.P].astype(np.float64)
        lam_err = float(np.max(np.abs(lam[big] - lo[big]) / lo[big]))
        keep = lam > 0
        fro = _gnys_frobenius_rel(U[keep].T, lam[keep], Uo, lo)
        print(f"c3 {name} sketch vs Alg. 6 (FP64): max rel err of lam_i >= 0.1 lam_1 ({int(big.sum())} of them) "
              f"= {lam_err:.2e}, ||G_nys - G_alg6||_F / ||G_alg6||_F = {fro:.2e}", flush=True)
        assert lam_err <= tol and fro <= tol
    U = pb.U[:, :gp.P].double()
    top = pb.lam_hat >= 1e-6 * pb.lam_hat[0]
    Uk = U[top]
    E = (Uk @ Uk.T - torch.eye(int(top.sum()), dtype=torch.float64, device="cuda")).abs().max().item()
    assert E <= 1e-5
    lb = pb.lam_hat.cpu().numpy()
    mu = max(10 * EPS["f32"] * lb[0], 1e-4 * loss.item() ** 2)
    out = gp.pcg_solve(J, grad, mu, precond=pb, rtol=1e-6, maxit=1000)
    assert out.converged
    _check_solve(J32, grad.cpu().numpy(), out.d.cpu().numpy(), mu, 1e-6)
    gp.close()


def test_c4_full_recompute():
    """The heat workload in recompute mode: JVP and adjoint products at full size against the oracle's
    Jacobian rows (sampled JVP outputs; an adjoint weight vector supported on the sampled rows)."""
    prob, th, gp = _setup("c4")
    theta = gp.theta(th)
    rows = _sample_rows(prob)
    J_o = mlp.jacobian(th, prob, rows)
    u = np.random.default_rng(4).standard_normal(gp.P).astype(np.float32)
    jv = gp.jvp(theta, torch.as_tensor(u, device="cuda")).cpu().numpy()
    assert rel(jv[rows], J_o @ u.astype(np.float64)) <= 1e-5
    wv = np.zeros(gp.N, dtype=np.float32)
    wv[rows] = np.random.default_rng(5).standard_normal(rows.size)
    g = gp.vjp(theta, torch.as_tensor(wv, device="cuda")).cpu().numpy()
    assert rel(g, J_o.T @ wv[rows].astype(np.float64)) <= 1e-5
    # the recompute-mode operator against the JVP/VJP composition it stands for
    v = torch.as_tensor(np.random.default_rng(6).standard_normal(gp.P), dtype=torch.float32, device="cuda")
    y = gp.gramian_matvec(Recompute(theta), v, 1e-3).cpu().numpy().astype(np.float64)
    t = gp.jvp(theta, v)
    y2 = gp.vjp(theta, t).cpu().numpy() + 1e-3 * v.cpu().numpy()
    assert rel(y, y2) <= 1e-5
    gp.close()


@pytest.mark.timeout(600)
def test_c4_full_recompute_sketch():
    """The heat workload's recompute-mode sketch (rows of J_w re-formed a block at a time and multiplied
    by the stored path's GEMMs) against Alg. 6 in FP64 on the GPU's own FP32 Jacobian, stored once for
    the check (and itself checked on sampled rows against the oracle), with the same Omega: eigenvalues
    above 1e-6 lam_1 and G_nys on probe vectors to 1e-5 lam_1."""
    prob, th, gp = _setup("c4")
    theta = gp.theta(th)
    J = gp.new_jacobian()
    gp.residual_jacobian(theta, J)
    rows = _sample_rows(prob)
    J32 = J.cpu().numpy()[:, :gp.P]
    assert rowwise_rel(J32[rows], mlp.jacobian(th, prob, rows)) <= 1e-5
    omega = gp.gaussian_omega(seed=0, counter=1, ell=prob.ell)
    pc = gp.nystrom_sketch(Recompute(theta), prob.ell, omega=omega, sketch_dtype="f32")
    torch.cuda.synchronize()
    Om = omega.cpu().numpy()[:, :gp.P].T.astype(np.float64)
    Uo, lo, _ = nystrom.nystrom_alg6(lambda V: _j64_mul(J32, V), Om)
    lam = pc.lam_hat.cpu().numpy()
    U = pc.U.cpu().numpy()[:, :gp.P].astype(np.float64)
    top = lo >= 1e-6 * lo[0]
    err = float(np.max(np.abs(lam[top] - lo[top])) / lo[0])
    X = wl.probe_vectors(gp.P, 5, seed=8)
    keep = lam > 0
    Gg = U[keep].T @ (lam[keep][:, None] * (U[keep] @ X))
    Go = Uo @ (lo[:, None] * (Uo.T @ X))
    pe = float(np.linalg.norm(Gg - Go) / (lo[0] * np.linalg.norm(X)))
    print(f"c4 recompute sketch vs Alg. 6: max |lam_i - lam_alg6_i| / lam_1 (lam_i >= 1e-6 lam_1) = {err:.2e}, "
          f"probe error / lam_1 = {pe:.2e}", flush=True)
    assert err <= 1e-5 and pe <= 1e-5
    gp.close()
