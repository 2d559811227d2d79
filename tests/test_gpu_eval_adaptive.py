"""GPU parity of the accuracy measure (relative L2 / H1 errors of Section 5) and of the adaptive
sketch size of Alg. 4 as the NGD driver applies it (MI355X).

The four error sums are FP64 on both sides, so they agree to 1e-12 relative on the same inputs (FP32
problems: the oracle runs on the FP32-rounded theta, points and reference values)."""
import ctypes as C
import dataclasses

import numpy as np
import pytest

import workloads as wl
from gpu_helpers import make

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from oracle import mlp, ngd as ongd  # noqa: E402
from paper_2505_11638_amd.api import Problem  # noqa: E402
from paper_2505_11638_amd.driver import NGD  # noqa: E402

CASES = {
    "poisson2d_f64": lambda: wl.small_problem(widths=(2, 32, 32, 1), n_interior=40, n_boundary=12, seed=1),
    "poisson3d_f64_paper_widths": lambda: wl.small_problem(d=3, widths=(3, 64, 64, 64, 1), n_interior=30,
                                                           n_boundary=10, seed=2),
    "poisson5d_f32": lambda: wl.small_problem(d=5, widths=(5, 48, 40, 1), n_interior=30, n_boundary=10, seed=3,
                                              dtype="f32"),
    "heat_f32_wide": lambda: wl.small_problem(pde=wl.PDE_HEAT, widths=(3, 128, 96, 1), n_interior=30, n_boundary=10,
                                              seed=4, dtype="f32"),
}


def _round(a, dtype):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64) if dtype == "f32" else np.asarray(a)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("n", [1, 37, 1000, 40001])
def test_solution_error_matches_oracle(name, n):
    prob, th = make(CASES[name]())
    gp = Problem(prob, dtype=prob.dtype, max_ell=4)
    rng = np.random.default_rng(n)
    X = _round(rng.uniform(0, 1, (n, prob.d)), prob.dtype)
    u_ref = _round(rng.standard_normal(n), prob.dtype)
    g_ref = _round(rng.standard_normal((n, prob.d)), prob.dtype)
    l2, h1, sums = gp.solution_error(gp.theta(th), X, u_ref, g_ref)
    want = mlp.solution_error_sums(th, prob.widths, X, u_ref, g_ref)
    got = sums.cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=1e-12)
    wl2, wh1 = mlp.relative_errors(want)
    assert abs(l2 - wl2) <= 1e-12 * wl2 and abs(h1 - wh1) <= 1e-12 * wh1
    gp.close()


def test_solution_error_empty_and_invalid():
    prob, th = make(CASES["poisson2d_f64"]())
    gp = Problem(prob, dtype=prob.dtype, max_ell=4)
    sums = torch.full((4,), 7.0, dtype=torch.float64, device="cuda")
    gp.solution_error(gp.theta(th), np.zeros((0, 2)), np.zeros(0), np.zeros((0, 2)), sums=sums)
    assert np.all(sums.cpu().numpy() == 0.0)
    # n < 0 and NULL inputs are refused on the host, before any launch
    st = gp.lib.ngd_solution_error(gp.h, None, None, -1, None, None, C.c_void_p(sums.data_ptr()), None)
    assert st != 0
    st = gp.lib.ngd_solution_error(gp.h, None, None, 5, None, None, C.c_void_p(sums.data_ptr()), None)
    assert st != 0
    with pytest.raises(ValueError):
        gp.solution_error(gp.theta(th), np.zeros((3, 3)), np.zeros(3), np.zeros((3, 3)))
    gp.close()


def test_solution_error_of_the_exact_network():
    """Against the network's own values and gradients (from the oracle) both errors vanish."""
    prob, th = make(CASES["poisson3d_f64_paper_widths"]())
    gp = Problem(prob, dtype=prob.dtype, max_ell=4)
    X = np.random.default_rng(9).uniform(0, 1, (500, 3))
    u, g, _, _, _ = mlp.taylor_forward(th, prob.widths, X, wl.PDE_POISSON)
    l2, h1, _ = gp.solution_error(gp.theta(th), X, u, g)
    assert l2 < 1e-13 and h1 < 1e-13
    gp.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_adaptive_rank_follows_alg4(dtype):
    """Every step's next sketch size is Alg. 4's rule applied to that step's own eigenvalue estimates
    and damping (re-derived here with the oracle's rule), the size actually sketched at each step is
    the one chosen before it, and the rank reaches both branches of the rule."""
    prob = wl.poisson_random(d=3, widths=(3, 24, 24, 1), n_interior=400, n_boundary=80, seed=5, dtype=dtype,
                             ell=8, sketch_dtype=dtype)
    prob = dataclasses.replace(prob, ell_max=48, dell=8, maxit=20)
    ngd = NGD(prob, wl.glorot_theta(prob.widths, 5), solver="nystrom", seed=5)
    expect = prob.ell
    grew = shrank = False
    for _ in range(12):
        rep = ngd.step()
        assert rep.rank == expect
        lam = ngd.pc.lam_hat.cpu().numpy()[:rep.rank].copy()
        assert np.all(np.diff(lam) <= 0)
        expect = ongd.next_rank(lam, rep.mu, rep.rank, prob.ell_max, prob.dell)
        assert ngd.ell == expect
        grew |= expect > rep.rank
        shrank |= expect < rep.rank
        assert rep.loss_new <= rep.loss
    assert grew
    ngd.gp.close()


def test_heat3d_paper_shape_parity_and_steps():
    """The heat equation in 3+1D (four inputs, three Laplacian coordinates, time last): residuals,
    Jacobian and gradient against the oracle, the error sums against the oracle's, and adaptive Nystrom
    NGD steps that decrease the loss."""
    prob = wl.heat3d_paper(widths=(4, 24, 20, 1), n_interior=70, n_boundary=35, seed=7, ell=8)
    prob = dataclasses.replace(prob, ell_max=40, dell=8, maxit=20)
    th = wl.glorot_theta(prob.widths, 7)
    gp = Problem(prob, dtype="f64", max_ell=40)
    theta = gp.theta(th)
    r, J, grad, loss = gp.residual_jacobian(theta, gp.new_jacobian())
    r_o, J_o = mlp.residual_and_jacobian(th, prob)
    assert np.linalg.norm(r.cpu().numpy() - r_o) <= 1e-10 * np.linalg.norm(r_o)
    assert np.linalg.norm(J.cpu().numpy()[:, :gp.P] - J_o) <= 1e-10 * np.linalg.norm(J_o)
    assert np.linalg.norm(grad.cpu().numpy() - J_o.T @ r_o) <= 1e-10 * np.linalg.norm(J_o.T @ r_o)
    X, u, g = wl.evaluation_set(prob, 3000, seed=1)
    _, _, sums = gp.solution_error(theta, X, u, g)
    np.testing.assert_allclose(sums.cpu().numpy(), mlp.solution_error_sums(th, prob.widths, X, u, g), rtol=1e-12)
    gp.close()
    ngd = NGD(prob, th, solver="nystrom", seed=7)
    L0 = None
    for _ in range(4):
        rep = ngd.step()
        L0 = rep.loss if L0 is None else L0
        assert rep.loss_new <= rep.loss
    assert rep.loss_new < L0
    ngd.gp.close()


def test_library_rank_rule_and_damping_match_oracle():
    """ngd_next_rank (Alg. 4's update) against the oracle's rule on 400 random cases (both branches, the
    threshold itself, zeros of dropped pairs, the cap), and ngd_damping (Section 4.3) against the
    rule written out, both branches, with and without a loss."""
    prob = wl.small_problem(widths=(2, 32, 32, 1), n_interior=61, n_boundary=22, seed=1, ell=24)
    gp = Problem(prob, dtype="f64", max_ell=24)
    rng = np.random.default_rng(0)
    for trial in range(400):
        ell = int(rng.integers(1, 60))
        ell_max = int(rng.integers(ell, 120))
        dell = int(rng.integers(1, 30))
        off = int(rng.integers(1, 3))
        lam = np.sort(10.0 ** rng.uniform(-8, 2, ell))[::-1]
        if trial % 5 == 0:
            lam[rng.integers(0, ell):] = 0.0  # dropped pairs are reported as zeros
        mu = float(10.0 ** rng.uniform(-7, 0))
        if trial % 7 == 0:
            mu = float(lam[ell - 1]) / 10.0  # on the threshold
        lam_dev = torch.as_tensor(lam.copy(), dtype=torch.float64, device="cuda")
        got = gp.next_rank(lam_dev, ell, mu, dell, off, ell_max)
        assert got == min(ongd.next_rank(lam, mu, ell, ell_max, dell, off), gp.P), (trial, got)
    for lam1, loss in [(3.0, 1e-2), (3.0, 10.0), (1e-9, None)]:
        l1 = torch.tensor([lam1], dtype=torch.float64, device="cuda")
        lt = None if loss is None else torch.tensor([loss], dtype=torch.float64, device="cuda")
        mu_dev, mu = gp.damping(l1, lt, 10 * 2.0 ** -52, 1e-4)
        want = max(10 * 2.0 ** -52 * lam1, 1e-4 * (loss or 0.0) * (loss or 0.0))
        assert mu == want and mu_dev.item() == want
    gp.close()

