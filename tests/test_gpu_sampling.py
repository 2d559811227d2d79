"""GPU parity of the Gramian diagonal (eq. gram_diagonal), pivot sampling (s ~ d) and the Nystrom
builder with a sampling test matrix (Section 5), through the C ABI (MI355X)."""
import dataclasses

import numpy as np
import pytest

import workloads as wl
from gpu_helpers import make

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from oracle import mlp, nystrom, sampling  # noqa: E402
from paper_2505_11638_amd import _lib as L  # noqa: E402
from paper_2505_11638_amd.api import Problem, Recompute  # noqa: E402
from paper_2505_11638_amd.driver import NGD  # noqa: E402

CASES = {
    "poisson2d_f64": lambda: wl.small_problem(widths=(2, 32, 32, 1), n_interior=61, n_boundary=22, seed=1, ell=24,
                                              lam=1e-6),
    "poisson2d_f32": lambda: wl.small_problem(widths=(2, 64, 64, 64, 1), n_interior=97, n_boundary=30, seed=2,
                                              dtype="f32", ell=40, lam=1e-4),
    "heat_f32": lambda: wl.small_problem(pde=wl.PDE_HEAT, widths=(3, 64, 64, 1), n_interior=70, n_boundary=26,
                                         seed=5, dtype="f32", ell=30, lam=1e-4),
}


def _setup(name):
    prob, th = make(CASES[name]())
    gp = Problem(prob, dtype=prob.dtype, max_ell=prob.ell)
    theta = gp.theta(th)
    J = gp.new_jacobian()
    gp.residual_jacobian(theta, J)
    return prob, th, gp, theta, J


@pytest.mark.parametrize("name", list(CASES))
def test_gramian_diagonal(name):
    prob, th, gp, theta, J = _setup(name)
    d = gp.gramian_diagonal(J).cpu().numpy()
    Jg = J.cpu().numpy().astype(np.float64)[:, :gp.P]
    # the kernel against the squared column norms of the same J (FP64 sums of the stored values)
    np.testing.assert_allclose(d, sampling.gram_diagonal(Jg), rtol=1e-12, atol=0)
    # and against the oracle's Jacobian
    Jo = mlp.jacobian(th, prob)
    tol = 1e-10 if prob.dtype == "f64" else 1e-5
    assert np.max(np.abs(d - sampling.gram_diagonal(Jo))) <= tol * np.max(sampling.gram_diagonal(Jo))
    # recompute mode: rows of J_w formed a block at a time
    dr = gp.gramian_diagonal(Recompute(theta)).cpu().numpy()
    np.testing.assert_allclose(dr, d, rtol=1e-12 if prob.dtype == "f64" else 1e-6, atol=0)
    gp.close()


@pytest.mark.parametrize("n", [1, 37, 1000, 4096])
def test_sample_pivots_match_oracle(n):
    prob, th, gp, theta, J = _setup("poisson2d_f32")
    w = gp.gramian_diagonal(J)
    w[::7] = 0.0   # zero weights are never drawn
    w[3] = -1.0    # negative weights count as zero
    idx, cnt = gp.sample_pivots(w, n, seed=9, counter=4, substream=2)
    got = idx.cpu().numpy()[:n]
    assert int(cnt.item()) == n
    wh = w.cpu().numpy()
    want = sampling.sample_pivots(wh, n, seed=9, counter=4, substream=2)
    mism = np.nonzero(got != want)[0]
    # the running sums are formed in another order: a draw may differ only where its target lies
    # within rounding of a boundary of the cumulative distribution
    cum = np.cumsum(np.maximum(wh, 0))
    u = sampling.sample_uniforms(n, 9, 4, 2) * cum[-1]
    for k in mism:
        assert min(abs(cum[got[k]] - u[k]), abs(cum[want[k]] - u[k])) <= 1e-12 * cum[-1]
    assert mism.size <= max(1, n // 1000)
    assert np.all(np.maximum(wh, 0)[got] > 0)
    gp.close()


def test_sample_pivots_unique_and_degenerate():
    prob, th, gp, theta, J = _setup("poisson2d_f64")
    w = torch.zeros(gp.P, dtype=torch.float64, device="cuda")
    w[5:25] = torch.arange(1, 21, dtype=torch.float64, device="cuda")
    idx, cnt = gp.sample_pivots(w, 20, seed=1, counter=0, substream=3, unique=True)
    c = int(cnt.item())
    got = idx.cpu().numpy()[:c]
    want = sampling.sample_pivots(w.cpu().numpy(), 20, 1, 0, 3, unique=True)
    np.testing.assert_array_equal(got, want)
    assert np.all(np.diff(got) > 0)
    z = torch.zeros(gp.P, dtype=torch.float64, device="cuda")
    idx, cnt = gp.sample_pivots(z, 8, seed=1)
    assert int(cnt.item()) == 0 and np.all(idx.cpu().numpy()[:8] == -1)
    gp.close()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("unique", [True, False])
def test_nystrom_sketch_columns_matches_alg6(name, unique):
    """The sampling test matrix: GPU eigenpairs and G_nys on probe vectors against the Nystrom
    approximation with the core shift the GPU keeps (nu = c eps tr(Omega^T G Omega), c = 1 for FP64 and
    10 for FP32 Jacobians), on the distinct
    sampled columns (repeats leave range(Omega) unchanged; their extra directions come out as ~0
    pairs). Against Alg. 6, which removes its shift, the difference is the shift's effect, amplified by
    the conditioning of G[S, S] (about 1e-10 lam_1 here); it is bounded below as well."""
    prob, th, gp, theta, J = _setup(name)
    tol = 1e-10 if prob.dtype == "f64" else 1e-5
    Jg = J.cpu().numpy().astype(np.float64)[:, :gp.P]
    d = sampling.gram_diagonal(Jg)
    cols = sampling.sample_pivots(d, prob.ell, seed=2, counter=1, unique=unique)
    ell = cols.size
    cdev = torch.as_tensor(cols, dtype=torch.int64, device="cuda")
    res = gp.nystrom_sketch(J, ell, cols=cdev)
    U = res.U.cpu().numpy().astype(np.float64)[:, :gp.P]
    lam = res.lam_hat.cpu().numpy()
    Om = sampling.column_test_matrix(gp.P, np.unique(cols))
    Om_all = sampling.column_test_matrix(gp.P, cols)
    G = Jg.T @ Jg
    Z = Jg @ Om_all
    nu = (1 if prob.dtype == "f64" else 10) * 2.0 ** -52 * np.trace(Z.T @ Z)  # the core's shift
    Gs = nystrom.nystrom_shifted(G, Om_all, nu)
    ls = np.sort(np.linalg.eigvalsh(Gs))[::-1]
    assert np.all(np.diff(lam) <= 0) and np.all(lam >= 0)
    r = Om.shape[1]
    assert np.max(np.abs(lam[:r] - ls[:r])) <= tol * ls[0]
    assert np.all(lam[r:] <= tol * ls[0])
    keep = lam > 0
    X = wl.probe_vectors(gp.P, 5, seed=3)
    Gg = U[keep].T @ (lam[keep][:, None] * (U[keep] @ X))
    assert np.linalg.norm(Gg - Gs @ X) <= tol * ls[0] * np.linalg.norm(X)
    _, lo, _ = nystrom.nystrom_alg6(lambda V: G @ V, Om)
    assert np.max(np.abs(lam[:r] - lo)) <= max(tol, 1e-9) * lo[0]
    # recompute mode gathers the same columns from rows formed a block at a time
    rr = gp.nystrom_sketch(Recompute(theta), ell, cols=cdev)
    assert np.max(np.abs(rr.lam_hat.cpu().numpy() - lam)) <= tol * lo[0]
    gp.close()


@pytest.mark.parametrize("name", ["poisson2d_f32", "heat_f32"])
def test_nystrom_sketch_columns_bf16(name):
    """A BF16 sketch with a sampling test matrix: Z is a gather of J's columns (no Omega is cast or
    read), only the product B^T = Q^T J runs in BF16. Eigenvalues and G_nys on probe vectors against
    the shifted Nystrom definition on the same columns, at the BF16 sketch tolerance (2e-2 of lam_1),
    and the padding columns of U stay zero."""
    prob, th, gp, theta, J = _setup(name)
    Jg = J.cpu().numpy().astype(np.float64)[:, :gp.P]
    cols = sampling.sample_pivots(sampling.gram_diagonal(Jg), prob.ell, seed=4, counter=2, unique=True)
    ell = cols.size
    cdev = torch.as_tensor(cols, dtype=torch.int64, device="cuda")
    res = gp.nystrom_sketch(J, ell, cols=cdev, sketch_dtype="bf16")
    torch.cuda.synchronize()
    Uf = res.U.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(Uf)) and np.all(Uf[:, gp.P:] == 0.0)
    U, lam = Uf[:, :gp.P], res.lam_hat.cpu().numpy()
    G = Jg.T @ Jg
    Om = sampling.column_test_matrix(gp.P, cols)
    Z = Jg @ Om
    Gs = nystrom.nystrom_shifted(G, Om, 10 * 2.0 ** -52 * np.trace(Z.T @ Z))
    ls = np.sort(np.linalg.eigvalsh(Gs))[::-1][:ell]
    assert np.all(np.diff(lam) <= 0) and np.all(lam >= 0)
    assert np.max(np.abs(lam - ls)) <= 2e-2 * ls[0]
    X = wl.probe_vectors(gp.P, 5, seed=3)
    Gg = U.T @ (lam[:, None] * (U @ X))
    assert np.linalg.norm(Gg - Gs @ X) <= 2e-2 * ls[0] * np.linalg.norm(X)
    # the FP32 column sketch of the same columns agrees to the same bound
    r32 = gp.nystrom_sketch(J, ell, cols=cdev, sketch_dtype="f32")
    assert np.max(np.abs(r32.lam_hat.cpu().numpy() - lam)) <= 2e-2 * ls[0]
    gp.close()


def test_ngd_with_sampling_test_matrix_decreases_loss():
    prob = wl.poisson_random(d=3, widths=(3, 24, 24, 1), n_interior=400, n_boundary=80, seed=5, dtype="f64",
                             ell=30, sketch_dtype="f64")
    prob = dataclasses.replace(prob, ell_max=60, dell=10, maxit=20)
    ngd = NGD(prob, wl.glorot_theta(prob.widths, 5), solver="nystrom", seed=5, test_matrix="sampling")
    losses = []
    for _ in range(6):
        rep = ngd.step()
        assert rep.loss_new <= rep.loss
        losses.append(rep.loss_new)
    assert losses[-1] < 0.5 * ngd_first_loss(prob)
    ngd.gp.close()


def ngd_first_loss(prob):
    return mlp.loss(wl.glorot_theta(prob.widths, 5), prob)


# ---- block RPCholesky and RPCholNGD ----

@pytest.mark.parametrize("name", ["poisson2d_f64", "poisson2d_f32"])
@pytest.mark.parametrize("ell_max,block,frac", [(40, 20, 0.0), (37, 8, 1e-3), (12, 5, 0.0)])
def test_rpcholesky_matches_oracle(name, ell_max, block, frac):
    """F against the oracle's block RPCholesky on the same diagonal and Gramian (columns of G from the
    GPU's own J in FP64); the rank, the residual trace and F F^T on probes agree."""
    prob, th, gp, theta, J = _setup(name)
    Jg = J.cpu().numpy().astype(np.float64)[:, :gp.P]
    G = Jg.T @ Jg
    d = gp.gramian_diagonal(J)
    eps = frac * float(np.trace(G))
    gp2 = Problem(prob, dtype=prob.dtype, max_ell=ell_max + 1)
    Ft, r, tr = gp2.rpcholesky(J, d, ell_max, block, seed=4, counter=3, eps=eps)
    Fo, piv, tro = sampling.block_rpcholesky(lambda S: G[:, S], d.cpu().numpy(), ell_max, block, 4, 3, eps)
    assert r == Fo.shape[1]
    F = Ft.cpu().numpy()[:r, :gp.P].T
    assert np.all(Ft.cpu().numpy()[r:, :gp.P] == 0)
    # the columns of the first block (a well-conditioned pivot block) agree entry by entry; later
    # columns come from nearly dependent pivots and carry the conditioning of their pivot blocks, so
    # the approximation F F^T is compared instead
    k0 = min(r, block)
    np.testing.assert_allclose(F[:, :k0], Fo[:, :k0], rtol=0, atol=1e-10 * np.abs(Fo).max())
    np.testing.assert_allclose(F @ F.T, Fo @ Fo.T, rtol=0, atol=1e-10 * np.abs(G).max())
    assert abs(tr - tro) <= 1e-9 * np.trace(G)
    X = wl.probe_vectors(gp.P, 4, seed=1)
    assert np.linalg.norm(F @ (F.T @ X) - Fo @ (Fo.T @ X)) <= 1e-9 * np.linalg.norm(G) * np.linalg.norm(X)
    gp2.close()
    gp.close()


@pytest.mark.parametrize("cfg", ["small", "c2"])
def test_rpcholesky_recompute_mode_matches_stored(cfg):
    """Block RPCholesky with J_w recomputed from theta a block of rows at a time (two blocks at the
    benchmark's 2D size) against the same call on the stored J_w: the same rank and trace, F to rounding."""
    if cfg == "small":
        prob, th = make(CASES["poisson2d_f64"]())
    else:
        prob = wl.config("c2")
        th = wl.glorot_theta(prob.widths, 0)
    print("rpcholesky recompute mode,", cfg, flush=True)
    ell_max = 60
    gp = Problem(prob, dtype=prob.dtype, max_ell=ell_max + 1)
    theta = gp.theta(th)
    J = gp.new_jacobian()
    gp.residual_jacobian(theta, J)
    d = gp.gramian_diagonal(J)
    Ft, r, tr = gp.rpcholesky(J, d, ell_max, 20, seed=5, counter=2, eps=0.0)
    Ft2, r2, tr2 = gp.rpcholesky(Recompute(theta), d, ell_max, 20, seed=5, counter=2, eps=0.0)
    assert r2 == r and abs(tr2 - tr) <= 1e-9 * float(d.sum())
    F, F2 = Ft.cpu().numpy()[:r, :gp.P], Ft2.cpu().numpy()[:r, :gp.P]
    tol = 1e-9 if prob.dtype == "f64" else 1e-6
    assert np.abs(F2 - F).max() <= tol * np.abs(F).max()
    gp.close()


def test_rpchol_ngd_steps_recompute_mode():
    """RPCholNGD with J_w never stored follows the stored-J_w steps (same pivots and ranks, losses to the
    solves' tolerance)."""
    prob = wl.poisson_random(d=3, widths=(3, 24, 24, 1), n_interior=400, n_boundary=80, seed=6, dtype="f64",
                             ell=40, sketch_dtype="f64")
    th0 = wl.glorot_theta(prob.widths, 6)
    a = NGD(prob, th0, solver="rpchol", seed=6, ell_max=60, maxit=20)
    b = NGD(prob, th0, solver="rpchol", seed=6, ell_max=60, maxit=20, recompute=True)
    L0 = None
    for _ in range(5):
        ra, rb = a.step(), b.step()
        L0 = ra.loss if L0 is None else L0
        assert rb.rank == ra.rank
        # the solves stop at rtol 1e-6 on either path, so the trajectories agree to about that
        assert abs(rb.loss_new - ra.loss_new) <= 1e-6 * ra.loss
    assert rb.loss_new < 0.5 * L0
    a.gp.close()
    b.gp.close()


@pytest.mark.parametrize("name", ["poisson2d_f64", "poisson2d_f32"])
def test_rpchol_preconditioner_and_solve(name):
    """(U, lam_hat) reproduce F F^T with a trailing zero pair, and PCG with it solves (G + mu I) d = g
    in about as many iterations as the oracle's PCG with the Woodbury form eq. rpchol_precond."""
    from oracle import cg, linalg
    prob, th, gp0, theta, J = _setup(name)
    gp0.close()
    ell_max = 30
    gp = Problem(prob, dtype=prob.dtype, max_ell=ell_max + 1)
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r_, J, grad, loss = gp.residual_jacobian(theta, J)
    Jg = J.cpu().numpy().astype(np.float64)[:, :gp.P]
    G = Jg.T @ Jg
    mu = prob.lam
    d = gp.gramian_diagonal(J)
    Ft, r, _ = gp.rpcholesky(J, d, ell_max, 10, seed=1, counter=0, eps=mu * gp.P)
    pc = gp.rpchol_precond(Ft, r)
    U = pc.U.cpu().numpy().astype(np.float64)[:, :gp.P]
    lam = pc.lam_hat.cpu().numpy()
    assert lam.size == r + 1 and lam[-1] == 0 and np.all(U[-1] == 0) and np.all(np.diff(lam) <= 0)
    F = Ft.cpu().numpy()[:r, :gp.P].T
    X = wl.probe_vectors(gp.P, 4, seed=2)
    tol = 1e-10 if prob.dtype == "f64" else 1e-5
    assert np.linalg.norm(U.T @ (lam[:, None] * (U @ X)) - F @ (F.T @ X)) <= tol * lam[0] * np.linalg.norm(X)
    g = grad.cpu().numpy()
    rtol = 1e-8 if prob.dtype == "f64" else 1e-6
    out = gp.pcg_solve(J, grad, mu, precond=pc, rtol=rtol, maxit=2000)
    assert out.converged
    dstar = linalg.solve_cholesky(G, g, mu)
    res = np.linalg.norm(g - G @ out.d.cpu().numpy() - mu * out.d.cpu().numpy())
    assert res <= 10 * rtol * np.linalg.norm(g)
    assert np.linalg.norm(out.d.cpu().numpy() - dstar) <= res / mu * (1 + 1e-6) + 1e-12 * np.linalg.norm(dstar)
    ref = cg.pcg(lambda v: G @ v + mu * v, g, rtol, 2000, lambda v: sampling.rpchol_precond_apply(F, mu, v))
    assert ref.converged
    if prob.dtype == "f64":
        assert abs(out.iters - ref.iters) <= max(3, 0.25 * ref.iters)
    else:
        # rtol 1e-6 sits a few units above FP32 roundoff: the FP32 matvec needs a few more iterations
        assert ref.iters - 3 <= out.iters <= ref.iters + max(6, 0.5 * ref.iters)
    gp.close()


@pytest.mark.parametrize("name", ["poisson2d_f64", "poisson2d_f32"])
@pytest.mark.parametrize("ell_max", [30, 7])
def test_rpchol_woodbury_preconditioner_and_solve(name, ell_max):
    """The Woodbury-Cholesky form (eq. rpchol_precond): U holds W^T = (F R^{-1})^T with R^T R = F^T F + mu I
    and a zero row, lam_hat = [inf, ..., inf, 0]; the apply it implies equals the oracle's Woodbury apply on
    the GPU's own F; PCG with it solves (G + mu I) d = g in the oracle's Woodbury-PCG iteration count."""
    from oracle import cg, linalg
    prob, th, gp0, theta, J = _setup(name)
    gp0.close()
    gp = Problem(prob, dtype=prob.dtype, max_ell=ell_max + 1)
    theta = gp.theta(th)
    J = gp.new_jacobian()
    r_, J, grad, loss = gp.residual_jacobian(theta, J)
    Jg = J.cpu().numpy().astype(np.float64)[:, :gp.P]
    G = Jg.T @ Jg
    mu = prob.lam
    d = gp.gramian_diagonal(J)
    Ft, r, _ = gp.rpcholesky(J, d, ell_max, 10, seed=1, counter=0, eps=mu * gp.P)
    pc = gp.rpchol_precond(Ft, r, mu=mu)
    U = pc.U.cpu().numpy().astype(np.float64)[:, :gp.P]
    lam = pc.lam_hat.cpu().numpy()
    assert lam.size == r + 1 and lam[-1] == 0 and np.all(np.isinf(lam[:-1])) and np.all(U[-1] == 0)
    F = Ft.cpu().numpy()[:r, :gp.P].T
    Lc = np.linalg.cholesky(F.T @ F + mu * np.eye(r))
    Wt = np.linalg.solve(Lc, F.T)  # rows of W^T = L^{-1} F^T
    tol = 1e-10 if prob.dtype == "f64" else 1e-5
    assert np.linalg.norm(U[:r] - Wt) <= tol * np.linalg.norm(Wt)
    X = wl.probe_vectors(gp.P, 4, seed=2)
    applied = (X - U[:r].T @ (U[:r] @ X)) / mu
    ref_apply = sampling.rpchol_precond_apply(F, mu, X)
    assert np.linalg.norm(applied - ref_apply) <= tol * np.linalg.norm(ref_apply)
    g = grad.cpu().numpy()
    rtol = 1e-8 if prob.dtype == "f64" else 1e-6
    out = gp.pcg_solve(J, grad, mu, precond=pc, rtol=rtol, maxit=2000)
    assert out.converged
    dstar = linalg.solve_cholesky(G, g, mu)
    res = np.linalg.norm(g - G @ out.d.cpu().numpy() - mu * out.d.cpu().numpy())
    assert res <= 10 * rtol * np.linalg.norm(g)
    assert np.linalg.norm(out.d.cpu().numpy() - dstar) <= res / mu * (1 + 1e-6) + 1e-12 * np.linalg.norm(dstar)
    ref = cg.pcg(lambda v: G @ v + mu * v, g, rtol, 2000, lambda v: sampling.rpchol_precond_apply(F, mu, v))
    assert ref.converged
    # the same operator as the form from the eigenpairs of F^T F: about the same iteration count
    out_svd = gp.pcg_solve(J, grad, mu, precond=gp.rpchol_precond(Ft, r), rtol=rtol, maxit=2000)
    if prob.dtype == "f64":
        assert abs(out.iters - ref.iters) <= max(3, 0.25 * ref.iters)
        assert abs(out_svd.iters - out.iters) <= max(2, 0.1 * out.iters)
    else:
        # U in FP32: both forms apply mu^{-1} v minus a near-equal FP32 correction along the kept directions
        # (the cancellation 1 - sigma^2 / (sigma^2 + mu)), so with few pivots (a weak preconditioner, rtol a few
        # units above FP32 roundoff) the FP32 solve takes more iterations than the FP64 oracle; the two forms
        # stay alike
        assert ref.iters - 3 <= out.iters <= 2 * ref.iters + 6
        assert abs(out_svd.iters - out.iters) <= max(3, 0.25 * out.iters)
    with pytest.raises(L.NgdError):
        gp.rpchol_precond(Ft, r, mu=0.0)
    gp.close()


def test_rpchol_ngd_steps():
    prob = wl.poisson_random(d=3, widths=(3, 24, 24, 1), n_interior=400, n_boundary=80, seed=6, dtype="f64",
                             ell=40, sketch_dtype="f64")
    ngd = NGD(prob, wl.glorot_theta(prob.widths, 6), solver="rpchol", seed=6, ell_max=60, maxit=20)
    L0 = None
    for _ in range(5):
        rep = ngd.step()
        L0 = rep.loss if L0 is None else L0
        assert rep.loss_new <= rep.loss and 1 <= rep.rank <= 60
    assert rep.loss_new < 0.5 * L0
    ngd.gp.close()


def test_rpcholesky_and_sampling_reject_bad_arguments():
    """Argument errors are refused on the host before any launch, with a message."""
    from paper_2505_11638_amd import _lib as L
    prob, th, gp, theta, J = _setup("poisson2d_f64")
    d = gp.gramian_diagonal(J)
    for kw in [dict(block=0), dict(block=65), dict(ell_max=0), dict(ell_max=gp.P + 1), dict(eps=-1.0)]:
        args = dict(ell_max=10, block=5, eps=0.0)
        args.update(kw)
        with pytest.raises(Exception):
            gp.rpcholesky(J, d, args["ell_max"], args["block"], eps=args["eps"])
    with pytest.raises(Exception):
        gp.sample_pivots(d, 4097)
    with pytest.raises(Exception):
        gp.sample_pivots(d, 4, substream=2 ** 31)
    assert "substream" in L.load().ngd_last_error().decode()
    # the handle still works after refused calls
    Ft, r, _ = gp.rpcholesky(J, d, 10, 5)
    assert 1 <= r <= 10
    gp.close()
