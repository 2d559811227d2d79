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
    approximation with the core shift the GPU keeps (nu = 10 eps tr(Omega^T G Omega)), on the distinct
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
    nu = 10 * 2.0 ** -52 * np.trace(Z.T @ Z)
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
