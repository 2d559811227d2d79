"""The FP64 Nystrom core at every register-resident shape it has (ceil(ell / 64) = 1 .. 16: the
tridiagonalisation's 2- and 3-row layouts, the one-launch Cholesky's 4- and 8-wave tilings, the
triangular solve's tilings) against Alg. 6 in FP64, through the C ABI (MI355X).

Few points and a wide network (N = 1,130 rows, P = 2,545 parameters) keep the oracle cheap while the
sketch size runs up to the library's maximum of 1,024."""
import numpy as np
import pytest

import workloads as wl
from gpu_helpers import make

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from oracle import nystrom  # noqa: E402
from paper_2505_11638_amd.api import Problem  # noqa: E402

# one sketch size per register shape of the core kernels (ceil(ell / 64) = 1, 2, ..., 16), ragged, and
# two where the last step of the tridiagonal recurrences sits at lane 63 of a register (ell - 1 = 64 k)
ELLS = [37, 65, 100, 129, 150, 250, 300, 380, 420, 500, 560, 620, 690, 750, 800, 880, 940, 1024]


@pytest.fixture(scope="module")
def problem():
    prob, th = make(wl.poisson_random(d=2, widths=(2, 48, 48, 1), n_interior=1000, n_boundary=130, seed=11,
                                      dtype="f64", ell=1024, sketch_dtype="f64"), seed=4)
    gp = Problem(prob, dtype="f64", max_ell=1024)
    J = gp.new_jacobian()
    gp.residual_jacobian(gp.theta(th), J)
    Jg = J.cpu().numpy()[:, :gp.P]
    yield gp, J, Jg, Jg.T @ Jg
    gp.close()


@pytest.mark.parametrize("ell", ELLS)
def test_core_matches_alg6_at_every_shape(problem, ell):
    gp, J, Jg, G = problem
    print(f"core sweep: ell={ell} qn={(ell + 63) // 64} N={gp.N} P={gp.P}", flush=True)
    omega = gp.gaussian_omega(seed=21, counter=ell, ell=ell)
    res = gp.nystrom_sketch(J, ell, omega=omega)
    torch.cuda.synchronize()
    U = res.U.cpu().numpy()[:, :gp.P]
    lam = res.lam_hat.cpu().numpy()
    Uo, lo, _ = nystrom.nystrom_alg6(lambda V: G @ V, omega.cpu().numpy()[:, :gp.P].T)
    assert np.all(np.isfinite(lam)) and np.all(np.isfinite(U))
    assert np.all(np.diff(lam) <= 0) and np.all(lam >= 0)
    err = np.max(np.abs(lam - lo)) / lo[0]
    print(f"  max |lam - lam_alg6| / lam_1 = {err:.2e}, rank = {res.info['rank']}")
    assert err <= 1e-10
    # G_nys on probe vectors (U is unique only up to rotations inside clusters)
    X = wl.probe_vectors(gp.P, 6, seed=ell)
    keep = lam > 0
    Gg = U[keep].T @ (lam[keep][:, None] * (U[keep] @ X))
    Go = Uo @ (lo[:, None] * (Uo.T @ X))
    assert np.linalg.norm(Gg - Go) <= 1e-10 * lo[0] * np.linalg.norm(X)
    top = lam >= 1e-6 * lam[0]
    assert np.max(np.abs(U[top] @ U[top].T - np.eye(int(top.sum())))) <= 1e-8


@pytest.fixture(scope="module")
def synthetic():
    """A Jacobian with a prescribed, slowly decaying spectrum (singular values 10^(-4 i / N), so every
    Nystrom eigenvalue lies far above the core's drop threshold), in the same handle shape."""
    prob, _ = make(wl.poisson_random(d=2, widths=(2, 48, 48, 1), n_interior=1000, n_boundary=130, seed=11,
                                     dtype="f64", ell=1024, sketch_dtype="f64"))
    gp = Problem(prob, dtype="f64", max_ell=1024)
    rng = np.random.default_rng(17)
    N, P = gp.N, gp.P
    Ul, _ = np.linalg.qr(rng.standard_normal((N, N)))
    Vr, _ = np.linalg.qr(rng.standard_normal((P, N)))
    sig = 10.0 ** (-4.0 * np.arange(N) / N)
    Jg = (Ul * sig) @ Vr.T
    J = torch.zeros((N, gp.ld), dtype=torch.float64, device="cuda")
    J[:, :P] = torch.as_tensor(Jg, device="cuda")
    yield gp, J, Jg, Jg.T @ Jg
    gp.close()


@pytest.mark.parametrize("ell", ELLS)
def test_core_full_rank_spectrum_every_shape(synthetic, ell):
    """Every one of the ell Nystrom eigenpairs is kept here (no drop), so all rows of the register-resident
    tridiagonalisation, the inverse iteration and the back-transformation carry significant values."""
    gp, J, Jg, G = synthetic
    print(f"core sweep (synthetic spectrum): ell={ell} qn={(ell + 63) // 64}", flush=True)
    omega = gp.gaussian_omega(seed=22, counter=ell, ell=ell)
    res = gp.nystrom_sketch(J, ell, omega=omega)
    torch.cuda.synchronize()
    U = res.U.cpu().numpy()[:, :gp.P]
    lam = res.lam_hat.cpu().numpy()
    Uo, lo, _ = nystrom.nystrom_alg6(lambda V: G @ V, omega.cpu().numpy()[:, :gp.P].T)
    assert res.info["rank"] == ell and lo[-1] > 1e-9 * lo[0]
    err = np.max(np.abs(lam - lo)) / lo[0]
    print(f"  max |lam - lam_alg6| / lam_1 = {err:.2e}, lam_ell / lam_1 = {lo[-1] / lo[0]:.1e}")
    assert err <= 1e-10
    X = wl.probe_vectors(gp.P, 6, seed=ell + 1)
    Gg = U.T @ (lam[:, None] * (U @ X))
    Go = Uo @ (lo[:, None] * (Uo.T @ X))
    assert np.linalg.norm(Gg - Go) <= 1e-10 * lo[0] * np.linalg.norm(X)
    assert np.max(np.abs(U @ U.T - np.eye(ell))) <= 1e-8
