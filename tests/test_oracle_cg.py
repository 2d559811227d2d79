"""Pins of the oracle's (preconditioned) conjugate gradients (CPU only)."""
import numpy as np

from oracle import cg


def _spd(n, eigs, seed=0):
    Q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, n)))
    return Q @ np.diag(eigs) @ Q.T


def test_terminates_within_dimension():
    """Tiny, well-conditioned FP64 SPD systems: residual below 1e-12 within n iterations (exact
    arithmetic terminates in n)."""
    rng = np.random.default_rng(1)
    for n in (5, 17, 40):
        A = _spd(n, np.logspace(0, 1, n), seed=n)
        b = rng.standard_normal(n)
        res = cg.pcg(lambda v: A @ v, b, 1e-12, n)
        assert res.converged and res.iters <= n
        np.testing.assert_allclose(res.x, np.linalg.solve(A, b), rtol=1e-8)


def test_distinct_eigenvalue_count():
    """k distinct eigenvalues: CG converges in k iterations (exact arithmetic; FP64 within 1e-10)."""
    A = _spd(30, np.repeat([1.0, 4.0, 9.0], 10), seed=3)
    b = np.random.default_rng(2).standard_normal(30)
    res = cg.pcg(lambda v: A @ v, b, 1e-10, 30)
    assert res.converged and res.iters <= 3


def test_exact_preconditioner_one_step():
    A = _spd(20, np.logspace(0, 6, 20), seed=4)
    Ainv = np.linalg.inv(A)
    b = np.random.default_rng(3).standard_normal(20)
    res = cg.pcg(lambda v: A @ v, b, 1e-10, 20, lambda v: Ainv @ v)
    assert res.converged and res.iters == 1


def test_recursive_residual_tracks_true_residual():
    A = _spd(25, np.logspace(0, 4, 25), seed=5)
    b = np.random.default_rng(4).standard_normal(25)
    res = cg.pcg(lambda v: A @ v, b, 1e-8, 25)
    true = np.linalg.norm(b - A @ res.x) / np.linalg.norm(b)
    assert abs(true - res.rel_res) <= 1e-9
    assert all(h >= 0 for h in res.history)


def test_zero_rhs_and_maxit():
    A = _spd(10, np.arange(1, 11.0), seed=6)
    r0 = cg.pcg(lambda v: A @ v, np.zeros(10), 1e-8, 5)
    assert r0.iters == 0 and r0.converged and not r0.x.any()
    r1 = cg.pcg(lambda v: A @ v, np.ones(10), 1e-14, 2)
    assert r1.iters == 2 and not r1.converged


def test_breakdown_on_indefinite_operator():
    A = np.diag([1.0, -1.0])
    res = cg.pcg(lambda v: A @ v, np.array([1.0, 1.0]), 1e-8, 10)
    assert res.breakdown and not res.converged
