"""Seeded synthetic PINN workloads shared by the oracle, the tests and the benchmark.

This module holds problem *data* only: collocation points and their kind, Monte Carlo quadrature
weights, the source / boundary / initial values of the manufactured solutions, Glorot-uniform initial
parameters and Gaussian test matrices. It contains none of the method's arithmetic (no network
evaluation, no Jacobian, no Gramian, no sketch, no CG), so both the FP64 oracle and the GPU path can
read the same inputs without sharing any computation.

Point sets follow the paper's Monte Carlo quadrature (uniform points drawn once and kept fixed,
experimental details of the appendix): interior weights are meas(domain)/N_interior and boundary
weights meas(boundary)/N_boundary, so that sum_r w_r res_r^2 approximates the L2 norms of the
least-squares energy of the Poisson problem (Section 5.1.1) and of the heat problem (Section 5.1.2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

KIND_INTERIOR = 0   # PDE residual row
KIND_BOUNDARY = 1   # Dirichlet row: res = u - g
KIND_INITIAL = 2    # initial-condition row (heat): res = u - g

PDE_POISSON = 0     # interior res = Laplace(u) + f      (-Laplace(u) = f)
PDE_HEAT = 1        # interior res = u_t - Laplace_x(u) - f (last input coordinate is time)
PDE_NAVIER_STOKES = 2  # steady incompressible flow, velocity and pressure networks (rows below)

# rows of the Navier-Stokes problem (Section 5.1.3, eq. navier_residual): an interior point gives the
# two momentum rows and the continuity row, a boundary point one Dirichlet row per velocity component
KIND_NS_MOMENTUM_X = 3  # -nu Laplace u_1 + (u . grad) u_1 + dp/dx - f
KIND_NS_MOMENTUM_Y = 4  # -nu Laplace u_2 + (u . grad) u_2 + dp/dy - f
KIND_NS_CONTINUITY = 5  # div u
KIND_NS_BOUNDARY_U = 6  # u_1 - g
KIND_NS_BOUNDARY_V = 7  # u_2 - g

# purposes for independent random streams
_P_THETA, _P_INTERIOR, _P_BOUNDARY, _P_INITIAL, _P_OMEGA, _P_PROBE, _P_SHAPES, _P_EVAL, _P_THETA_P = range(9)


@dataclasses.dataclass
class Problem:
    """One PINN least-squares problem: network shape plus the fixed quadrature data."""

    name: str
    pde: int                      # PDE_POISSON or PDE_HEAT
    widths: tuple                 # (d, n_1, ..., n_L, 1)
    X: np.ndarray                 # (N, d) float64 collocation points
    kind: np.ndarray              # (N,) int8 row kind
    w: np.ndarray                 # (N,) float64 quadrature weights
    f: np.ndarray                 # (N,) float64 source on interior rows (0 elsewhere)
    g: np.ndarray                 # (N,) float64 target value on boundary / initial rows (0 elsewhere)
    dtype: str = "f64"            # working precision of the GPU path ("f64" | "f32")
    ell: int = 100                # sketch size
    lam: Optional[float] = None   # fixed damping, or None for the adaptive rule
    sketch_dtype: str = "f64"     # "f64" | "f32" | "bf16"
    seed: int = 0
    recompute: bool = False       # products with J_w recomputed from theta instead of a stored J_w
    ell_max: Optional[int] = None # adaptive sketch size up to ell_max (None: ell fixed)
    dell: int = 20                # rank increase of the adaptive rule
    maxit: Optional[int] = None   # PCG iteration cap (None: driver.NGD's default)
    solution: str = ""            # manufactured solution ("sinprod", "sinsum", "heat") for evaluation
    nu: float = 0.0               # viscosity (Navier-Stokes rows only)
    damping: str = "rule"         # "rule" (Section 4.3) or "lm" (Levenberg-Marquardt, Section 5.1.3)

    @property
    def n_rows(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.X.shape[1])

    @property
    def n_params(self) -> int:
        if self.pde == PDE_NAVIER_STOKES:
            return ns_num_params(self.widths)
        return num_params(self.widths)

    def cast(self, dtype: str) -> "Problem":
        """The same problem with all floating data rounded to `dtype` and promoted back to float64.

        Comparing the FP64 oracle against a reduced-precision GPU run on the rounded inputs isolates
        the arithmetic error of the GPU path from the rounding of its inputs.
        """
        if dtype == "f64":
            return self
        np_t = {"f32": np.float32}[dtype]
        rd = lambda a: a.astype(np_t).astype(np.float64)
        return dataclasses.replace(self, X=rd(self.X), w=rd(self.w), f=rd(self.f), g=rd(self.g))


def num_params(widths: Sequence[int]) -> int:
    """p = sum_l (n_l n_{l-1} + n_l) (Section 2.3)."""
    return int(sum(a * b + b for a, b in zip(widths[:-1], widths[1:])))


def pressure_widths(widths: Sequence[int]) -> tuple:
    """The pressure network of the Navier-Stokes problem: the velocity network's input and hidden
    widths with one output (Section 5.1.3 uses two such networks with three hidden layers of 45)."""
    return tuple(int(v) for v in widths[:-1]) + (1,)


def ns_num_params(widths: Sequence[int]) -> int:
    """p of theta = [theta_u, theta_p] (Section 5.1.3): both networks' parameters."""
    return num_params(widths) + num_params(pressure_widths(widths))


def _rng(seed: int, purpose: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(purpose)]))


def glorot_theta(widths: Sequence[int], seed: int) -> np.ndarray:
    """Flat parameters [W_1, b_1, ..., W_{L+1}, b_{L+1}] (W row-major, out x in), Glorot-uniform
    weights U(-a, a) with a = sqrt(6 / (n_in + n_out)) and zero biases."""
    rng = _rng(seed, _P_THETA)
    parts = []
    for n_in, n_out in zip(widths[:-1], widths[1:]):
        a = math.sqrt(6.0 / (n_in + n_out))
        parts.append(rng.uniform(-a, a, size=(n_out, n_in)).ravel())
        parts.append(np.zeros(n_out))
    return np.concatenate(parts)


def ns_glorot_theta(widths: Sequence[int], seed: int) -> np.ndarray:
    """theta = [theta_u, theta_p] for the Navier-Stokes problem, each network Glorot-uniform as
    glorot_theta, the pressure network from its own stream."""
    rng = _rng(seed, _P_THETA_P)
    parts = [glorot_theta(widths, seed)]
    pw = pressure_widths(widths)
    for n_in, n_out in zip(pw[:-1], pw[1:]):
        a = math.sqrt(6.0 / (n_in + n_out))
        parts.append(rng.uniform(-a, a, size=(n_out, n_in)).ravel())
        parts.append(np.zeros(n_out))
    return np.concatenate(parts)


def gaussian_omega(n_params: int, ell: int, seed: int, counter: int = 0) -> np.ndarray:
    """Standard normal test matrix Omega, shape (p, ell), for sketch number `counter`."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), _P_OMEGA, int(counter)]))
    return rng.standard_normal((n_params, ell))


def probe_vectors(n: int, k: int, seed: int) -> np.ndarray:
    """k standard normal probe vectors of length n, shape (n, k)."""
    return _rng(seed, _P_PROBE).standard_normal((n, k))


# ----------------------------------------------------------------------------------------------
# manufactured solutions
# ----------------------------------------------------------------------------------------------

def _sinprod(X: np.ndarray) -> np.ndarray:
    return np.prod(np.sin(np.pi * X), axis=1)


def _sinsum(X: np.ndarray) -> np.ndarray:
    return np.sum(np.sin(np.pi * X), axis=1)


def _box_boundary(rng, n: int, d: int) -> np.ndarray:
    """n points uniform on the boundary of [0,1]^d: a face (2d of them) uniformly, then uniform on it."""
    X = rng.uniform(0.0, 1.0, size=(n, d))
    face = rng.integers(0, 2 * d, size=n)
    X[np.arange(n), face // 2] = (face % 2).astype(np.float64)
    return X


def _assemble(name, pde, widths, blocks, **kw) -> Problem:
    X = np.concatenate([b[0] for b in blocks])
    kind = np.concatenate([np.full(len(b[0]), b[1], np.int8) for b in blocks])
    w = np.concatenate([np.full(len(b[0]), b[2]) for b in blocks])
    f = np.concatenate([b[3] for b in blocks])
    g = np.concatenate([b[4] for b in blocks])
    return Problem(name=name, pde=pde, widths=tuple(int(v) for v in widths), X=X, kind=kind, w=w,
                   f=f, g=g, **kw)


def poisson2d_grid(widths=(2, 32, 32, 1), n_side=30, seed=0, dtype="f64", ell=100, lam=1e-6,
                   sketch_dtype="f64") -> Problem:
    """2D Poisson on [0,1]^2, u* = sin(pi x) sin(pi y), f = 2 pi^2 u*, g = 0.

    Interior: the n_side^2 cell centres of a uniform grid. Boundary: n_side points per edge at the
    edge-cell midpoints (no corners, no duplicates)."""
    c = (np.arange(n_side) + 0.5) / n_side
    xx, yy = np.meshgrid(c, c, indexing="ij")
    Xi = np.stack([xx.ravel(), yy.ravel()], axis=1)
    z, o = np.zeros(n_side), np.ones(n_side)
    Xb = np.concatenate([np.stack([c, z], 1), np.stack([c, o], 1), np.stack([z, c], 1), np.stack([o, c], 1)])
    ni, nb = len(Xi), len(Xb)
    blocks = [(Xi, KIND_INTERIOR, 1.0 / ni, 2 * np.pi ** 2 * _sinprod(Xi), np.zeros(ni)),
              (Xb, KIND_BOUNDARY, 4.0 / nb, np.zeros(nb), np.zeros(nb))]
    return _assemble("poisson2d_grid", PDE_POISSON, widths, blocks, dtype=dtype, ell=ell, lam=lam,
                     sketch_dtype=sketch_dtype, seed=seed, solution="sinprod")


def poisson_random(d=2, widths=(2, 64, 64, 64, 1), n_interior=4096, n_boundary=512, seed=0,
                   dtype="f32", ell=400, lam=None, sketch_dtype="f32", solution="sinprod") -> Problem:
    """Poisson on [0,1]^d with uniform random interior and boundary points.

    solution="sinprod": u* = prod_i sin(pi x_i), f = d pi^2 u*, g = u* on the boundary (= 0).
    solution="sinsum":  u* = sum_i sin(pi x_i),  f = pi^2 u*,   g = u* on the boundary."""
    rng_i, rng_b = _rng(seed, _P_INTERIOR), _rng(seed, _P_BOUNDARY)
    Xi = rng_i.uniform(0.0, 1.0, size=(n_interior, d))
    Xb = _box_boundary(rng_b, n_boundary, d)
    if solution == "sinprod":
        fi, gb = d * np.pi ** 2 * _sinprod(Xi), _sinprod(Xb)
    elif solution == "sinsum":
        fi, gb = np.pi ** 2 * _sinsum(Xi), _sinsum(Xb)
    else:
        raise ValueError(solution)
    blocks = [(Xi, KIND_INTERIOR, 1.0 / n_interior, fi, np.zeros(n_interior)),
              (Xb, KIND_BOUNDARY, 2.0 * d / n_boundary, np.zeros(n_boundary), gb)]
    return _assemble(f"poisson{d}d_random", PDE_POISSON, widths, blocks, dtype=dtype, ell=ell,
                     lam=lam, sketch_dtype=sketch_dtype, seed=seed, solution=solution)


def heat2d(widths=(3, 64, 64, 64, 64, 1), n_interior=8192, n_lateral=1024, n_initial=1024, seed=0,
           dtype="f32", ell=400, lam=None, sketch_dtype="f32") -> Problem:
    """Heat equation u_t = Laplace_x u on [0,1]^2 x [0,1]; u* = exp(-2 pi^2 t) sin(pi x) sin(pi y).

    Inputs are (x, y, t). Lateral rows have g = 0, initial rows (t = 0) have g = sin(pi x) sin(pi y)."""
    rng_i, rng_b, rng_0 = _rng(seed, _P_INTERIOR), _rng(seed, _P_BOUNDARY), _rng(seed, _P_INITIAL)
    Xi = rng_i.uniform(0.0, 1.0, size=(n_interior, 3))
    Xl = np.concatenate([_box_boundary(rng_b, n_lateral, 2), rng_b.uniform(0, 1, (n_lateral, 1))], 1)
    X0 = np.concatenate([rng_0.uniform(0, 1, (n_initial, 2)), np.zeros((n_initial, 1))], 1)
    blocks = [(Xi, KIND_INTERIOR, 1.0 / n_interior, np.zeros(n_interior), np.zeros(n_interior)),
              (Xl, KIND_BOUNDARY, 4.0 / n_lateral, np.zeros(n_lateral), np.zeros(n_lateral)),
              (X0, KIND_INITIAL, 1.0 / n_initial, np.zeros(n_initial), _sinprod(X0[:, :2]))]
    return _assemble("heat2d", PDE_HEAT, widths, blocks, dtype=dtype, ell=ell, lam=lam,
                     sketch_dtype=sketch_dtype, seed=seed, solution="heat")


def exact_solution(solution: str, X: np.ndarray) -> tuple:
    """Value and gradient (over all inputs) of a manufactured solution at the points X (n x d)."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    s, c = np.sin(np.pi * X), np.cos(np.pi * X)
    if solution == "sinprod":
        u = np.prod(s, axis=1)
        grad = np.empty((n, d))
        for j in range(d):
            grad[:, j] = np.pi * c[:, j] * np.prod(np.delete(s, j, axis=1), axis=1)
        return u, grad
    if solution == "sinsum":
        return np.sum(s, axis=1), np.pi * c
    if solution == "heatcos":  # (cos(pi x) + cos(pi y) + cos(pi z)) exp(-pi^2 t / 4), inputs (x, y, z, t)
        e = np.exp(-np.pi ** 2 * X[:, 3] / 4.0)
        u = (c[:, 0] + c[:, 1] + c[:, 2]) * e
        grad = np.stack([-np.pi * s[:, 0] * e, -np.pi * s[:, 1] * e, -np.pi * s[:, 2] * e,
                         -np.pi ** 2 / 4.0 * u], axis=1)
        return u, grad
    if solution == "heat":  # exp(-2 pi^2 t) sin(pi x) sin(pi y), inputs (x, y, t)
        e = np.exp(-2.0 * np.pi ** 2 * X[:, 2])
        u = e * s[:, 0] * s[:, 1]
        grad = np.stack([np.pi * e * c[:, 0] * s[:, 1], np.pi * e * s[:, 0] * c[:, 1],
                         -2.0 * np.pi ** 2 * u], axis=1)
        return u, grad
    raise ValueError(solution)


def evaluation_set(prob: Problem, n: int = 100_000, seed: int = 0) -> tuple:
    """n uniform random points of the problem's domain [0,1]^d (the paper's evaluation sets: 100,000
    random points, appendix table of discretisations) with the exact solution and its gradient there:
    (X, u, grad u)."""
    X = _rng(seed, _P_EVAL).uniform(0.0, 1.0, size=(n, prob.d))
    u, grad = exact_solution(prob.solution, X)
    return X, u, grad


def heat3d_paper(widths=(4, 64, 64, 64, 1), n_interior=10000, n_boundary=1000, seed=0, dtype="f64", ell=20,
                 sketch_dtype="f64") -> Problem:
    """The paper's heat equation in 3+1D (Section 5.1.2): u_t - Laplace u = f on (0,1)^3 x (0,1) with
    u* = (cos(pi x) + cos(pi y) + cos(pi z)) exp(-pi^2 t / 4), so f = 3 pi^2 / 4 u*; Dirichlet data
    g = u* on the lateral boundary and the initial value u*(., 0). Inputs (x, y, z, t).

    The n_boundary random boundary points are split between the lateral boundary and t = 0 in
    proportion to their measures (6 : 1); weights are measure / count as elsewhere."""
    rng_i, rng_b, rng_0 = _rng(seed, _P_INTERIOR), _rng(seed, _P_BOUNDARY), _rng(seed, _P_INITIAL)
    n_init = int(round(n_boundary / 7.0))
    n_lat = n_boundary - n_init
    Xi = rng_i.uniform(0.0, 1.0, size=(n_interior, 4))
    Xl = np.concatenate([_box_boundary(rng_b, n_lat, 3), rng_b.uniform(0, 1, (n_lat, 1))], 1)
    X0 = np.concatenate([rng_0.uniform(0, 1, (n_init, 3)), np.zeros((n_init, 1))], 1)
    ui, _ = exact_solution("heatcos", Xi)
    ul, _ = exact_solution("heatcos", Xl)
    u0, _ = exact_solution("heatcos", X0)
    blocks = [(Xi, KIND_INTERIOR, 1.0 / n_interior, 0.75 * np.pi ** 2 * ui, np.zeros(n_interior)),
              (Xl, KIND_BOUNDARY, 6.0 / n_lat, np.zeros(n_lat), ul),
              (X0, KIND_INITIAL, 1.0 / n_init, np.zeros(n_init), u0)]
    return _assemble("heat3d_paper", PDE_HEAT, widths, blocks, dtype=dtype, ell=ell, lam=None,
                     sketch_dtype=sketch_dtype, seed=seed, solution="heatcos")


# Kovasznay flow (Section 5.1.3) on (-1/2, 1) x (-1/2, 3/2)
_KOV_BOX = ((-0.5, 1.0), (-0.5, 1.5))


def kovasznay_lambda(nu: float) -> float:
    """lambda = 1/(2 nu) - sqrt(1/(4 nu^2) + 4 pi^2) of the Kovasznay solution."""
    return 1.0 / (2.0 * nu) - math.sqrt(1.0 / (4.0 * nu * nu) + 4.0 * math.pi ** 2)


def kovasznay_solution(X: np.ndarray, nu: float = 1.0 / 40.0) -> tuple:
    """The exact Kovasznay flow at the points X (n x 2): velocity (n, 2), its gradient (n, 2, 2) with
    [k, j] = d u_k / d x_j, and the pressure (n,) normalised to mean zero over the domain."""
    X = np.asarray(X, dtype=np.float64)
    lam = kovasznay_lambda(nu)
    x, y = X[:, 0], X[:, 1]
    e = np.exp(lam * x)
    c, s = np.cos(2 * np.pi * y), np.sin(2 * np.pi * y)
    u = np.stack([1.0 - e * c, lam / (2 * np.pi) * e * s], axis=1)
    grad = np.empty((X.shape[0], 2, 2))
    grad[:, 0, 0] = -lam * e * c
    grad[:, 0, 1] = 2 * np.pi * e * s
    grad[:, 1, 0] = lam * lam / (2 * np.pi) * e * s
    grad[:, 1, 1] = lam * e * c
    (x0, x1), (y0, y1) = _KOV_BOX
    # mean of 1/2 (1 - exp(2 lambda x)) over the box (it does not depend on y)
    mean = 0.5 * (1.0 - (math.exp(2 * lam * x1) - math.exp(2 * lam * x0)) / (2 * lam * (x1 - x0)))
    p = 0.5 * (1.0 - np.exp(2 * lam * x)) - mean
    return u, grad, p


def _kovasznay_boundary(rng, n: int) -> np.ndarray:
    """n points uniform on the boundary of the Kovasznay box: an edge with probability proportional to
    its length, then a uniform point on it."""
    (x0, x1), (y0, y1) = _KOV_BOX
    lx, ly = x1 - x0, y1 - y0
    t = rng.uniform(0.0, 2 * (lx + ly), size=n)
    X = np.empty((n, 2))
    for i, ti in enumerate(t):
        if ti < lx:
            X[i] = (x0 + ti, y0)
        elif ti < lx + ly:
            X[i] = (x1, y0 + ti - lx)
        elif ti < 2 * lx + ly:
            X[i] = (x1 - (ti - lx - ly), y1)
        else:
            X[i] = (x0, y1 - (ti - 2 * lx - ly))
    return X


def kovasznay(widths=(2, 45, 45, 45, 2), n_interior=10000, n_boundary=1000, nu=1.0 / 40.0, seed=0,
              dtype="f64", ell=20, sketch_dtype="f64") -> Problem:
    """The paper's Kovasznay flow (Section 5.1.3, Re = 1/nu = 40, f = 0) as Navier-Stokes rows.

    Uniform random interior and boundary points of (-1/2, 1) x (-1/2, 3/2). Every interior point gives
    three rows (momentum x, momentum y, continuity) with weight area / n_interior, every boundary point
    two rows (u_1 - g_1, u_2 - g_2, g the exact velocity) with weight perimeter / n_boundary. `widths` is
    the velocity network (two outputs); the pressure network has the same hidden widths and one output."""
    rng_i, rng_b = _rng(seed, _P_INTERIOR), _rng(seed, _P_BOUNDARY)
    (x0, x1), (y0, y1) = _KOV_BOX
    Xi = np.stack([rng_i.uniform(x0, x1, n_interior), rng_i.uniform(y0, y1, n_interior)], axis=1)
    Xb = _kovasznay_boundary(rng_b, n_boundary)
    ub, _, _ = kovasznay_solution(Xb, nu)
    wi = (x1 - x0) * (y1 - y0) / n_interior
    wb = 2 * ((x1 - x0) + (y1 - y0)) / n_boundary
    zi, zb = np.zeros(n_interior), np.zeros(n_boundary)
    blocks = [(Xi, KIND_NS_MOMENTUM_X, wi, zi, zi), (Xi, KIND_NS_MOMENTUM_Y, wi, zi, zi),
              (Xi, KIND_NS_CONTINUITY, wi, zi, zi),
              (Xb, KIND_NS_BOUNDARY_U, wb, zb, ub[:, 0]), (Xb, KIND_NS_BOUNDARY_V, wb, zb, ub[:, 1])]
    return _assemble("kovasznay", PDE_NAVIER_STOKES, widths, blocks, dtype=dtype, ell=ell, lam=None,
                     sketch_dtype=sketch_dtype, seed=seed, solution="kovasznay", nu=float(nu), damping="lm")


def kovasznay_evaluation_set(nu: float = 1.0 / 40.0, n: int = 100_000, seed: int = 0) -> tuple:
    """n uniform random points of the Kovasznay box with the exact velocity and its gradient there:
    (X, u (n, 2), grad u (n, 2, 2))."""
    (x0, x1), (y0, y1) = _KOV_BOX
    rng = _rng(seed, _P_EVAL)
    X = np.stack([rng.uniform(x0, x1, n), rng.uniform(y0, y1, n)], axis=1)
    u, grad, _ = kovasznay_solution(X, nu)
    return X, u, grad


# ----------------------------------------------------------------------------------------------
# named configurations
# ----------------------------------------------------------------------------------------------

def config(name: str, seed: int = 0) -> Problem:
    """The named workloads.

    c1: 2D Poisson, 2-32-32-1, 30x30 grid + 120 boundary points, FP64, lambda = 1e-6, ell = 100.
    c2: 2D Poisson, 2-64-64-64-1, 4,096 + 512 random points, FP32, ell = 400, adaptive damping.
    c3: 5D Poisson (u* = sum sin), 5-128-128-128-1, 16,384 + 2,048 points, BF16 sketch, ell = 800.
    c4: 2+1D heat, 3-64-64-64-64-1, 8,192 + 1,024 lateral + 1,024 initial points, FP32, ell = 400,
        J_w recomputed (never stored).
    paper3d: the paper's 3D Poisson setup (Section 5.1.1 and the experimental setup of Section 5):
        3-64-64-64-1 tanh (P = 8,641), 10,000 + 1,000 random points, FP64, u* = prod sin(pi x_i),
        adaptive sketch size from 20 in steps of 20 up to 500, at most 20 PCG iterations.
    paper_heat: the paper's heat equation in 3+1D (Section 5.1.2), 4-64-64-64-1 tanh (P = 8,705), 10,000 +
        1,000 random points, FP64, the same solver settings as paper3d.
    paper_ns: the paper's Kovasznay flow (Section 5.1.3), velocity 2-45-45-45-2 and pressure 2-45-45-45-1
        tanh networks (P = 8,688), 10,000 + 1,000 random points (32,000 rows), FP64, the same sketch-size
        settings as paper3d.
    """
    if name == "paper_ns":
        return dataclasses.replace(kovasznay(seed=seed), name="paper_ns", ell_max=500, dell=20, maxit=20)
    if name == "paper_heat":
        return dataclasses.replace(heat3d_paper(seed=seed), name="paper_heat", ell_max=500, dell=20, maxit=20)
    if name == "paper3d":
        prob = poisson_random(d=3, widths=(3, 64, 64, 64, 1), n_interior=10000, n_boundary=1000, seed=seed,
                              dtype="f64", ell=20, sketch_dtype="f64", solution="sinprod")
        return dataclasses.replace(prob, name="paper3d", ell_max=500, dell=20, maxit=20)
    if name == "c1":
        return poisson2d_grid(seed=seed)
    if name == "c2":
        return poisson_random(seed=seed)
    if name == "c3":
        return poisson_random(d=5, widths=(5, 128, 128, 128, 1), n_interior=16384, n_boundary=2048,
                              seed=seed, ell=800, sketch_dtype="bf16", solution="sinsum")
    if name == "c4":
        return dataclasses.replace(heat2d(seed=seed), recompute=True)
    raise KeyError(name)


def batch_instances(n=32, seed=0, widths=(32, 48, 64, 96), depths=(2, 3, 4), n_min=1024, n_max=8192,
                    ells=(50, 100, 200, 400), dims=(2, 3)) -> list:
    """The batched workload: n independent Poisson problems on [0,1]^d (d from `dims`) with
    u* = prod sin(pi x_i); per problem a hidden width from `widths` (all hidden layers alike), a depth
    from `depths`, N_int uniform in [n_min, n_max] plus N_int // 8 boundary points, and ell from `ells`,
    all drawn from one seeded stream; FP32. Problem i uses data seed 1000 * seed + i."""
    rng = _rng(seed, _P_SHAPES)
    out = []
    for i in range(n):
        d = int(rng.choice(dims))
        wdt = int(rng.choice(widths))
        depth = int(rng.choice(depths))
        n_int = int(rng.integers(n_min, n_max + 1))
        ell = int(rng.choice(ells))
        prob = poisson_random(d=d, widths=(d,) + (wdt,) * depth + (1,), n_interior=n_int, n_boundary=n_int // 8,
                              seed=1000 * seed + i, dtype="f32", ell=ell, sketch_dtype="f32")
        out.append(dataclasses.replace(prob, name=f"batch{i}"))
    return out


def small_problem(pde=PDE_POISSON, d=2, widths=(2, 8, 8, 1), n_interior=24, n_boundary=12, seed=0,
                  dtype="f64", ell=10, lam=1e-3) -> Problem:
    """Tiny instances for brute-force pins (random points, sinprod manufactured data)."""
    if pde == PDE_HEAT:
        return heat2d(widths=widths, n_interior=n_interior, n_lateral=n_boundary // 2,
                      n_initial=n_boundary - n_boundary // 2, seed=seed, dtype=dtype, ell=ell, lam=lam,
                      sketch_dtype=dtype)
    return poisson_random(d=d, widths=widths, n_interior=n_interior, n_boundary=n_boundary, seed=seed,
                          dtype=dtype, ell=ell, lam=lam, sketch_dtype=dtype)
