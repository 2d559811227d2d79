"""Natural gradient descent loop (Alg. 1) on top of the C ABI.

One step: residuals, Jacobian and gradient; the direction from matrix-free PCG (Alg. 3) with the
Nystrom builder of Alg. 4 at a fixed sketch size, or plain CG; the damping rule; Armijo backtracking
and the update. Every numerical operation is a libngd call; the host only moves a few scalars
(loss, largest eigenvalue estimate, Armijo decisions).

Damping (Section 4.3 and the experimental setup of Section 5): mu = max(gamma eps lam1_hat, 1e-4 L^2)
with gamma = 10 and eps the unit roundoff of the working precision, unless a fixed mu is given; the
rule runs in the library (ngd_pcg_solve_damped, ngd_damping). Plain CG, RPCholNGD and NGD full take
lam1_hat from 4 power iterations.

Levenberg-Marquardt damping (damping="lm", the Navier-Stokes experiment of Section 5.1.3): the first
step takes mu from the rule above, every later one from ngd_lm_damping's update after the previous
step (gain ratio of the actual over the Gauss-Newton model's decrease), never below gamma eps lam1_hat.

Sketch size: fixed, or adaptive as in Alg. 4 (Section 4.3) when a maximum is given: after each step
ngd_next_rank gives the next size (grow by dell while lam_hat_ell > 10 mu, else the first index with
lam_hat_i < 10 mu plus one, never above ell_max).

Solvers: "nystrom" (Alg. 3 with the Nystrom preconditioner of Alg. 4), "cg" (no preconditioner),
"rpchol" (Alg. 5) and "direct" (NGD full, Alg. 2: the explicit Gramian and its Cholesky factor).
"""
from __future__ import annotations

import dataclasses
import types
from typing import Optional

import numpy as np
import torch

from .api import Batch, Problem, Recompute

EPS = {"f64": 2.0 ** -52, "f32": 2.0 ** -23}


@dataclasses.dataclass
class StepReport:
    loss: float
    mu: float
    lam1: float
    iters: int
    rel_res: float
    converged: bool
    alpha: float
    loss_new: float
    rank: int = -1


class NGD:
    def __init__(self, data, theta0, *, solver="nystrom", ell=None, sketch_dtype=None, rtol=1e-6,
                 maxit=None, lam=None, gamma=10.0, seed=0, power_v0=None, dtype=None, recompute=None,
                 ell_max=None, dell=None, rank_offset=1, test_matrix="gaussian", damping=None,
                 rpchol_form="woodbury"):
        # adaptive sketch size when a maximum is given (here or by the problem)
        self.ell_max = ell_max if ell_max is not None else getattr(data, "ell_max", None)
        self.dell = int(dell if dell is not None else getattr(data, "dell", 20))
        self.rank_offset = int(rank_offset)
        # RPCholNGD (Alg. 5) keeps one more row for the preconditioner's trailing zero pair
        max_ell = self.ell_max or ell or getattr(data, "ell", 1)
        if solver == "rpchol":
            self.ell_max = int(self.ell_max or ell or getattr(data, "ell", 1))
            max_ell = self.ell_max + 1
        self.gp = Problem(data, dtype=dtype, max_ell=max_ell)
        gp = self.gp
        self.solver = solver
        if test_matrix not in ("gaussian", "sampling"):
            raise ValueError("test_matrix must be 'gaussian' or 'sampling'")
        # sampling: Omega = identity columns drawn with probability proportional to diag(G) (Section 5)
        self.test_matrix = test_matrix
        self.diag = None
        if self.ell_max is not None:
            self.ell_max = min(int(self.ell_max), gp.P - (1 if solver == "rpchol" else 0))
        self.rp_block = 20  # block size of the block RPCholesky (experimental setup of Section 5)
        if rpchol_form not in ("woodbury", "svd"):
            raise ValueError("rpchol_form must be 'woodbury' or 'svd'")
        self.rpchol_form = rpchol_form  # Woodbury-Cholesky (eq. rpchol_precond) or the SVD form
        self.Ft = None
        self.ell = min(int(ell or data.ell), gp.P, self.ell_max or gp.P)
        self.sketch_dtype = sketch_dtype or getattr(data, "sketch_dtype", None)
        if gp.dtype_name == "f64":
            self.sketch_dtype = "f64"
        self.rtol = rtol
        if maxit is None:
            maxit = getattr(data, "maxit", None)
        self.maxit = maxit if maxit is not None else (gp.P if solver == "cg" else 1000)
        self.lam = lam if lam is not None else getattr(data, "lam", None)
        self.damping = damping or getattr(data, "damping", "rule")
        if self.damping not in ("rule", "lm"):
            raise ValueError("damping must be 'rule' or 'lm'")
        self.mu_lm = None  # the Levenberg-Marquardt damping for the next step
        self.gamma = gamma
        self.seed = seed
        self.eps = EPS[gp.dtype_name]
        self.theta = gp.theta(theta0)
        # recompute mode (J_w never stored; products by the tangent / adjoint kernels): asked for, or
        # the problem's own setting
        self.recompute = bool(getattr(data, "recompute", False) if recompute is None else recompute)
        self.J = None if self.recompute else gp.new_jacobian()
        if power_v0 is None:
            power_v0 = np.random.default_rng(np.random.SeedSequence([seed, 99])).standard_normal(gp.P)
        self.v0 = torch.as_tensor(power_v0, dtype=torch.float64, device=gp.device)
        # pinned landing slots of the loss and of lambda_hat_1: their copies ride the stream and are
        # read after the next synchronisation (the power iteration's or the solve's)
        self.loss_host = torch.empty(1, dtype=torch.float64, pin_memory=True)
        self.lam1_host = torch.empty(1, dtype=torch.float64, pin_memory=True)
        self.loss_np, self.lam1_np = self.loss_host.numpy(), self.lam1_host.numpy()
        # device slots of the power method's estimate and of the damping (plain CG, RPCholNGD, NGD full)
        self.lam1_dev = torch.zeros(1, dtype=torch.float64, device=gp.device)
        self.mu_dev = torch.zeros(1, dtype=torch.float64, device=gp.device)
        if solver not in ("nystrom", "cg", "rpchol", "direct"):
            raise ValueError("solver must be 'nystrom', 'cg', 'rpchol' or 'direct'")
        # per-step device buffers, reused: residuals, gradient, loss and the search direction
        self.bufs = None
        self.pc = None
        self.d = torch.empty(gp.P, dtype=torch.float64, device=gp.device)
        self.k = 0

    def step(self) -> StepReport:
        gp = self.gp
        r, J, grad, loss = gp.residual_jacobian(self.theta, self.J, out=self.bufs)
        self.bufs = (r, grad, loss)
        if self.recompute:
            J = Recompute(self.theta)
        self.loss_host.copy_(loss, non_blocking=True)
        if self.solver == "nystrom":
            # sketch, damping (Section 4.3) and solve with no host round trip in between: the sketch
            # returns no summary and the solve takes mu on the device
            ell = self.ell
            cols = None
            if self.test_matrix == "sampling":
                self.diag = gp.gramian_diagonal(J, out=self.diag)
                cols, _ = gp.sample_pivots(self.diag, ell, seed=self.seed, counter=self.k)
            pc = gp.nystrom_sketch(J, ell, seed=self.seed, counter=self.k, sketch_dtype=self.sketch_dtype,
                                   want_info=False, out=self.pc, cols=cols)
            self.pc = pc
            self.lam1_host.copy_(pc.lam_hat[:1], non_blocking=True)
            fixed = self.lam if self.lam is not None else self.mu_lm
            if fixed is not None:
                out = gp.pcg_solve(J, grad, fixed, precond=pc, rtol=self.rtol, maxit=self.maxit, out=self.d)
                mu = fixed
            else:
                out = gp.pcg_solve(J, grad, None, precond=pc, rtol=self.rtol, maxit=self.maxit,
                                   damping=(self.gamma * self.eps, 1e-4, loss), out=self.d)
                mu = out.mu
            lam1 = float(self.lam1_np[0])
            L0 = float(self.loss_np[0])
            if self.ell_max is not None:  # Alg. 4's next sketch size, evaluated by the library
                self.ell = gp.next_rank(pc.lam_hat, ell, mu, self.dell, self.rank_offset, self.ell_max)
        else:
            # plain CG, RPCholNGD (Alg. 5) or NGD full (Alg. 2): lambda_1 from 4 power iterations, then the
            # damping rule on the device
            lam1 = gp.power_lambda_max(J, self.v0, 4, out=self.lam1_dev)
            L0 = float(self.loss_np[0])
            if self.lam is not None or self.mu_lm is not None:
                mu = self.lam if self.lam is not None else self.mu_lm
            else:
                _, mu = gp.damping(self.lam1_dev, loss, self.gamma * self.eps, 1e-4, out=self.mu_dev)
            pc = None
            if self.solver == "rpchol":
                # F with G ~ F F^T until the residual trace is below mu p; P = F F^T + mu I
                self.diag = gp.gramian_diagonal(J, out=self.diag)
                self.Ft, rank, _ = gp.rpcholesky(J, self.diag, self.ell_max, self.rp_block, seed=self.seed,
                                                 counter=self.k, eps=mu * gp.P, Ft=self.Ft)
                # the Woodbury-Cholesky form the paper adopts (eq. rpchol_precond), for this step's mu
                pc = gp.rpchol_precond(self.Ft, rank, mu=mu if self.rpchol_form == "woodbury" else None)
                self.last_rank = rank
            if self.solver == "direct":
                d = gp.direct_solve(J, grad, mu, out=self.d)
                out = types.SimpleNamespace(d=d, iters=0, rel_res=0.0, converged=True)
            else:
                out = gp.pcg_solve(J, grad, mu, precond=pc, rtol=self.rtol, maxit=self.maxit, out=self.d)
        _, alpha, L1 = gp.line_search(self.theta, out.d, grad, L0, theta_out=self.theta)
        if self.damping == "lm" and self.lam is None:
            # J and grad still belong to the step's starting point
            self.mu_lm, _ = gp.lm_damping(J, out.d, grad, alpha, L0, L1, mu, self.gamma * self.eps * float(lam1))
        self.k += 1
        rank = ell if self.solver == "nystrom" else (self.last_rank if self.solver == "rpchol" else -1)
        return StepReport(L0, mu, lam1, out.iters, out.rel_res, out.converged, alpha, L1, rank)



class BatchNGD:
    """NGD (Alg. 1) on many independent problems at once: residuals and Jacobians of all problems in
    one batched launch, every problem's Nystrom sketch (Alg. 4/6, its own ell) side by side with no host
    round trip, each problem's damping on the device and one batched PCG solve for all, then every
    problem's Armijo step in one batched line search. Plain CG ("cg") takes each problem's lam1_hat from
    4 power iterations."""

    def __init__(self, datas, thetas0, *, solver="nystrom", rtol=1e-6, gamma=10.0, seed=0):
        self.batch = Batch(datas, dtype="f32")
        self.solver = solver
        self.rtol = rtol
        self.gamma = gamma
        self.seed = seed
        self.eps = EPS["f32"]
        self.ells = [min(int(d.ell), m.P) for d, m in zip(datas, self.batch.members)]
        self.thetas = [m.theta(t) for m, t in zip(self.batch.members, thetas0)]
        self.Js = [m.new_jacobian() for m in self.batch.members]
        self.pcs = None
        self.k = 0

    def step(self):
        b = self.batch
        _, grads, losses = b.residual_jacobian(self.thetas, self.Js)
        if self.solver == "nystrom":
            self.pcs = b.nystrom_sketch(self.Js, self.ells, seed=self.seed, counter=self.k, sketch_dtype="f32",
                                        outs=self.pcs)
            outs = b.pcg_solve_damped(self.Js, grads, self.gamma * self.eps, 1e-4, losses, self.pcs, rtol=self.rtol,
                                      maxit=1000)
        else:
            mus = []
            for m, J, loss in zip(b.members, self.Js, losses):
                l1 = torch.empty(1, dtype=torch.float64, device=m.device)
                m.power_lambda_max(J, torch.ones(m.P, dtype=torch.float64, device=m.device), 4, out=l1)
                mus.append(m.damping(l1, loss, self.gamma * self.eps, 1e-4)[1])
            outs = b.pcg_solve(self.Js, grads, mus, None, rtol=self.rtol, maxit=max(m.P for m in b.members))
        L0 = torch.cat(losses).cpu().numpy()
        _, _, news = b.line_search(self.thetas, [o.d for o in outs], grads, L0, theta_outs=self.thetas)
        self.k += 1
        return L0, np.array(news), outs
