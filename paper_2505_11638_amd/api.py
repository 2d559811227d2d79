"""Thin Python binding of libngd with the C ABI's names. PyTorch supplies device memory and streams;
every computation runs in the library's HIP kernels.

The functions take torch tensors on a ROCm device, check dtypes / shapes / contiguity, and pass
raw pointers and the current stream to the corresponding `ngd_*` entry point.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

import numpy as np
import torch

from . import _lib as L

_TORCH = {L.NGD_F64: torch.float64, L.NGD_F32: torch.float32}
_DTYPE = {"f64": L.NGD_F64, "f32": L.NGD_F32, "bf16": L.NGD_BF16}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


_RAW_STREAM = getattr(torch._C, "_cuda_getCurrentRawStream", None)


def _stream():
    """The current stream of the current device, as the void* the ABI takes."""
    if _RAW_STREAM is not None:
        return C.c_void_p(_RAW_STREAM(torch.cuda.current_device()))
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t: torch.Tensor, dtype, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")


@dataclasses.dataclass
class NystromResult:
    U: torch.Tensor          # (ell, ldU), rows = eigenvectors
    lam_hat: torch.Tensor    # (ell,) float64 descending
    info: dict


@dataclasses.dataclass
class PcgResult:
    d: torch.Tensor          # (P,) float64
    iters: int
    rel_res: float
    converged: bool
    breakdown: bool
    status: int
    mu: Optional[float] = None  # the damping of the solve (set when the device chose it)


class Recompute:
    """Operator marker for the recompute mode: every product with J_w or J_w^T is formed from theta by
    the forward-tangent and adjoint kernels; J_w is never stored."""

    def __init__(self, theta: torch.Tensor):
        self.theta = theta


class Problem:
    """A PINN least-squares problem bound to a libngd handle.

    `data` needs attributes widths, pde, X (N x d), w, f, g, kind (as in `workloads.Problem`); they are
    copied to the device in the working precision `dtype` ("f64" or "f32")."""

    def __init__(self, data, dtype: Optional[str] = None, max_ell: Optional[int] = None, device="cuda",
                 _batch=None):
        self.lib = L.load()
        self.dtype_name = dtype or data.dtype
        self.dtype = _DTYPE[self.dtype_name]
        self.tdtype = _TORCH[self.dtype]
        self.device = torch.device(device)
        self.widths = tuple(int(v) for v in data.widths)
        self.pde = int(data.pde)
        to = lambda a, t: torch.as_tensor(np.ascontiguousarray(a), dtype=t, device=self.device)
        self.X = to(data.X, self.tdtype)
        self.w = to(data.w, self.tdtype)
        self.f = to(data.f, self.tdtype)
        self.g = to(data.g, self.tdtype)
        self.kind = to(data.kind, torch.int8)
        self.N = int(self.X.shape[0])
        self._widths_c = (C.c_int32 * len(self.widths))(*self.widths)
        self.desc = L.ProblemDesc(len(self.widths) - 1, self._widths_c, self.pde, self.dtype, self.N,
                                  self.X.data_ptr(), self.w.data_ptr(), self.f.data_ptr(), self.g.data_ptr(),
                                  self.kind.data_ptr(), int(max_ell or getattr(data, "ell", 1)),
                                  float(getattr(data, "nu", 0.0)))
        self._owned = _batch is None
        if _batch is not None:  # a batch member: the batch creates and owns the handle
            return
        h = C.c_void_p()
        L.check(self.lib.ngd_problem_create(C.byref(self.desc), C.byref(h)), "ngd_problem_create")
        self._bind(h)

    def _bind(self, h):
        self.h = h
        self.P = int(self.lib.ngd_num_params(h))
        self.ld = int(self.lib.ngd_recommended_ld(h))

    def close(self):
        if getattr(self, "h", None):
            if self._owned:
                self.lib.ngd_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        import sys
        if sys.is_finalizing():  # the HIP runtime may already be torn down: leave it to process exit
            return
        try:
            self.close()
        except Exception:
            pass

    # -- buffers ----------------------------------------------------------------------------------
    def theta(self, values) -> torch.Tensor:
        return torch.as_tensor(np.asarray(values), dtype=self.tdtype, device=self.device).contiguous()

    def new_jacobian(self) -> torch.Tensor:
        return torch.empty((self.N, self.ld), dtype=self.tdtype, device=self.device)

    def _op(self, J, theta: Optional[torch.Tensor] = None) -> L.Operator:
        if isinstance(J, Recompute):
            _need(J.theta, self.tdtype, "theta")
            return L.Operator(J.theta.data_ptr(), None, 0)
        _need(J, self.tdtype, "J")
        if J.dim() != 2 or J.shape[0] != self.N or J.stride(1) != 1:
            raise ValueError("J must be an N x ld row-major tensor")
        return L.Operator(None if theta is None else theta.data_ptr(), J.data_ptr(), J.stride(0))

    # -- entry points -------------------------------------------------------------------------------
    def residual_jacobian(self, theta: torch.Tensor, J: Optional[torch.Tensor] = None, want_grad=True,
                          want_loss=True, out=None):
        """ngd_residual_jacobian: returns (r_w, J or None, grad or None, loss tensor or None). `out`, if
        given, is an (r_w, grad, loss) triple of buffers from a previous call to write into."""
        _need(theta, self.tdtype, "theta")
        if out is not None:
            r, grad, loss = out
            grad = grad if want_grad else None
            loss = loss if want_loss else None
        else:
            r = torch.empty(self.N, dtype=self.tdtype, device=self.device)
            grad = torch.empty(self.P, dtype=torch.float64, device=self.device) if want_grad else None
            loss = torch.empty(1, dtype=torch.float64, device=self.device) if want_loss else None
        ldJ = J.stride(0) if J is not None else 0
        if J is not None:
            _need(J, self.tdtype, "J")
        L.check(self.lib.ngd_residual_jacobian(self.h, _ptr(theta), _ptr(r), _ptr(J), ldJ, _ptr(grad), _ptr(loss),
                                               _stream()), "ngd_residual_jacobian")
        return r, J, grad, loss

    def gramian_matvec(self, J: torch.Tensor, V: torch.Tensor, lam: float) -> torch.Tensor:
        """ngd_gramian_matvec: V (k, ld) or (P,) in the working dtype; returns Y of the same shape."""
        _need(V, self.tdtype, "V")
        vec = V.dim() == 1
        V2 = V.reshape(1, -1) if vec else V
        Y = torch.empty_like(V2)
        L.check(self.lib.ngd_gramian_matvec(self.h, C.byref(self._op(J)), _ptr(V2), V2.stride(0), V2.shape[0],
                                            float(lam), _ptr(Y), Y.stride(0), _stream()), "ngd_gramian_matvec")
        return Y.reshape(-1) if vec else Y

    def jvp(self, theta: torch.Tensor, V: torch.Tensor) -> torch.Tensor:
        """ngd_jvp: J_w(theta) V for V (P,) or (k, ld); returns (N,) or (k, N) in the working dtype."""
        _need(theta, self.tdtype, "theta")
        _need(V, self.tdtype, "V")
        vec = V.dim() == 1
        V2 = V.reshape(1, -1) if vec else V
        Y = torch.empty((V2.shape[0], self.N), dtype=self.tdtype, device=self.device)
        L.check(self.lib.ngd_jvp(self.h, _ptr(theta), _ptr(V2), V2.stride(0), V2.shape[0], _ptr(Y), Y.stride(0),
                                 _stream()), "ngd_jvp")
        return Y.reshape(-1) if vec else Y

    def vjp(self, theta: torch.Tensor, wv: torch.Tensor) -> torch.Tensor:
        """ngd_vjp: J_w(theta)^T wv for wv (N,) in the working dtype; returns P doubles."""
        _need(theta, self.tdtype, "theta")
        _need(wv, self.tdtype, "wv")
        out = torch.empty(self.P, dtype=torch.float64, device=self.device)
        L.check(self.lib.ngd_vjp(self.h, _ptr(theta), _ptr(wv), _ptr(out), _stream()), "ngd_vjp")
        return out

    def gaussian_omega(self, seed: int, counter: int, ell: int) -> torch.Tensor:
        out = torch.zeros((ell, self.ld), dtype=self.tdtype, device=self.device)
        L.check(self.lib.ngd_gaussian_omega(self.h, seed, counter, ell, _ptr(out), self.ld, _stream()),
                "ngd_gaussian_omega")
        return out

    def nystrom_sketch(self, J: torch.Tensor, ell: int, seed: int = 0, counter: int = 0,
                       omega: Optional[torch.Tensor] = None, sketch_dtype: Optional[str] = None,
                       want_info=True, out: Optional[NystromResult] = None,
                       cols: Optional[torch.Tensor] = None) -> NystromResult:
        """ngd_nystrom_sketch (Gaussian test matrix), or ngd_nystrom_sketch_columns when `cols` (device
        int64 indices) gives a sampling test matrix; `out`, if given, is a previous result of the same
        ell to write into."""
        sd = _DTYPE[sketch_dtype or ("f64" if self.dtype == L.NGD_F64 else "f32")]
        if out is not None and out.lam_hat.numel() == ell:
            U, lam = out.U, out.lam_hat
        else:
            # zeros: the library writes columns 0..P-1 only, so the padding stays defined
            U = torch.zeros((ell, self.ld), dtype=self.tdtype, device=self.device)
            lam = torch.empty(ell, dtype=torch.float64, device=self.device)
        info = L.NystromInfo()
        ldO = 0
        if omega is not None:
            _need(omega, self.tdtype, "omega")
            ldO = omega.stride(0)
        if cols is not None:
            if not (cols.is_cuda and cols.dtype == torch.int64 and cols.numel() >= ell and cols.is_contiguous()):
                raise ValueError("cols must be a contiguous device int64 tensor of at least ell indices")
            L.check(self.lib.ngd_nystrom_sketch_columns(self.h, C.byref(self._op(J)), ell, _ptr(cols), sd, _ptr(U),
                                                        U.stride(0), _ptr(lam), C.byref(info) if want_info else None,
                                                        _stream()), "ngd_nystrom_sketch_columns")
        else:
            L.check(self.lib.ngd_nystrom_sketch(self.h, C.byref(self._op(J)), ell, seed, counter, _ptr(omega), ldO,
                                                sd, _ptr(U), U.stride(0), _ptr(lam),
                                                C.byref(info) if want_info else None, _stream()), "ngd_nystrom_sketch")
        d = {k: getattr(info, k) for k, _ in L.NystromInfo._fields_} if want_info else {}
        return NystromResult(U, lam, d)

    def pcg_solve(self, J: torch.Tensor, g: torch.Tensor, lam: float, precond: Optional[NystromResult] = None,
                  rtol: float = 1e-6, maxit: int = 1000, raise_on_fail=False, damping=None,
                  out: Optional[torch.Tensor] = None) -> PcgResult:
        """ngd_pcg_solve with damping lam; or, with damping = (c_lam, c_loss, loss tensor) and a
        preconditioner, ngd_pcg_solve_damped: lam = max(c_lam lam_hat[0], c_loss loss^2) on the device.
        `out`, if given, is a P-double device buffer for d."""
        _need(g, torch.float64, "g")
        d = torch.empty(self.P, dtype=torch.float64, device=self.device) if out is None else out
        if d.numel() != self.P or d.dtype != torch.float64 or not d.is_contiguous():
            raise ValueError("out must be a contiguous P-double tensor")
        info = L.PcgInfo()
        pc = None
        if precond is not None:
            pc = L.Precond(precond.U.data_ptr(), precond.U.stride(0), precond.lam_hat.data_ptr(),
                           precond.lam_hat.numel())
        mu = None
        if damping is not None:
            if pc is None:
                raise ValueError("the device damping rule needs a preconditioner")
            c_lam, c_loss, loss = damping
            _need(loss, torch.float64, "loss")
            lam_used = C.c_double()
            st = self.lib.ngd_pcg_solve_damped(self.h, C.byref(self._op(J)), _ptr(g), float(c_lam), float(c_loss),
                                               _ptr(loss), C.byref(pc), float(rtol), int(maxit), _ptr(d),
                                               C.byref(info), C.byref(lam_used), _stream())
            mu = float(lam_used.value)
            where = "ngd_pcg_solve_damped"
        else:
            st = self.lib.ngd_pcg_solve(self.h, C.byref(self._op(J)), _ptr(g), float(lam),
                                        C.byref(pc) if pc is not None else None, float(rtol), int(maxit), _ptr(d),
                                        C.byref(info), _stream())
            where = "ngd_pcg_solve"
        allow = () if raise_on_fail else (L.NGD_ERR_NOT_CONVERGED, L.NGD_ERR_BREAKDOWN)
        L.check(st, where, allow)
        return PcgResult(d, int(info.iters), float(info.rel_res), bool(info.converged), bool(info.breakdown), st,
                         mu)

    def direct_solve(self, J, g: torch.Tensor, lam: float, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """ngd_direct_solve (Alg. 2): d = (J_w^T J_w + lam I)^{-1} g through the explicit FP64 Gramian and
        its Cholesky factor; synchronises."""
        _need(g, torch.float64, "g")
        d = torch.empty(self.P, dtype=torch.float64, device=self.device) if out is None else out
        L.check(self.lib.ngd_direct_solve(self.h, C.byref(self._op(J)), _ptr(g), float(lam), _ptr(d), _stream()),
                "ngd_direct_solve")
        return d

    def power_lambda_max(self, J: torch.Tensor, v0: torch.Tensor, iters: int = 4,
                         out: Optional[torch.Tensor] = None) -> float:
        """ngd_power_lambda_max: the estimate on the host; also into `out` (a device double) when given."""
        _need(v0, torch.float64, "v0")
        res = C.c_double()
        L.check(self.lib.ngd_power_lambda_max(self.h, C.byref(self._op(J)), _ptr(v0), iters, C.byref(res),
                                              _ptr(out), _stream()), "ngd_power_lambda_max")
        return res.value

    def damping(self, lam1: torch.Tensor, loss: Optional[torch.Tensor], c_lam: float, c_loss: float,
                out: Optional[torch.Tensor] = None, host: bool = True):
        """ngd_damping (the rule of Section 4.3) on device doubles: returns (mu device tensor, mu on the host
        or None when host=False)."""
        _need(lam1, torch.float64, "lam1")
        mu = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        mh = C.c_double()
        L.check(self.lib.ngd_damping(self.h, _ptr(lam1), _ptr(loss), float(c_lam), float(c_loss), _ptr(mu),
                                     C.byref(mh) if host else None, _stream()), "ngd_damping")
        return mu, (mh.value if host else None)

    def lm_damping(self, J, d: torch.Tensor, grad: torch.Tensor, alpha: float, loss0: float, loss1: float, mu: float,
                   mu_floor: float = 0.0):
        """ngd_lm_damping: the Levenberg-Marquardt update of mu from the step just taken; returns
        (mu_next, rho)."""
        _need(d, torch.float64, "d")
        _need(grad, torch.float64, "grad")
        mn, rho = C.c_double(), C.c_double()
        L.check(self.lib.ngd_lm_damping(self.h, C.byref(self._op(J)), _ptr(d), _ptr(grad), float(alpha), float(loss0),
                                        float(loss1), float(mu), float(mu_floor), C.byref(mn), C.byref(rho),
                                        _stream()), "ngd_lm_damping")
        return mn.value, rho.value

    def next_rank(self, lam_hat: torch.Tensor, ell: int, mu: float, dell: int, offset: int, ell_max: int) -> int:
        """ngd_next_rank: Alg. 4's next sketch size from lam_hat[:ell] and the step's damping mu."""
        _need(lam_hat, torch.float64, "lam_hat")
        out = C.c_int64()
        L.check(self.lib.ngd_next_rank(self.h, _ptr(lam_hat), int(ell), float(mu), int(dell), int(offset),
                                       int(ell_max), C.byref(out), _stream()), "ngd_next_rank")
        return int(out.value)

    def timing(self, enable: bool, only=None):
        """Turn the kernel timers on (all, or only the named ones) or off; resets the counters."""
        if enable and only is not None:
            mask = 0
            for name in only:
                mask |= 1 << L.TIMERS[name]
            L.check(self.lib.ngd_timing_enable_mask(self.h, mask), "ngd_timing_enable_mask")
        else:
            L.check(self.lib.ngd_timing_enable(self.h, 1 if enable else 0), "ngd_timing_enable")

    def timers(self) -> dict:
        """{name: (launches, total_ms)} of the library's kernel timers."""
        out = {}
        for name, tid in L.TIMERS.items():
            n, ms = C.c_int64(), C.c_double()
            L.check(self.lib.ngd_timing_read(self.h, tid, C.byref(n), C.byref(ms)), "ngd_timing_read")
            out[name] = (int(n.value), float(ms.value))
        return out

    def line_search(self, theta: torch.Tensor, d: torch.Tensor, grad: torch.Tensor, loss0: float, c1=1e-4,
                    max_halvings=30, theta_out: Optional[torch.Tensor] = None):
        theta_out = torch.empty_like(theta) if theta_out is None else theta_out
        a, ln = C.c_double(), C.c_double()
        L.check(self.lib.ngd_line_search(self.h, _ptr(theta), _ptr(d), _ptr(grad), float(loss0), float(c1),
                                         int(max_halvings), _ptr(theta_out), C.byref(a), C.byref(ln), _stream()),
                "ngd_line_search")
        return theta_out, a.value, ln.value

    def gramian_diagonal(self, J, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """diag(J_w^T J_w) (eq. gram_diagonal), P doubles on the device."""
        out = torch.empty(self.P, dtype=torch.float64, device=self.device) if out is None else out
        L.check(self.lib.ngd_gramian_diagonal(self.h, C.byref(self._op(J)), _ptr(out), _stream()),
                "ngd_gramian_diagonal")
        return out

    def sample_pivots(self, weights: torch.Tensor, n: int, seed: int = 0, counter: int = 0, substream: int = 0,
                      unique: bool = False, out: Optional[torch.Tensor] = None):
        """n indices drawn with probability proportional to max(weights, 0) (ngd_sample_pivots):
        (idx device int64 tensor, count device int32 tensor)."""
        _need(weights, torch.float64, "weights")
        idx = torch.empty(max(int(n), 1), dtype=torch.int64, device=self.device) if out is None else out
        cnt = torch.empty(1, dtype=torch.int32, device=self.device)
        L.check(self.lib.ngd_sample_pivots(self.h, _ptr(weights), int(n), int(seed), int(counter), int(substream),
                                           1 if unique else 0, _ptr(idx), _ptr(cnt), _stream()), "ngd_sample_pivots")
        return idx, cnt

    def rpcholesky(self, J, diag: torch.Tensor, ell_max: int, block: int = 20, seed: int = 0, counter: int = 0,
                   eps: float = 0.0, Ft: Optional[torch.Tensor] = None):
        """Block RPCholesky (ngd_rpcholesky): (Ft (ell_max x ld) float64 device tensor, rank, trace)."""
        _need(diag, torch.float64, "diag")
        Ft = torch.empty((ell_max, self.ld), dtype=torch.float64, device=self.device) if Ft is None else Ft
        r, tr = C.c_int64(), C.c_double()
        L.check(self.lib.ngd_rpcholesky(self.h, C.byref(self._op(J)), _ptr(diag), int(ell_max), int(block), int(seed),
                                        int(counter), float(eps), _ptr(Ft), Ft.stride(0), C.byref(r), C.byref(tr),
                                        _stream()), "ngd_rpcholesky")
        return Ft, int(r.value), float(tr.value)

    def rpchol_precond(self, Ft: torch.Tensor, rank: int, mu: Optional[float] = None) -> NystromResult:
        """The RPCholesky preconditioner as (U, lam_hat) with a trailing zero pair; use it as `precond` of
        pcg_solve. With mu: the Woodbury-Cholesky form for solves with lambda = mu
        (ngd_rpchol_precond_woodbury); without: the form from the eigenpairs of F^T F (ngd_rpchol_precond),
        valid for any lambda."""
        U = torch.zeros((rank + 1, self.ld), dtype=self.tdtype, device=self.device)
        lam = torch.empty(rank + 1, dtype=torch.float64, device=self.device)
        if mu is None:
            L.check(self.lib.ngd_rpchol_precond(self.h, _ptr(Ft), Ft.stride(0), int(rank), _ptr(U), U.stride(0),
                                                _ptr(lam), _stream()), "ngd_rpchol_precond")
            return NystromResult(U, lam, {"rank": rank})
        L.check(self.lib.ngd_rpchol_precond_woodbury(self.h, _ptr(Ft), Ft.stride(0), int(rank), float(mu), _ptr(U),
                                                     U.stride(0), _ptr(lam), _stream()), "ngd_rpchol_precond_woodbury")
        return NystromResult(U, lam, {"rank": rank, "woodbury_mu": float(mu)})

    def solution_error(self, theta: torch.Tensor, X, u_ref, grad_u_ref, sums: Optional[torch.Tensor] = None):
        """Relative L2 and H1 errors of u_theta against (u_ref, grad u_ref) on the points X (n x d), the
        accuracy measure of Section 5 (Monte Carlo over the evaluation set). Returns
        (rel_l2, rel_h1, sums) with the four FP64 device sums of the entry point; synchronises."""
        to = lambda a: torch.as_tensor(np.asarray(a), dtype=self.tdtype, device=self.device).contiguous()
        X, u_ref, grad_u_ref = to(X), to(u_ref), to(grad_u_ref)
        n = int(X.shape[0]) if X.ndim == 2 else 0
        if self.pde == L.NGD_PDE_NAVIER_STOKES:  # the velocity: u_ref n x 2, grad_u_ref n x 2 x 2 ([k][j])
            if X.ndim != 2 or X.shape[1] != 2 or u_ref.shape != (n, 2) or grad_u_ref.shape != (n, 2, 2):
                raise ValueError("solution_error: X must be n x 2, u_ref n x 2, grad_u_ref n x 2 x 2")
        elif X.ndim != 2 or X.shape[1] != self.widths[0] or u_ref.shape != (n,) or grad_u_ref.shape != X.shape:
            raise ValueError("solution_error: X must be n x d, u_ref n, grad_u_ref n x d")
        _need(theta, self.tdtype, "theta")
        sums = torch.empty(4, dtype=torch.float64, device=self.device) if sums is None else sums
        L.check(self.lib.ngd_solution_error(self.h, _ptr(theta), _ptr(X), n, _ptr(u_ref), _ptr(grad_u_ref),
                                            _ptr(sums), _stream()), "ngd_solution_error")
        s = sums.cpu().numpy()
        rel_l2 = float(np.sqrt(s[0] / s[2])) if s[2] > 0 else float("nan")
        rel_h1 = float(np.sqrt((s[0] + s[1]) / (s[2] + s[3]))) if s[2] + s[3] > 0 else float("nan")
        return rel_l2, rel_h1, sums


class Batch:
    """Several independent problems (one dtype) bound to one libngd batch. `members[i]` is a `Problem`
    view of member i's handle (for its sketch, line search, ...); `residual_jacobian` and `pcg_solve`
    run all members together through the batched entry points."""

    def __init__(self, datas, dtype: Optional[str] = None, device="cuda"):
        self.lib = L.load()
        self.members = [Problem(d, dtype=dtype, device=device, _batch=self) for d in datas]
        descs = (L.ProblemDesc * len(self.members))(*[m.desc for m in self.members])
        b = C.c_void_p()
        L.check(self.lib.ngd_batch_create(descs, len(self.members), C.byref(b)), "ngd_batch_create")
        self.b = b
        for i, m in enumerate(self.members):
            m._bind(C.c_void_p(self.lib.ngd_batch_problem(b, i)))

    def __len__(self):
        return len(self.members)

    def close(self):
        if getattr(self, "b", None):
            for m in self.members:
                m.h = None
            self.lib.ngd_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        import sys
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _ptrs(ts):
        return (C.c_void_p * len(ts))(*[None if t is None else t.data_ptr() for t in ts])

    def residual_jacobian(self, thetas, Js, want_grad=True, want_loss=True):
        """ngd_batch_residual_jacobian: returns lists (r_w, grad or None, loss or None) per member."""
        n = len(self.members)
        rs = [torch.empty(m.N, dtype=m.tdtype, device=m.device) for m in self.members]
        grads = [torch.empty(m.P, dtype=torch.float64, device=m.device) if want_grad else None for m in self.members]
        losses = [torch.empty(1, dtype=torch.float64, device=m.device) if want_loss else None for m in self.members]
        for m, t, J in zip(self.members, thetas, Js):
            _need(t, m.tdtype, "theta")
            _need(J, m.tdtype, "J")
        lds = (C.c_int64 * n)(*[J.stride(0) for J in Js])
        L.check(self.lib.ngd_batch_residual_jacobian(self.b, self._ptrs(thetas), self._ptrs(rs), self._ptrs(Js), lds,
                                                     self._ptrs(grads) if want_grad else None,
                                                     self._ptrs(losses) if want_loss else None, _stream()),
                "ngd_batch_residual_jacobian")
        return rs, grads, losses

    def nystrom_sketch(self, Js, ells, seed=0, counter=0, sketch_dtype="f32", outs=None):
        """ngd_batch_nystrom_sketch: every member's Gaussian sketch side by side, no host round trip.
        Returns a NystromResult per member (info empty); `outs`, if given, are previous results of the
        same ells to write into."""
        n = len(self.members)
        res = []
        for i, (m, ell) in enumerate(zip(self.members, ells)):
            o = outs[i] if outs is not None else None
            if o is not None and o.lam_hat.numel() == ell:
                res.append(o)
            else:
                res.append(NystromResult(torch.zeros((ell, m.ld), dtype=m.tdtype, device=m.device),
                                         torch.empty(ell, dtype=torch.float64, device=m.device), {}))
        ops = (L.Operator * n)(*[m._op(J) for m, J in zip(self.members, Js)])
        ell_a = (C.c_int64 * n)(*[int(e) for e in ells])
        ld_a = (C.c_int64 * n)(*[r.U.stride(0) for r in res])
        L.check(self.lib.ngd_batch_nystrom_sketch(self.b, ops, ell_a, int(seed), int(counter), _DTYPE[sketch_dtype],
                                                  self._ptrs([r.U for r in res]), ld_a,
                                                  self._ptrs([r.lam_hat for r in res]), _stream()),
                "ngd_batch_nystrom_sketch")
        return res

    def line_search(self, thetas, ds, grads, loss0, c1=1e-4, max_halvings=30, theta_outs=None):
        """ngd_batch_line_search: every member's Armijo step with the decisions on the device. loss0:
        host floats. Returns (theta_outs, alphas, new losses) as lists."""
        n = len(self.members)
        theta_outs = [torch.empty_like(t) for t in thetas] if theta_outs is None else theta_outs
        l0 = (C.c_double * n)(*[float(x) for x in loss0])
        a, ln = (C.c_double * n)(), (C.c_double * n)()
        L.check(self.lib.ngd_batch_line_search(self.b, self._ptrs(thetas), self._ptrs(ds), self._ptrs(grads), l0,
                                               float(c1), int(max_halvings), self._ptrs(theta_outs), a, ln,
                                               _stream()), "ngd_batch_line_search")
        return theta_outs, list(a), list(ln)

    def pcg_solve_damped(self, Js, gs, c_lam, c_loss, losses, precs, rtol=1e-6, maxit=1000):
        """ngd_batch_pcg_solve_damped: the damping rule on the device per member. Returns the PcgResults
        (with mu set)."""
        n = len(self.members)
        ops = (L.Operator * n)(*[m._op(J) for m, J in zip(self.members, Js)])
        ds = [torch.empty(m.P, dtype=torch.float64, device=m.device) for m in self.members]
        pcs = (L.Precond * n)(*[L.Precond(p.U.data_ptr(), p.U.stride(0), p.lam_hat.data_ptr(), p.lam_hat.numel())
                                for p in precs])
        infos = (L.PcgInfo * n)()
        used = (C.c_double * n)()
        for m, gv in zip(self.members, gs):
            _need(gv, torch.float64, "g")
        st = self.lib.ngd_batch_pcg_solve_damped(self.b, ops, self._ptrs(gs), float(c_lam), float(c_loss),
                                                 self._ptrs(losses) if losses is not None else None, pcs,
                                                 float(rtol), int(maxit), self._ptrs(ds), infos, used, _stream())
        L.check(st, "ngd_batch_pcg_solve_damped", (L.NGD_ERR_NOT_CONVERGED, L.NGD_ERR_BREAKDOWN))
        return [PcgResult(d, int(i.iters), float(i.rel_res), bool(i.converged), bool(i.breakdown), st, float(u))
                for d, i, u in zip(ds, infos, used)]

    def matvec_time(self, reps: int = 10) -> float:
        """ngd_batch_matvec_time: average ms of one batched matvec launch (after a batched solve)."""
        out = C.c_double()
        L.check(self.lib.ngd_batch_matvec_time(self.b, int(reps), C.byref(out), _stream()), "ngd_batch_matvec_time")
        return out.value

    def pcg_solve(self, Js, gs, lams, precs=None, rtol=1e-6, maxit=1000):
        """ngd_batch_pcg_solve: precs is None or a list of NystromResult / None per member."""
        n = len(self.members)
        ops = (L.Operator * n)(*[m._op(J) for m, J in zip(self.members, Js)])
        ds = [torch.empty(m.P, dtype=torch.float64, device=m.device) for m in self.members]
        lam = (C.c_double * n)(*[float(v) for v in lams])
        pcs = None
        if precs is not None:
            pcs = (L.Precond * n)(*[L.Precond(p.U.data_ptr(), p.U.stride(0), p.lam_hat.data_ptr(), p.lam_hat.numel())
                                    if p is not None else L.Precond(None, 0, None, 0) for p in precs])
        infos = (L.PcgInfo * n)()
        for m, gv in zip(self.members, gs):
            _need(gv, torch.float64, "g")
        st = self.lib.ngd_batch_pcg_solve(self.b, ops, self._ptrs(gs), lam, pcs, float(rtol), int(maxit),
                                          self._ptrs(ds), infos, _stream())
        L.check(st, "ngd_batch_pcg_solve", (L.NGD_ERR_NOT_CONVERGED, L.NGD_ERR_BREAKDOWN))
        return [PcgResult(d, int(i.iters), float(i.rel_res), bool(i.converged), bool(i.breakdown), st)
                for d, i in zip(ds, infos)]
