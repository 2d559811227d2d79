"""The no-allocation Gramian product (ngd_gramian_matvec_noalloc) against the handle's
ngd_gramian_matvec on the same J_w and v, through the C ABI: two calls in a row, the second on a
smaller problem (the static scratch keeps the first call's contents), FP64 and FP32, and the
largest problem of the benchmark set (5D Poisson, N = 18,432, P = 33,921). Both run the same
one-pass kernels with the same workgroup count, so the results agree to the last bit; the test asks
for the FP64 / FP32 parity tolerance (1e-10 / 1e-5 relative) and reports the exact match as well."""
import ctypes as C

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_11638_amd import _lib as L  # noqa: E402
from paper_2505_11638_amd.api import Problem, _stream  # noqa: E402


def _jacobian(prob, dtype):
    gp = Problem(prob, dtype=dtype, max_ell=1)
    theta = gp.theta(wl.glorot_theta(prob.widths, 3))
    J = gp.new_jacobian()
    gp.residual_jacobian(theta, J, want_grad=False, want_loss=False)
    return gp, J


def _noalloc(gp, J, v, lam):
    y = torch.full_like(v, float("nan"))
    st = gp.lib.ngd_gramian_matvec_noalloc(gp.dtype, C.c_void_p(J.data_ptr()), J.stride(0), gp.N, gp.P,
                                           C.c_void_p(v.data_ptr()), float(lam), C.c_void_p(y.data_ptr()), _stream())
    L.check(st, "ngd_gramian_matvec_noalloc")
    return y


def _case(prob, dtype, lam, seed):
    print(f"noalloc case: {dtype} N={prob.n_rows} P={prob.n_params} lam={lam}", flush=True)
    gp, J = _jacobian(prob, dtype)
    v = torch.as_tensor(np.random.default_rng(seed).standard_normal(gp.P), dtype=gp.tdtype, device="cuda")
    y_ref = gp.gramian_matvec(J, v, lam)
    y = _noalloc(gp, J, v, lam)
    torch.cuda.synchronize()
    a, b = y.double().cpu().numpy(), y_ref.double().cpu().numpy()
    tol = 1e-10 if dtype == "f64" else 1e-5
    assert np.all(np.isfinite(a))
    assert np.linalg.norm(a - b) <= tol * np.linalg.norm(b)
    exact = bool(np.array_equal(a, b))
    gp.close()
    return exact


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_handle_twice_second_smaller(dtype):
    big = wl.poisson_random(d=2, widths=(2, 64, 64, 64, 1), n_interior=2048, n_boundary=256, seed=1, dtype=dtype)
    small = wl.poisson_random(d=3, widths=(3, 24, 24, 1), n_interior=150, n_boundary=40, seed=2, dtype=dtype)
    e1 = _case(big, dtype, 1e-3, 5)
    e2 = _case(small, dtype, 0.0, 6)
    print(f"bitwise equal to ngd_gramian_matvec: {e1}, {e2}")


def test_noalloc_full_size_and_refusals():
    prob = wl.config("c3")
    _case(prob, "f32", 1e-4, 7)
    # argument errors are refused on the host, before anything is enqueued
    gp, J = _jacobian(wl.small_problem(widths=(2, 8, 8, 1), n_interior=20, n_boundary=8, seed=0), "f64")
    v = torch.zeros(gp.P, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(v)
    f = gp.lib.ngd_gramian_matvec_noalloc
    args = lambda dt, ld, lam: (dt, C.c_void_p(J.data_ptr()), ld, gp.N, gp.P, C.c_void_p(v.data_ptr()), lam,
                                C.c_void_p(y.data_ptr()), _stream())
    assert f(*args(L.NGD_BF16, J.stride(0), 0.0)) == L.NGD_ERR_INVALID
    assert f(*args(L.NGD_F64, J.stride(0), -1.0)) == L.NGD_ERR_INVALID
    assert f(*args(L.NGD_F64, 1 << 20, 0.0)) == L.NGD_ERR_INVALID
    assert b"too large" in gp.lib.ngd_last_error()
    assert f(L.NGD_F64, None, J.stride(0), gp.N, gp.P, None, 0.0, None, _stream()) == L.NGD_ERR_INVALID
    torch.cuda.synchronize()
    gp.close()
