"""Batched problems (uneven P, N, ell in one launch per stage): the batched residual / Jacobian launch
against each member's own single-problem call, and the batched, graph-replayed PCG against each
member's single-problem solve and the FP64 oracle's direct solve (MI355X)."""
import numpy as np
import pytest

import workloads as wl
from gpu_helpers import make

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from oracle import linalg, mlp  # noqa: E402
from paper_2505_11638_amd.api import Batch  # noqa: E402
from paper_2505_11638_amd.driver import BatchNGD  # noqa: E402


def _members(n=5, seed=3):
    """Small uneven members (ragged N, mixed depth / width / dimension / ell)."""
    probs = wl.batch_instances(n=n, seed=seed, widths=(8, 16, 24), depths=(1, 2, 3), n_min=40, n_max=120,
                               ells=(6, 10, 16), dims=(2, 3))
    out = []
    for i, p in enumerate(probs):
        p64, th = make(p, seed=i)
        out.append((p64, th))
    return out


def test_batch_residual_jacobian_matches_members():
    mem = _members()
    b = Batch([p for p, _ in mem], dtype="f32")
    thetas = [m.theta(th) for m, (_, th) in zip(b.members, mem)]
    Js = [m.new_jacobian() for m in b.members]
    rs, grads, losses = b.residual_jacobian(thetas, Js)
    torch.cuda.synchronize()
    for m, th, J, r, g, l in zip(b.members, thetas, Js, rs, grads, losses):
        J1 = m.new_jacobian()
        r1, J1, g1, l1 = m.residual_jacobian(th, J1)
        torch.cuda.synchronize()
        # the same kernel body and tile size per member: identical arithmetic
        assert torch.equal(r, r1)
        assert torch.equal(J[:, :m.P], J1[:, :m.P])
        assert torch.equal(g, g1)
        assert l.item() == l1.item()
    b.close()


def test_batch_pcg_matches_members_and_direct_solve():
    mem = _members(n=6, seed=5)
    b = Batch([p for p, _ in mem], dtype="f32")
    thetas = [m.theta(th) for m, (_, th) in zip(b.members, mem)]
    Js = [m.new_jacobian() for m in b.members]
    _, grads, _ = b.residual_jacobian(thetas, Js)
    lams = [1e-3 * (1 + i) for i in range(len(mem))]
    # members 0, 2, 4 preconditioned (Nystrom, own ell), the others plain CG
    pcs = [m.nystrom_sketch(J, p.ell, seed=1, counter=0, sketch_dtype="f32") if i % 2 == 0 else None
           for i, (m, J, (p, _)) in enumerate(zip(b.members, Js, mem))]
    rtol = 1e-5
    for rep in range(2):  # the second solve replays the captured iteration graph with new right-hand sides
        gs = [g * (1.0 + 0.5 * rep) for g in grads]
        outs = b.pcg_solve(Js, gs, lams, pcs, rtol=rtol, maxit=2000)
        for i, (m, J, o) in enumerate(zip(b.members, Js, outs)):
            assert o.converged, (rep, i, o)
            single = m.pcg_solve(J, gs[i], lams[i], precond=pcs[i], rtol=rtol, maxit=2000)
            assert abs(o.iters - single.iters) <= max(2, 0.25 * single.iters), (rep, i, o.iters, single.iters)
            # against the direct solve on the member's FP32 Jacobian promoted to FP64
            Jn = J[:, :m.P].cpu().numpy().astype(np.float64)
            G = linalg.gramian(Jn)
            gn = gs[i].cpu().numpy()
            dn = o.d.cpu().numpy()
            res = linalg.true_relative_residual(G, lams[i], gn, dn)
            assert res <= 20 * rtol, (rep, i, res)
            d_star = linalg.solve_cholesky(G, gn, lams[i])
            assert np.linalg.norm(dn - d_star) <= 1.01 * res * np.linalg.norm(gn) / lams[i] + 1e-9
    b.close()


def test_batch_ngd_steps_decrease_loss():
    mem = _members(n=4, seed=7)
    ngd = BatchNGD([p for p, _ in mem], [th for _, th in mem], solver="nystrom", seed=2)
    for _ in range(3):
        L0, L1, outs = ngd.step()
        assert np.all(L1 <= L0 + 1e-12)
        assert all(o.converged for o in outs)
    ngd.batch.close()
