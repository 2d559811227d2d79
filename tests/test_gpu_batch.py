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


@pytest.mark.timeout(900)
def test_c5_workload_members_against_oracle():
    """The batched workload itself (32 problems, hidden widths 32-96, depths 2-4, N 1,152-9,216, ell up to
    400, FP32) through the batched entry points: residual/Jacobian launch, the side-by-side sketches and
    the graph-replayed solve with the damping rule on the device. Members that cover both dimensions,
    every depth and the largest and smallest P and ell are checked against the oracle: sampled Jacobian
    rows and all residuals; the gradient, Alg. 6's eigenvalues (same Omega) and the solve's true residual
    in FP64 on the member's own FP32 Jacobian; the damping against the rule."""
    from oracle import nystrom
    from gpu_helpers import check_fp32_solve, jt_mul, rowwise_rel
    probs = wl.batch_instances(seed=0)
    b = Batch(probs, dtype="f32")
    ths = [wl.glorot_theta(p.widths, i) for i, p in enumerate(probs)]
    ths = [t.astype(np.float32).astype(np.float64) for t in ths]
    thetas = [m.theta(t) for m, t in zip(b.members, ths)]
    Js = [m.new_jacobian() for m in b.members]
    rs, grads, losses = b.residual_jacobian(thetas, Js)
    ells = [p.ell for p in probs]
    pcs = b.nystrom_sketch(Js, ells, seed=3, counter=1)
    eps32 = 2.0 ** -23
    outs = b.pcg_solve_damped(Js, grads, 10 * eps32, 1e-4, losses, pcs, rtol=1e-6, maxit=1000)
    torch.cuda.synchronize()
    assert all(o.converged for o in outs)
    P = [m.P for m in b.members]
    pick = {int(np.argmax(P)), int(np.argmin(P)), int(np.argmax(ells)), int(np.argmin(ells))}
    for key in (lambda p: p.d, lambda p: len(p.widths)):
        seen = {}
        for i, p in enumerate(probs):
            seen.setdefault(key(p), i)
        pick |= set(seen.values())
    for i in sorted(pick):
        p, m = probs[i], b.members[i]
        p64 = p.cast("f32")
        print(f"c5 member {i}: d={p.d} widths={p.widths} N={m.N} P={m.P} ell={ells[i]}", flush=True)
        rng = np.random.default_rng(i)
        rows = np.unique(np.concatenate([rng.choice(m.N, 10, replace=False), [0, m.N - 1]]))
        J32 = Js[i].cpu().numpy()[:, :m.P]
        assert rowwise_rel(J32[rows], mlp.jacobian(ths[i], p64, rows)) <= 1e-5
        r_o = mlp.weighted_residual(ths[i], p64)
        assert np.linalg.norm(rs[i].cpu().numpy() - r_o) <= 1e-5 * np.linalg.norm(r_o)
        r32 = rs[i].cpu().numpy().astype(np.float64)
        g_ref = np.zeros(m.P)
        for s in range(0, m.N, 2048):
            g_ref += J32[s:s + 2048].astype(np.float64).T @ r32[s:s + 2048]
        assert np.linalg.norm(grads[i].cpu().numpy() - g_ref) <= 1e-5 * np.linalg.norm(g_ref)
        # Alg. 6 on the member's own FP32 Jacobian with the test matrix it drew, (3, 1 + i 2^32)
        om = m.gaussian_omega(3, 1 + (i << 32), ells[i]).cpu().numpy()[:, :m.P].T.astype(np.float64)
        _, lo, _ = nystrom.nystrom_alg6(lambda V: jt_mul(J32, V), om)
        lam = pcs[i].lam_hat.cpu().numpy()
        top = lo >= 1e-6 * lo[0]
        err = np.max(np.abs(lam[top] - lo[top])) / lo[0]
        L0 = float(losses[i].item())
        mu = max(10 * eps32 * lam[0], 1e-4 * (L0 * L0))
        assert outs[i].mu == mu
        res = check_fp32_solve(J32, grads[i].cpu().numpy(), outs[i].d.cpu().numpy(), mu, 1e-6)
        print(f"  Alg. 6 max |lam - lam_o| / lam_1 (lam >= 1e-6 lam_1) {err:.1e}; mu {mu:.3e}; "
              f"PCG {outs[i].iters} its, true residual {res:.1e}", flush=True)
        assert err <= 1e-5
    b.close()


def test_batch_sketch_equals_member_sketches():
    """The batched sketch (each member's core tridiagonalised in batched launches, one per register
    shape, with the rest of each core side by side) against every member's own single-problem sketch
    with the same test matrix: the same arithmetic, so U and the eigenvalues agree bitwise. The c5
    members span ell = 50-400, i.e. four register shapes, and several matrices share each launch."""
    probs = wl.batch_instances(seed=0)
    b = Batch(probs, dtype="f32")
    ths = [wl.glorot_theta(p.widths, i) for i, p in enumerate(probs)]
    thetas = [m.theta(t) for m, t in zip(b.members, ths)]
    Js = [m.new_jacobian() for m in b.members]
    b.residual_jacobian(thetas, Js)
    ells = [p.ell for p in probs]
    pcs = b.nystrom_sketch(Js, ells, seed=5, counter=2)
    torch.cuda.synchronize()
    print(f"batched sketch of {len(probs)} members, ell in {sorted(set(ells))}", flush=True)
    for i, (m, J) in enumerate(zip(b.members, Js)):
        one = m.nystrom_sketch(J, ells[i], seed=5, counter=2 + (i << 32), sketch_dtype="f32")
        assert torch.equal(one.lam_hat, pcs[i].lam_hat), f"member {i}: eigenvalues differ"
        assert torch.equal(one.U[:, :m.P], pcs[i].U[:, :m.P]), f"member {i}: U differs"
    b.close()


def test_batch_line_search_equals_member_line_searches():
    """The batched line search (decisions on the device, one host wait per round for all members) against
    each member's own ngd_line_search from the same theta, d, gradient and loss: the same step, the same
    new loss and the same theta_out, bitwise. Members get a descent direction (the gradient, scaled so
    that some accept alpha = 1 and some need halvings) or an ascent direction (never accepted: alpha = 0
    after max_halvings halvings, theta unchanged)."""
    mem = _members(n=6, seed=11)
    b = Batch([p for p, _ in mem], dtype="f32")
    thetas = [m.theta(th) for m, (_, th) in zip(b.members, mem)]
    Js = [m.new_jacobian() for m in b.members]
    _, grads, losses = b.residual_jacobian(thetas, Js)
    L0 = [float(l.item()) for l in losses]
    scales = [1.0, 40.0, -1.0, 0.3, 300.0, -5.0]
    ds = [g * s for g, s in zip(grads, scales)]
    for max_h in (4, 30):
        ref = []
        for m, th, d, g, l0 in zip(b.members, thetas, ds, grads, L0):
            out, a, ln = m.line_search(th, d, g, l0, max_halvings=max_h)
            ref.append((out, a, ln))
        outs, alphas, news = b.line_search(thetas, ds, grads, L0, max_halvings=max_h)
        torch.cuda.synchronize()
        for i, (out, a, ln) in enumerate(ref):
            print(f"max_halvings {max_h} member {i}: scale {scales[i]}, alpha {a} / {alphas[i]}, "
                  f"loss {l0_fmt(L0[i])} -> {ln:.6e} / {news[i]:.6e}", flush=True)
            assert alphas[i] == a and news[i] == ln
            assert torch.equal(outs[i], out)
            if scales[i] < 0:
                assert a == 0.0 and torch.equal(out, thetas[i])
    # in place: theta_outs aliasing thetas
    before = [t.clone() for t in thetas]
    _, alphas, _ = b.line_search(thetas, ds, grads, L0, theta_outs=thetas)
    for i, m in enumerate(b.members):
        exp, _, _ = m.line_search(before[i], ds[i], grads[i], L0[i])
        assert torch.equal(thetas[i], exp)
    b.close()


def l0_fmt(x):
    return f"{x:.6e}"
