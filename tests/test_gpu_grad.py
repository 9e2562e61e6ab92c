"""The differentiable loss: backward returns dV/drho0 = Phi and dV/drho1 =
-Phi (dual problem, Sec. 3.2).  Checked against the oracle's potential, the
convexity sandwich of one-sided differences, and central differences."""
import numpy as np
import pytest

import oracle as O
from gpu_util import cuda, note, to_dev
from paper_1712_10279_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_loss_backward_matches_oracle_potential():
    torch = cuda()
    from paper_1712_10279_amd import omt
    r0, r1 = I.random_pair(70, 20, 24, 3)
    a = to_dev(torch, r0, torch.float64).requires_grad_(True)
    b = to_dev(torch, r1, torch.float64).requires_grad_(True)
    V = omt.omt_loss(a, b, I.TRIANGLE, max_iters=3000, tol=0.0, tau=1.0)
    V.backward()
    r = O.solve_pair(r0, r1, I.TRIANGLE, tau=1.0, max_iters=3000)
    note(f"V gpu {V.item():.12g} oracle {r['primal']:.12g}")
    assert abs(V.item() - r["primal"]) <= 1e-9 * r["primal"]
    assert np.abs(a.grad.cpu().numpy() - r["Phi"]).max() <= 1e-9 * np.abs(r["Phi"]).max()
    assert torch.equal(b.grad, -a.grad)


def test_loss_finite_differences():
    """Converged FP64 solves: one-sided differences bracket <Phi, d> and the
    central difference approximates it (V is convex in rho0).  Perturbed
    solves start from the base solution."""
    torch = cuda()
    from paper_1712_10279_amd import omt
    m, n = 16, 18
    r0, r1 = I.random_pair(71, m, n, 3)
    tol, cap = 1e-8, 2_000_000
    base = omt.Solver(to_dev(torch, r0, torch.float64), to_dev(torch, r1, torch.float64), I.TRIANGLE, tau=2.0)
    info = base.solve(cap, tol, 64)
    note(f"base: {info['iters']} iterations, residual {info['residual']:.2e}")
    assert info["converged"]
    V0 = base.distance()[0]
    Phi = base.grad()[0].cpu().numpy()
    st = base.get_state()
    rng = np.random.default_rng(3)
    N = r0.size
    delta = 1e-3

    def V_at(rho0):
        s = omt.Solver(to_dev(torch, rho0, torch.float64), to_dev(torch, r1, torch.float64), I.TRIANGLE, tau=2.0)
        s.set_state(st["phi"], st["u"], st["w"])
        assert s.solve(cap, tol, 64)["converged"]
        return s.distance()[0]

    for q in range(6):
        p = int(rng.integers(N))
        d = -np.full(N, 1.0 / N)
        d[p] += 1.0
        d = d.reshape(r0.shape)
        vp, vm = V_at(r0 + delta * d), V_at(r0 - delta * d)
        g = float((Phi * d).sum())
        lo, hi, cen = (V0 - vm) / delta, (vp - V0) / delta, (vp - vm) / (2 * delta)
        note(f"  d{q}: one-sided [{lo:.6f}, {hi:.6f}] central {cen:.6f} <Phi,d> {g:.6f}")
        slack = 1e-4
        assert lo - slack <= g <= hi + slack
        assert abs(cen - g) <= 1e-3 * max(1.0, abs(g)) + (hi - lo)


def test_batched_loss_shapes():
    torch = cuda()
    from paper_1712_10279_amd import omt
    pairs = [I.random_pair(72 + q, 12, 14, 3) for q in range(3)]
    a = torch.stack([to_dev(torch, p[0], torch.float32) for p in pairs]).requires_grad_(True)
    b = torch.stack([to_dev(torch, p[1], torch.float32) for p in pairs])
    V = omt.omt_loss(a, b, I.TRIANGLE, max_iters=500, tol=0.0)
    assert V.shape == (3,)
    wts = torch.tensor([1.0, -2.0, 0.5], device="cuda")
    (V * wts).sum().backward()
    assert a.grad.shape == a.shape
    for q in range(3):
        # the batched forward solves every pair exactly as its own solve does
        s = omt.Solver(a[q].detach(), b[q], I.TRIANGLE)
        s.solve(500, 0.0, 64)
        assert float(V[q].detach()) == float(torch.tensor(s.distance()[0], dtype=torch.float32))
        assert torch.equal(wts[q] * s.grad()[0], a.grad[q])


def test_batched_loss_falls_back_for_graphs_the_batch_does_not_compile():
    torch = cuda()
    from paper_1712_10279_amd import omt
    pairs = [I.random_pair(80 + q, 10, 12, 5) for q in range(2)]
    a = torch.stack([to_dev(torch, p[0], torch.float32) for p in pairs]).requires_grad_(True)
    b = torch.stack([to_dev(torch, p[1], torch.float32) for p in pairs])
    V = omt.omt_loss(a, b, I.path_edges(5), max_iters=200, tol=0.0)
    V.sum().backward()
    s = omt.Solver(a[1].detach(), b[1], I.path_edges(5))
    s.solve(200, 0.0, 64)
    assert torch.equal(s.grad()[0], a.grad[1])


def test_loss_flags_unconverged_solves():
    torch = cuda()
    from paper_1712_10279_amd import omt
    note("case: loss stopped above tol, 20x24 k3, 128 iterations")
    r0, r1 = I.random_pair(72, 20, 24, 3)
    a = to_dev(torch, r0, torch.float64)
    b = to_dev(torch, r1, torch.float64)
    with pytest.warns(omt.NotConvergedWarning):
        omt.omt_loss(a, b, I.TRIANGLE, max_iters=128, tol=1e-9, tau=1.0)
    with pytest.raises(omt.OMTError) as e:
        omt.omt_loss(a[None], b[None], I.TRIANGLE, max_iters=128, tol=1e-9, tau=1.0, on_notconv="raise")
    assert e.value.status == omt.ENOTCONV
