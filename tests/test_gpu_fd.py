"""Finite-difference study of the differentiable loss against the FP64
oracle's gradient (dual problem, Sec. 3.2: dV/drho0 = Phi).

64 x 64, k = 3 triangle, the loss workload's generator at that size,
FP64.  The base problem is solved to a relative residual of 1e-7; 64
random (pixel, channel) directions d_p = e_p - 1/N (zero total mass, so the
mass class stays balanced) are applied to rho0 with step 1e-4 in both
signs, and the 128 perturbed problems are solved together in one batched
solve, each started from the base solution.  V is convex in rho0 (it is a
norm of rho0 - rho1), so for any optimal potential the one-sided
differences bracket <Phi, d_p> = Phi_p up to the solve tolerance, and the
central difference lies within the bracket's width of it; Phi is the
oracle's, run to the same residual (tests/golden/fd_potential_64x64_k3.npz,
written by tests/golden/make_fd_potential.py).
"""
import os

import numpy as np
import pytest

from gpu_util import cuda, note, to_dev
from paper_1712_10279_amd import inputs as I

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fd_potential_64x64_k3.npz")


def test_central_differences_against_oracle_gradient():
    torch = cuda()
    from paper_1712_10279_amd import omt
    g = np.load(GOLDEN)
    Phi_orc = g["Phi"]
    tol, tau = float(g["tol"]), float(g["tau"])
    side, delta, nprobe = 64, 1e-4, 64
    d = I.loss_512(0, m=side, n=side)
    r0, r1 = d["rho0"], d["rho1"]
    dev = lambda x: to_dev(torch, x, torch.float64)
    note(f"case: FD study 64x64 k3, base solve to {tol:g}")
    base = omt.Solver(dev(r0), dev(r1), d["edges"], alpha=d["alpha"], tau=tau)
    info = base.solve(20_000_000, tol, 64)
    assert info["converged"]
    V0 = base.distance()[0]
    Phi_gpu = base.grad()[0].cpu().numpy()
    note(f"base: {info['iters']} iterations (oracle {int(g['iters'])}), V {V0:.12g} (oracle {float(g['V']):.12g}), "
         f"max|Phi_gpu - Phi_orc| {np.abs(Phi_gpu - Phi_orc).max():.2e} of {np.abs(Phi_orc).max():.2e}")
    assert abs(V0 - float(g["V"])) <= 1e-6 * V0
    st = base.get_state()
    N = r0.size
    rng = np.random.default_rng(64)
    picks = rng.choice(N, size=nprobe, replace=False)
    probs, dirs = [], []
    for p in picks:
        dp = -np.full(N, 1.0 / N)
        dp[p] += 1.0
        dp = dp.reshape(r0.shape)
        dirs.append(dp)
        for sgn in (1.0, -1.0):
            probs.append(dict(rho0=dev(r0 + sgn * delta * dp), rho1=dev(r1), edges=d["edges"], alpha=d["alpha"],
                              tau=tau))
    b = omt.BatchSolver(probs)
    for q in range(len(probs)):
        b.set_state(q, st["phi"], st["u"], st["w"])
    infos = b.solve(20_000_000, tol, 64)
    assert all(i["converged"] for i in infos)
    V = b.distance()
    note(f"perturbed solves: iterations min {min(i['iters'] for i in infos)} max {max(i['iters'] for i in infos)}")
    slack = 1e-4  # solve tolerance in V over the step: |dV| <~ 1e-8 / 1e-4
    worst_c, worst_b = 0.0, 0.0
    for q, (p, dp) in enumerate(zip(picks, dirs)):
        vp, vm = V[2 * q], V[2 * q + 1]
        lo, hi, cen = (V0 - vm) / delta, (vp - V0) / delta, (vp - vm) / (2 * delta)
        gq = float((Phi_orc * dp).sum())
        worst_b = max(worst_b, lo - gq, gq - hi)
        worst_c = max(worst_c, abs(cen - gq) - (hi - lo))
        assert lo - slack <= gq <= hi + slack, (q, lo, gq, hi)
        assert abs(cen - gq) <= 1e-3 * max(1.0, abs(gq)) + (hi - lo), (q, cen, gq, hi - lo)
    note(f"64 directions: bracket violation {worst_b:.2e}, central difference beyond bracket width {worst_c:.2e}")
