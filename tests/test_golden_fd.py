"""The stored oracle potential of the finite-difference study
(tests/golden/fd_potential_64x64_k3.npz, written by make_fd_potential.py)
is a near-optimal dual solution of its problem (dual problem, Sec. 3.2):
zero mean over the mass class, the Euler identity V = <Phi, rho0 - rho1>,
and dual feasibility |grad Phi| <= 1 per channel and |Phi_a - Phi_b| <=
alpha per edge, each to the run's tolerance."""
import os

import numpy as np

import oracle as O
from paper_1712_10279_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fd_potential_64x64_k3.npz")


def test_stored_potential_is_dual_optimal():
    g = np.load(GOLDEN)
    Phi, V = g["Phi"], float(g["V"])
    d = I.loss_512(0, m=64, n=64)
    assert Phi.shape == (64, 64, 3)
    assert abs(Phi.mean()) < 1e-12
    f, _ = O.prepare_f(d["rho0"], d["rho1"], d["edges"])
    # <Phi, rho0 - rho1> with the class mean removed from rho1 - rho0
    euler = float((Phi * -f).sum())
    assert abs(euler - V) <= 1e-6 * V, (euler, V)
    h = 1.0 / 63
    gx = np.zeros_like(Phi)
    gy = np.zeros_like(Phi)
    gx[:-1] = (Phi[1:] - Phi[:-1]) / h
    gy[:, :-1] = (Phi[:, 1:] - Phi[:, :-1]) / h
    assert np.sqrt(gx ** 2 + gy ** 2).max() <= 1.0 + 1e-2
    for a, b in d["edges"]:
        assert np.abs(Phi[..., a] - Phi[..., b]).max() <= d["alpha"] * (1.0 + 1e-2)
