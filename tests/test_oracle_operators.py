"""Pins of the oracle's building blocks against the paper and the mathematics.

Each test checks the oracle against something other than itself: the
printed incidence matrix (Sec. 3.1), closed-form spectra, adjointness stated
in Sec. 3.1 and App. A, and the optimality conditions that define the shrink
operators (App. B).
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1712_10279_amd import inputs as I

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _read_incidence_golden():
    rows, edges = [], None
    with open(os.path.join(GOLD, "incidence_fig_graph_example.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("edges:"):
                edges = [tuple(int(t) for t in p.split()) for p in line[6:].split(",")]
            else:
                rows.append([float(t) for t in line.split()])
    return edges, np.array(rows)


def test_incidence_matches_printed_example(orc):
    edges, D_printed = _read_incidence_golden()
    D = orc.incidence(4, edges)
    assert np.array_equal(D, D_printed)


@pytest.mark.parametrize("k", [2, 3, 5, 8])
def test_graph_lambda_max_path_closed_form(orc, k):
    # Laplacian of the unit path on k nodes: eigenvalues 2 - 2 cos(pi q / k).
    edges = [(c, c + 1) for c in range(k - 1)]
    assert orc.graph_lambda_max(k, edges) == pytest.approx(2 + 2 * math.cos(math.pi / k), abs=1e-13)


@pytest.mark.parametrize("k", [2, 3, 4, 6])
def test_graph_lambda_max_complete_closed_form(orc, k):
    # Laplacian of the unit complete graph K_k: eigenvalues 0 and k.
    edges = [(a, b) for a in range(k) for b in range(a + 1, k)]
    assert orc.graph_lambda_max(k, edges) == pytest.approx(k, abs=1e-12)


def test_graph_lambda_max_weighted_vs_library(orc):
    rng = np.random.default_rng(3)
    edges = [(0, 1), (0, 2), (1, 2), (1, 3), (2, 4), (3, 4)]
    cost = rng.uniform(0.3, 2.0, len(edges))
    D = np.zeros((5, len(edges)))
    for e, (a, b) in enumerate(edges):
        D[a, e], D[b, e] = 1, -1
    ref = np.linalg.eigvalsh(D @ np.diag(1 / cost ** 2) @ D.T).max()
    assert orc.graph_lambda_max(5, edges, cost) == pytest.approx(ref, rel=1e-12)


def test_graph_lambda_max_single_edge_and_empty(orc):
    assert orc.graph_lambda_max(2, [(0, 1)]) == pytest.approx(2.0, abs=1e-14)
    assert orc.graph_lambda_max(1, np.zeros((0, 2))) == 0.0


@pytest.mark.parametrize("m,n", [(4, 4), (5, 7), (8, 3)])
def test_grid_laplacian_full_spectrum(orc, m, n):
    # -div_x grad_x with zero-flux ghosts is the Neumann 5-point Laplacian,
    # whose eigenvalues are (4/h^2)(sin^2(pi p/2m) + sin^2(pi q/2n)).
    h = 1.0 / (max(m, n) - 1)
    N = m * n
    A = np.zeros((N, N))
    for t in range(N):
        e = np.zeros((m, n, 1))
        e.reshape(-1)[t] = 1.0
        gx, gy = orc.grad_x(e, h)
        A[:, t] = -orc.div_x(gx, gy, h).reshape(-1)
    assert np.allclose(A, A.T, atol=1e-12)
    ev = np.sort(np.linalg.eigvalsh(A))
    p, q = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    ref = np.sort((4 / h ** 2 * (np.sin(np.pi * p / (2 * m)) ** 2 + np.sin(np.pi * q / (2 * n)) ** 2)).ravel())
    assert np.allclose(ev, ref, rtol=1e-10, atol=1e-9)
    # the bound lambda_max(-Delta_x) <= 8/h^2 used for mu (Sec. 7.1)
    assert ev.max() * h * h < 8.0


def test_spatial_adjoint(orc):
    # grad_x is the transpose of -div_x (App. A), ghost entries included.
    rng = np.random.default_rng(0)
    m, n, k = 6, 9, 3
    h = 1.0 / 8
    phi = rng.standard_normal((m, n, k))
    ux, uy = rng.standard_normal((m, n, k)), rng.standard_normal((m, n, k))
    ux[m - 1] = 0
    uy[:, n - 1] = 0
    gx, gy = orc.grad_x(phi, h)
    lhs = (gx * ux).sum() + (gy * uy).sum()
    rhs = -(phi * orc.div_x(ux, uy, h)).sum()
    assert lhs == pytest.approx(rhs, rel=1e-13, abs=1e-12)
    # ghosts of grad are zero
    assert np.all(gx[m - 1] == 0) and np.all(gy[:, n - 1] == 0)


def test_graph_adjoint_and_laplacian(orc):
    # div_G = -grad_G^* and Delta_G = div_G grad_G = -D diag(1/c^2) D^T (Sec. 3.1).
    rng = np.random.default_rng(1)
    m, n, k = 3, 4, 4
    edges = [(0, 1), (0, 2), (1, 2), (0, 3), (2, 3)]
    cost = rng.uniform(0.5, 2.0, 5)
    phi = rng.standard_normal((m, n, k))
    w = rng.standard_normal((m, n, 5))
    gG = orc.grad_G(phi, edges, cost)
    assert (gG * w).sum() == pytest.approx(-(phi * orc.div_G(w, k, edges, cost)).sum(), rel=1e-13)
    _, D = _read_incidence_golden()
    lap = orc.div_G(orc.grad_G(phi, edges, cost), k, edges, cost)
    ref = -np.einsum("ck,ijk->ijc", D @ np.diag(1 / cost ** 2) @ D.T, phi)
    assert np.allclose(lap, ref, atol=1e-13)
    # grad_G of one pixel: (phi_a - phi_b) / c_e
    assert gG[1, 2, 3] == pytest.approx((phi[1, 2, 0] - phi[1, 2, 3]) / cost[3])


# ------------------------------------------------------------- shrinks

def _prox_ok(x, z, t, norm, dual_norm, grad):
    """z = argmin t*norm(z) + 1/2 |z - x|^2  iff  (x - z)/t is a subgradient
    of the norm at z: norm(z) = <g, z> and dual_norm(g) <= 1."""
    g = (x - z) / t
    return dual_norm(g) <= 1 + 1e-12 and abs(norm(z) - float(np.dot(g, z))) <= 1e-12 * (1 + norm(z))


def test_shrink1_definition(orc):
    # App. B: (1 - t/|x|) x for |x| >= t, else 0; ties give 0.
    assert orc.shrink1(3.0, 1.0) == 2.0
    assert orc.shrink1(-3.0, 1.0) == -2.0
    assert orc.shrink1(0.5, 1.0) == 0.0
    assert orc.shrink1(1.0, 1.0) == 0.0
    assert orc.shrink1(0.0, 1.0) == 0.0


@pytest.mark.parametrize("d", [1, 2, 3, 7])
def test_shrink2_is_prox_of_euclidean_norm(orc, d):
    rng = np.random.default_rng(d)
    for _ in range(200):
        x = rng.standard_normal(d) * rng.uniform(0.1, 3)
        t = rng.uniform(0.05, 2)
        z = orc.shrink2(x, t)
        assert _prox_ok(x, z, t, np.linalg.norm, np.linalg.norm, None)
    assert np.all(orc.shrink2(np.zeros(d), 1.0) == 0)


def test_shrink_u_norms_are_prox(orc):
    rng = np.random.default_rng(7)
    k = 3
    for unorm, norm, dual in [
        (orc.U_L12, lambda v: sum(np.hypot(v[:k], v[k:])), lambda g: np.hypot(g[:k], g[k:]).max()),
        (orc.U_L1, lambda v: np.abs(v).sum(), lambda g: np.abs(g).max()),
        (orc.U_L2, np.linalg.norm, np.linalg.norm),
    ]:
        for _ in range(200):
            bx, by = rng.standard_normal(k), rng.standard_normal(k)
            t = rng.uniform(0.1, 1.5)
            zx, zy = orc.shrink_u(unorm, bx, by, t)
            x = np.concatenate([bx, by])
            z = np.concatenate([zx, zy])
            assert _prox_ok(x, z, t, norm, dual, None), unorm


def test_shrink_w_norms_are_prox(orc):
    rng = np.random.default_rng(8)
    for wnorm, norm, dual in [(orc.W_L1, lambda v: np.abs(v).sum(), lambda g: np.abs(g).max()),
                              (orc.W_L2, np.linalg.norm, np.linalg.norm)]:
        for _ in range(200):
            w = rng.standard_normal(4)
            t = rng.uniform(0.1, 1.5)
            z = orc.shrink_w(wnorm, w, t)
            assert _prox_ok(w, z, t, norm, dual, None)


# ----------------------------------------------------------- set-up

def test_default_steps_rule(orc):
    # mu = 1/(32 tau (n-1)^2), nu = 1/(4 tau lambda_max) (Sec. 7.2);
    # mu = 1/(16 tau (n-1)^2) without edges (Sec. 7.1).
    p = orc.Problem(33, 33, 3, edges=[(0, 1), (0, 2), (1, 2)], tau=3.0)
    assert p.h == pytest.approx(1 / 32)
    assert p.mu == pytest.approx(1 / (32 * 3.0 * 32 ** 2))
    assert p.nu == pytest.approx(1 / (4 * 3.0 * 3.0))
    # step-size condition of Sec. 7.2 with the grid bound 8/h^2
    assert p.tau * p.mu * 8 / p.h ** 2 + p.tau * p.nu * 3.0 < 1
    q = orc.Problem(17, 9, 1, tau=1.0)
    assert q.h == pytest.approx(1 / 16) and q.mu == pytest.approx(1 / (16 * 16 ** 2)) and q.nu == 0.0


def test_mass_classes_and_mean_removal(orc):
    cls = orc.mass_classes(5, [(0, 1), (3, 4)])
    assert cls[0] == cls[1] and cls[3] == cls[4] and len(set(cls.tolist())) == 3
    rng = np.random.default_rng(2)
    r0, r1 = rng.random((4, 5, 5)), rng.random((4, 5, 5))
    f, imb = orc.prepare_f(r0, r1, [(0, 1), (3, 4)])
    for group in ([0, 1], [2], [3, 4]):
        assert abs(f[:, :, group].sum()) < 1e-12
    # f differs from rho1 - rho0 only by a constant per class
    d = f - (r1 - r0)
    for group in ([0, 1], [2], [3, 4]):
        assert np.ptp(d[:, :, group]) < 1e-14
    assert imb > 0


def test_second_iterate_worked_by_hand(orc):
    with open(os.path.join(GOLD, "second_iterate_2x2x2.json")) as fh:
        g = json.load(fh)
    s = (1 - 1 / math.sqrt(2)) / 32
    ev = lambda v: [eval(x, {"s": s, "sqrt": math.sqrt}) if isinstance(x, str) else float(x) for x in v]  # noqa: E731
    p = orc.Problem(2, 2, 2, edges=[(0, 1)], alpha=0.5, tau=1.0)
    assert p.h == 1.0 and p.mu == 1 / 32 and p.nu == pytest.approx(1 / 8, rel=1e-14)
    f = np.zeros((2, 2, 2))
    f[:, :, 0] = np.array(ev(g["f_ch0"])).reshape(2, 2)
    f[:, :, 1] = np.array(ev(g["f_ch1"])).reshape(2, 2)
    s1 = orc.step(p, f, orc.zero_state(p))
    assert np.all(s1["ux"] == 0) and np.all(s1["uy"] == 0) and np.all(s1["w"] == 0)
    assert np.array_equal(s1["phi"], p.tau * f)
    s2 = orc.step(p, f, s1)
    assert np.allclose(s2["ux"][:, :, 0].ravel(), ev(g["ux2_ch0"]), atol=1e-16)
    assert np.allclose(s2["uy"][:, :, 0].ravel(), ev(g["uy2_ch0"]), atol=1e-16)
    assert np.all(s2["ux"][:, :, 1] == 0) and np.all(s2["uy"][:, :, 1] == 0)
    assert np.allclose(s2["w"][:, :, 0].ravel(), ev(g["w2"]), atol=1e-16)
    assert np.allclose(s2["phi"][:, :, 0].ravel(), ev(g["phi2_ch0"]), atol=1e-15)
    assert np.allclose(s2["phi"][:, :, 1].ravel(), ev(g["phi2_ch1"]), atol=1e-15)


def test_second_iterate_check_quantities_worked_by_hand(orc):
    """R^k (Sec. 6.1, 1/nu on the w block), primal and dual objectives, gap and
    constraint residual of the step 1 -> 2 of the hand-worked 2x2x2 problem."""
    with open(os.path.join(GOLD, "second_iterate_2x2x2.json")) as fh:
        g = json.load(fh)
    s = (1 - 1 / math.sqrt(2)) / 32
    ev = lambda x: eval(x, {"s": s, "sqrt": math.sqrt})  # noqa: E731
    p = orc.Problem(2, 2, 2, edges=[(0, 1)], alpha=0.5, tau=1.0)
    f = np.zeros((2, 2, 2))
    f[:, :, 0] = np.array(g["f_ch0"], float).reshape(2, 2)
    s1 = orc.step(p, f, orc.zero_state(p))
    s2 = orc.step(p, f, s1)
    met = orc.metrics(p, f, s1, s2)
    assert met[0] == pytest.approx(ev(g["R2"]), rel=1e-13)
    assert met[1] == pytest.approx(ev(g["primal2"]), rel=1e-13)
    assert met[2] == pytest.approx(ev(g["dual2"]), rel=1e-13)
    assert met[3] == pytest.approx(ev(g["mass2_sq"]), rel=1e-13)
    assert met[4] == pytest.approx(ev(g["fnorm2"]), rel=1e-15)
    # the same through the solver's report after exactly two iterations
    r = orc.solve(p, f, 2, 0.0, 64)
    P, D = ev(g["primal2"]), ev(g["dual2"])
    assert r["iters"] == 2
    assert r["mass_residual"] == pytest.approx(math.sqrt(ev(g["mass2_sq"]) / ev(g["fnorm2"])), rel=1e-13)
    assert r["rel_gap"] == pytest.approx((P - D) / P, rel=1e-13)
    assert r["residual"] == pytest.approx(math.sqrt(ev(g["R2"]) / (p.tau * ev(g["fnorm2"]))), rel=1e-13)


@pytest.mark.parametrize("k,edges", [(3, I.TRIANGLE), (4, I.path_edges(4)), (1, np.zeros((0, 2)))])
def test_mass_residual_is_one_after_the_first_step(orc, k, edges):
    """From the zero start the first step leaves u = w = 0 (Sec. 7.2), so the
    constraint residual div_x u + div_G w + f equals f: relative value 1."""
    r0, r1 = I.random_pair(41, 7, 9, k)
    r = orc.solve_pair(r0, r1, edges, max_iters=1)
    assert r["mass_residual"] == 1.0
    assert r["primal"] == 0.0
