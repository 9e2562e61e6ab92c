"""Solver-level pins of the oracle (run to convergence on small grids).

The transport cost V of the discrete problem (App. A) is pinned by:
* an exact min-cost-flow LP for the norms ||u||_1, ||w||_1 (scipy HiGHS);
* the closed form for strips (1-D W1 = h sum |cumulative rho0 - rho1|);
* closed forms for large alpha (channels decouple) and small alpha (pure
  colour change at every pixel), derived from the dual problem of Sec. 3.2;
* a certified bracket [dual-feasible lower bound, repaired-primal upper
  bound] for the isotropic norm ||u||_{1,2} on general data;
* invariants: R^k decreases monotonically (Sec. 6.1), R^0 = tau ||f||^2,
  the metric properties (Sec. 3.3), symmetry, shift and scale.
"""
import numpy as np
import pytest

import certify as CF
from paper_1712_10279_amd import inputs as I


def _solve(orc, r0, r1, edges, alpha=1.0, tau=1.0, unorm=0, wnorm=0, iters=400000, tol=1e-11, cost=None):
    return orc.solve_pair(r0, r1, edges, alpha=alpha, tau=tau, unorm=unorm, wnorm=wnorm,
                          max_iters=iters, tol=tol, cost=cost)


@pytest.mark.parametrize("m,n,k,edges,alpha", [
    (6, 7, 3, I.TRIANGLE, 0.3),
    (6, 7, 3, I.TRIANGLE, 1.0),
    (8, 8, 4, I.path_edges(4), 0.3),
    (5, 9, 2, [(0, 1)], 2.0),
    (7, 6, 1, np.zeros((0, 2)), 1.0),
])
def test_l1_norms_match_exact_min_cost_flow(orc, m, n, k, edges, alpha):
    r0, r1 = I.random_pair(11, m, n, k)
    h = 1.0 / (max(m, n) - 1)
    edges = np.asarray(edges, np.int32).reshape(-1, 2)
    V = CF.lp_value(r0, r1, edges, np.ones(len(edges)), alpha, h)
    r = _solve(orc, r0, r1, edges, alpha, unorm=orc.U_L1, wnorm=orc.W_L1)
    assert r["converged"]
    assert r["primal"] == pytest.approx(V, rel=1e-8)
    assert r["dual"] == pytest.approx(V, rel=1e-8)


def test_weighted_edges_match_min_cost_flow(orc):
    r0, r1 = I.random_pair(12, 6, 6, 3)
    cost = np.array([0.5, 2.0, 1.25])
    V = CF.lp_value(r0, r1, I.TRIANGLE, cost, 0.7, 0.2)
    r = _solve(orc, r0, r1, I.TRIANGLE, 0.7, unorm=orc.U_L1, wnorm=orc.W_L1, cost=cost)
    assert r["primal"] == pytest.approx(V, rel=1e-8)


@pytest.mark.parametrize("unorm", [0, 1, 2])
def test_strips_closed_form(orc, unorm):
    # Data constant along j, one channel: V = h sum_i |F_i| for every norm,
    # and grad phi is h sign(F_i) wherever F_i != 0 (Phi = -phi).
    m, n = 9, 6
    rng = np.random.default_rng(4)
    a, b = rng.random(m) + 0.1, rng.random(m) + 0.1
    r0 = np.repeat(a[:, None], n, 1)[:, :, None]
    r1 = np.repeat(b[:, None], n, 1)[:, :, None]
    r0 /= r0.sum()
    r1 /= r1.sum()
    h = 1.0 / (max(m, n) - 1)
    V = CF.strip_value(r0, r1, h)
    r = _solve(orc, r0, r1, np.zeros((0, 2)), unorm=unorm)
    assert r["primal"] == pytest.approx(V, rel=1e-9)
    F = np.cumsum((r0 - r1).sum(axis=(1, 2)))[:-1]
    phi = r["state"]["phi"][:, :, 0]
    d = phi[1:, :] - phi[:-1, :]
    sel = np.abs(F) > 1e-3 * np.abs(F).max()
    assert np.allclose(d[sel], (h * np.sign(F))[sel][:, None], atol=1e-7)


def test_large_alpha_decouples_channels(orc):
    # Every channel balanced and alpha >= the range of the channel potentials:
    # no colour change pays, V = sum_c V_c.  With strip data V_c is the 1-D W1.
    m, n, k = 8, 5, 3
    rng = np.random.default_rng(5)
    r0 = np.zeros((m, n, k))
    r1 = np.zeros((m, n, k))
    for c in range(k):
        a, b = rng.random(m) + 0.1, rng.random(m) + 0.1
        r0[:, :, c] = a[:, None] / a.sum() / n / k
        r1[:, :, c] = b[:, None] / b.sum() / n / k
    h = 1.0 / (max(m, n) - 1)
    V = sum(CF.strip_value(r0[:, :, c:c + 1], r1[:, :, c:c + 1], h) for c in range(k))
    r = _solve(orc, r0, r1, I.TRIANGLE, alpha=2.0)
    assert r["primal"] == pytest.approx(V, rel=1e-8)


@pytest.mark.parametrize("edges,w1", [(I.TRIANGLE, CF.w1_triangle), (I.path_edges(4), CF.w1_path)])
def test_small_alpha_pure_colour_change(orc, edges, w1):
    # Every pixel balanced across channels and alpha * diam(G) <= h / sqrt(2):
    # V = alpha sum_ij W1_G(rho0_ij, rho1_ij).
    m, n = 6, 7
    k = int(np.max(edges)) + 1
    diam = 1 if k == 3 else k - 1
    rng = np.random.default_rng(6)
    tot = rng.random((m, n)) + 0.5
    p0 = rng.dirichlet(np.ones(k), size=(m, n))
    p1 = rng.dirichlet(np.ones(k), size=(m, n))
    r0 = tot[:, :, None] * p0
    r1 = tot[:, :, None] * p1
    s = r0.sum()
    r0 /= s
    r1 /= s
    h = 1.0 / (max(m, n) - 1)
    alpha = 0.99 * h / np.sqrt(2) / diam
    V = alpha * w1(r0, r1).sum()
    r = _solve(orc, r0, r1, edges, alpha=alpha)
    assert r["primal"] == pytest.approx(V, rel=1e-8)


@pytest.mark.parametrize("unorm,wnorm", [(0, 0), (0, 1), (2, 0), (1, 1)])
def test_certified_bracket_general_data(orc, unorm, wnorm):
    # V lies in [<phi_s, f>, ||u_rep|| + alpha ||w_rep||] for any iterate;
    # at convergence the bracket closes around the oracle's primal value.
    m, n = 10, 12
    r0, r1 = I.random_pair(13, m, n, 3)
    h = 1.0 / (max(m, n) - 1)
    one = np.ones(3)
    r = _solve(orc, r0, r1, I.TRIANGLE, alpha=0.8, unorm=unorm, wnorm=wnorm, tol=1e-10)
    st = r["state"]
    lb = CF.lower_bound(st["phi"], r["f"], h, I.TRIANGLE, one, 0.8, unorm, wnorm)
    ub, _ = CF.upper_bound(st["ux"], st["uy"], st["w"], r["f"], h, I.TRIANGLE, one, 0.8, unorm, wnorm)
    assert lb <= ub * (1 + 1e-12)
    assert (ub - lb) / ub < 1e-7
    assert lb * (1 - 1e-7) <= r["primal"] <= ub * (1 + 1e-7)


def test_bracket_contains_v_early_and_tightens(orc):
    m, n = 12, 12
    r0, r1 = I.random_pair(14, m, n, 3)
    h = 1.0 / (m - 1)
    one = np.ones(3)
    widths = []
    for iters in (200, 2000, 20000):
        r = _solve(orc, r0, r1, I.TRIANGLE, iters=iters, tol=0.0)
        st = r["state"]
        lb = CF.lower_bound(st["phi"], r["f"], h, I.TRIANGLE, one, 1.0)
        ub, _ = CF.upper_bound(st["ux"], st["uy"], st["w"], r["f"], h, I.TRIANGLE, one, 1.0)
        assert lb <= ub
        widths.append(ub - lb)
    assert widths[0] > widths[1] > widths[2]


def test_residual_monotone_and_first_value(orc):
    # R^k decreases monotonically (Sec. 6.1); from zeros R^0 = tau ||f||^2.
    r0, r1 = I.random_pair(15, 16, 16, 3)
    p = orc.Problem(16, 16, 3, edges=I.TRIANGLE, tau=1.0)
    f, _ = orc.prepare_f(r0, r1, p.edges)
    r = orc.solve(p, f, 3000, 0.0, check_every=1)
    hist = r["hist"]
    assert hist[0] == pytest.approx(1.0, rel=1e-12)
    assert np.all(np.diff(hist) <= 1e-12 * hist[:-1])
    s1 = orc.step(p, f, orc.zero_state(p))
    met = orc.metrics(p, f, orc.zero_state(p), s1)
    assert met[0] == pytest.approx(p.tau * (f ** 2).sum(), rel=1e-14)


def test_metric_properties(orc):
    # V(a, a) = 0, symmetry with Phi -> -Phi, triangle inequality, shift and
    # scale invariance, alpha monotonicity (Sec. 3.3 and the primal form).
    m, n = 8, 8
    a, b = I.random_pair(16, m, n, 3)
    c, _ = I.random_pair(17, m, n, 3)
    V = lambda x, y, alpha=1.0: _solve(orc, x, y, I.TRIANGLE, alpha=alpha, tol=1e-11)  # noqa: E731
    rab, rba = V(a, b), V(b, a)
    assert V(a, a)["primal"] == 0.0
    assert rab["primal"] == pytest.approx(rba["primal"], rel=1e-8)
    assert np.allclose(rab["Phi"], -rba["Phi"], atol=1e-6)
    assert rab["primal"] <= V(a, c)["primal"] + V(c, b)["primal"] + 1e-9
    g = np.random.default_rng(0).random((m, n, 3))
    assert V(a + g, b + g)["primal"] == pytest.approx(rab["primal"], rel=1e-8)
    assert V(3 * a, 3 * b)["primal"] == pytest.approx(3 * rab["primal"], rel=1e-8)
    assert V(a, b, 0.5)["primal"] <= rab["primal"] + 1e-10 <= V(a, b, 2.0)["primal"] + 2e-10


def test_dual_mean_conserved_and_euler_identity(orc):
    r0, r1 = I.random_pair(18, 10, 9, 3)
    r = _solve(orc, r0, r1, I.TRIANGLE, tol=1e-11)
    phi = r["state"]["phi"]
    assert abs(phi.mean()) < 1e-13
    # V = <dV/drho0, rho0> + <dV/drho1, rho1> with dV/drho0 = Phi = -dV/drho1
    Phi = r["Phi"]
    assert (Phi * r0).sum() - (Phi * r1).sum() == pytest.approx(r["primal"], rel=1e-8)


def test_gradient_convexity_sandwich(orc):
    # V is convex in rho0 (a norm of rho0 - rho1), so one-sided differences
    # bracket the directional derivative <Phi, d> (Phi = dV/drho0).
    m, n = 7, 8
    r0, r1 = I.random_pair(19, m, n, 3)
    base = _solve(orc, r0, r1, I.TRIANGLE, tol=1e-12)
    Phi = base["Phi"]
    rng = np.random.default_rng(1)
    N = r0.size
    for _ in range(6):
        p = rng.integers(N)
        d = -np.full(N, 1.0 / N)
        d[p] += 1.0
        d = d.reshape(r0.shape)
        delta = 1e-4
        vp = _solve(orc, r0 + delta * d, r1, I.TRIANGLE, tol=1e-12)["primal"]
        vm = _solve(orc, r0 - delta * d, r1, I.TRIANGLE, tol=1e-12)["primal"]
        g = (Phi * d).sum()
        lo, hi = (base["primal"] - vm) / delta, (vp - base["primal"]) / delta
        slack = 1e-6
        assert lo - slack <= g <= hi + slack


@pytest.mark.parametrize("unorm", [0, 1, 2])
def test_regularised_strips_closed_form(orc, unorm):
    # Quadratic regularisation (Sec. 9), eps sum |u|^2: for strips the row sums
    # of u_x are forced (h F_i), and both |.| and |.|^2 are smallest with the
    # flux spread evenly over the n columns and u_y = 0, so
    # V_eps = h sum |F_i| + eps h^2 sum F_i^2 / n exactly.
    m, n = 9, 6
    rng = np.random.default_rng(8)
    a, b = rng.random(m) + 0.1, rng.random(m) + 0.1
    r0 = np.repeat(a[:, None], n, 1)[:, :, None]
    r1 = np.repeat(b[:, None], n, 1)[:, :, None]
    r0 /= r0.sum()
    r1 /= r1.sum()
    h = 1.0 / (max(m, n) - 1)
    F = np.cumsum((r0 - r1).sum(axis=(1, 2)))[:-1]
    eps = 3.0
    V = h * np.abs(F).sum() + eps * h * h * (F ** 2).sum() / n
    r = orc.solve_pair(r0, r1, np.zeros((0, 2)), unorm=unorm, eps=eps, max_iters=400000, tol=1e-11)
    assert r["primal"] == pytest.approx(V, rel=1e-9)
    ux = r["state"]["ux"][:-1, :, 0]
    assert np.allclose(ux, (h * F / n)[:, None], atol=1e-9)
    assert np.abs(r["state"]["uy"]).max() < 1e-9


def test_regularisation_vanishes_as_eps_goes_to_zero(orc):
    r0, r1 = I.random_pair(9, 8, 9, 3)
    base = _solve(orc, r0, r1, I.TRIANGLE, tol=1e-11)["primal"]
    vals = [orc.solve_pair(r0, r1, I.TRIANGLE, eps=e, max_iters=400000, tol=1e-11)["primal"] for e in (1e-1, 1e-2, 1e-3)]
    gaps = [v - base for v in vals]
    assert all(g >= -1e-10 for g in gaps)
    assert gaps[0] > gaps[1] > gaps[2]
    assert gaps[2] < 1e-3 * base


@pytest.mark.parametrize("k,edges,cost", [
    (2, [(0, 1)], [1.0]),
    (2, [(0, 1)], [2.0]),
    (3, I.path_edges(3), [1.0, 1.0]),
    (4, I.path_edges(4), [1.0, 0.5, 1.5]),
])
def test_regularised_pixel_balanced_closed_form(orc, k, edges, cost):
    # Quadratic regularisation (Sec. 9) with the transfer w active.  Every
    # pixel carries the same total mass in rho0 and rho1, and the graph is a
    # path.  With alpha and eps small against h no spatial flux pays: u = 0,
    # and the constraint div_G w = rho0 - rho1 (div_G = -D diag(1/c), Sec. 3.1)
    # fixes the transfer on the path's edge e = (e, e+1) at every pixel:
    #   w_e = c_e * sum_{c <= e} (rho1 - rho0)_c.
    # The unique optimum (the objective is strictly convex) therefore has
    #   V_eps = sum_pixels sum_e (alpha |w_e| + eps w_e^2).
    # Its dual potential satisfies the transfer's optimality condition at every
    # pixel, (phi_a - phi_b) / c_e = alpha sign(w_e) + 2 eps w_e, and the
    # potential built from these differences has spatial differences below
    # h / sqrt(2) per channel by the choice of alpha and eps (so u = 0 is
    # optimal: the dual constraint of the isotropic norm holds).
    m, n = 5, 6
    rng = np.random.default_rng(31 + k)
    tot = rng.random((m, n)) + 0.5
    r0 = tot[:, :, None] * rng.dirichlet(np.ones(k), size=(m, n))
    r1 = tot[:, :, None] * rng.dirichlet(np.ones(k), size=(m, n))
    scale = r0.sum()
    r0 /= scale
    r1 /= scale
    cost = np.asarray(cost, float)
    h = 1.0 / (max(m, n) - 1)
    F = np.cumsum(r1 - r0, axis=2)[:, :, :-1]          # sum_{c <= e} (rho1 - rho0)_c
    w_star = cost[None, None, :] * F
    wmax = np.abs(w_star).max()
    # per-pixel potential range <= sum_e c_e (alpha + 2 eps |w_e|); spatial
    # differences at most twice that; need sqrt(2) * 2 * range <= h
    budget = h / (2 * np.sqrt(2)) / cost.sum()
    alpha = 0.45 * budget
    eps = 0.45 * budget / (2 * wmax)
    V = (alpha * np.abs(w_star) + eps * w_star ** 2).sum()
    r = orc.solve_pair(r0, r1, edges, alpha=alpha, eps=eps, cost=cost, max_iters=2000000, tol=1e-12)
    assert r["converged"]
    st = r["state"]
    assert np.abs(st["ux"]).max() < 1e-9 * wmax and np.abs(st["uy"]).max() < 1e-9 * wmax
    assert np.allclose(st["w"], w_star, rtol=0, atol=1e-8 * wmax)
    assert r["primal"] == pytest.approx(V, rel=1e-9)
    # the regulariser term is a sizeable part of V, so dropping it is visible
    assert (eps * w_star ** 2).sum() > 0.05 * V
    # transfer optimality: (phi_a - phi_b) / c_e = alpha sign(w_e) + 2 eps w_e
    phi = st["phi"]
    dG = (phi[:, :, :-1] - phi[:, :, 1:]) / cost[None, None, :]
    want = alpha * np.sign(w_star) + 2 * eps * w_star
    assert np.abs(dG - want).max() < 1e-6 * alpha
    # at the optimum the constraint holds: relative residual -> 0
    assert r["mass_residual"] < 1e-8
