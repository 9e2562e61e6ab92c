"""Pins of the 3-D oracle (oracle/omt3_oracle.c), the method of Sec. 7.2 on
an m x n x p grid with App. A's discretisation along each axis (the paper
leaves 3-D as future work, Sec. 8.2).  None of them retypes the oracle:

* a single slice (p = 1, or n = 1, or m = 1) is the 2-D problem on the other
  two axes, and with the same h, mu, nu the 3-D iterates equal the 2-D
  oracle's (itself pinned by exact LPs and closed forms);
* permuting the axes permutes the iterates (catches an axis mixed up);
* for the norms ||u||_1, ||w||_1 the problem is a min-cost flow on the
  product of the 3-D grid and the channel graph, solved exactly by scipy
  HiGHS;
* data varying along z only: V = h sum |cumulative mass difference| (the
  1-D W1), for every u-norm;
* adjointness grad_x = -div_x^T, the first iterate phi = tau f, and the
  step rule's margin against the 3-D Laplacian's largest eigenvalue.
"""
import numpy as np
import pytest

import certify as CF
import oracle as O
import oracle.grid3 as G3
from paper_1712_10279_amd import inputs as I

NORMS = [(0, 0), (1, 0), (2, 1)]


def _state2to3(st, axis):
    """Insert a unit axis into a 2-D state so that it is the 3-D state of a
    single slice: axis 2 (z) keeps (u_x, u_y); axis 1 (y) maps the 2-D
    (u_x, u_y) to (u_x, u_z); axis 0 maps them to (u_y, u_z)."""
    z = np.zeros_like(st["phi"])
    if axis == 2:
        e = lambda a: a[:, :, None, :]  # noqa: E731
        return {"phi": e(st["phi"]), "ux": e(st["ux"]), "uy": e(st["uy"]), "uz": e(z), "w": e(st["w"])}
    if axis == 1:
        e = lambda a: a[:, None, :, :]  # noqa: E731
        return {"phi": e(st["phi"]), "ux": e(st["ux"]), "uy": e(z), "uz": e(st["uy"]), "w": e(st["w"])}
    e = lambda a: a[None, :, :, :]  # noqa: E731
    return {"phi": e(st["phi"]), "ux": e(z), "uy": e(st["ux"]), "uz": e(st["uy"]), "w": e(st["w"])}


@pytest.mark.parametrize("axis", [2, 1, 0])
@pytest.mark.parametrize("unorm,wnorm", NORMS)
@pytest.mark.parametrize("eps", [0.0, 0.7])
def test_single_slice_equals_two_dimensional_oracle(orc, axis, unorm, wnorm, eps):
    a, b = 9, 11
    r0, r1 = I.random_pair(41, a, b, 3)
    p2 = O.Problem(a, b, 3, edges=I.TRIANGLE, alpha=0.4, tau=1.5, unorm=unorm, wnorm=wnorm, eps=eps)
    f2, _ = O.prepare_f(r0, r1, p2.edges)
    s2 = O.solve(p2, f2, 300, 0.0, 1 << 30)["state"]
    shape = [a, b]
    shape.insert(axis, 1)
    e3 = lambda x: np.expand_dims(x, axis)  # noqa: E731
    q = G3.Problem3(*shape, 3, edges=I.TRIANGLE, alpha=0.4, tau=1.5, h=p2.h, mu=p2.mu, nu=p2.nu, unorm=unorm,
                    wnorm=wnorm, eps=eps)
    f3, _ = G3.prepare_f(e3(r0), e3(r1), q.edges)
    r3 = G3.solve(q, f3, 300, 0.0, 1 << 30)
    want = _state2to3(s2, axis)
    for key in ("phi", "ux", "uy", "uz", "w"):
        scale = max(np.abs(want[key]).max(), 1e-300)
        assert np.abs(r3["state"][key] - want[key]).max() <= 1e-13 * scale, key
    assert r3["residual"] > 0


@pytest.mark.parametrize("unorm", [0, 2])
def test_axis_permutation_permutes_iterates(orc, unorm):
    m, n, p = 4, 5, 7
    r0, r1 = I.random_volume_pair(42, m, n, p, 3)
    kw = dict(edges=I.TRIANGLE, alpha=0.5, tau=1.0, unorm=unorm, max_iters=200)
    ra = G3.solve_pair(r0, r1, **kw)["state"]
    t = lambda x: np.ascontiguousarray(np.transpose(x, (2, 1, 0, 3)))  # noqa: E731 (swap x and z)
    rb = G3.solve_pair(t(r0), t(r1), **kw)["state"]
    for ka, kb in (("phi", "phi"), ("ux", "uz"), ("uy", "uy"), ("uz", "ux"), ("w", "w")):
        scale = max(np.abs(ra[ka]).max(), 1e-300)
        assert np.abs(t(ra[ka]) - rb[kb]).max() <= 1e-12 * scale, (ka, kb)


@pytest.mark.parametrize("m,n,p,k,edges,alpha", [
    (3, 4, 3, 3, I.TRIANGLE, 0.3),
    (4, 3, 3, 2, [(0, 1)], 1.0),
    (3, 3, 4, 1, np.zeros((0, 2)), 1.0),
])
def test_l1_norms_match_exact_min_cost_flow_3d(orc, m, n, p, k, edges, alpha):
    r0, r1 = I.random_volume_pair(43, m, n, p, k)
    edges = np.asarray(edges, np.int32).reshape(-1, 2)
    h = 1.0 / (max(m, n, p) - 1)
    V = CF.lp_value3(r0, r1, edges, np.ones(len(edges)), alpha, h)
    r = G3.solve_pair(r0, r1, edges, alpha=alpha, tau=1.0, unorm=1, wnorm=0, max_iters=400000, tol=1e-11)
    assert r["converged"]
    assert r["primal"] == pytest.approx(V, rel=1e-8)
    assert r["dual"] == pytest.approx(V, rel=1e-8)


@pytest.mark.parametrize("unorm", [0, 1, 2])
def test_z_strips_closed_form(orc, unorm):
    # data constant over (i, j), one channel: V = h sum_z |F_z| (1-D W1 along z)
    m, n, p = 4, 3, 9
    rng = np.random.default_rng(44)
    a, b = rng.random(p) + 0.1, rng.random(p) + 0.1
    r0 = np.broadcast_to(a[None, None, :, None], (m, n, p, 1)).copy()
    r1 = np.broadcast_to(b[None, None, :, None], (m, n, p, 1)).copy()
    r0 /= r0.sum()
    r1 /= r1.sum()
    h = 1.0 / (max(m, n, p) - 1)
    F = np.cumsum((r0 - r1).sum(axis=(0, 1, 3)))
    V = h * np.abs(F[:-1]).sum()
    r = G3.solve_pair(r0, r1, np.zeros((0, 2)), unorm=unorm, max_iters=400000, tol=1e-11)
    assert r["primal"] == pytest.approx(V, rel=1e-9)


def test_gradient_is_minus_adjoint_of_divergence(orc):
    rng = np.random.default_rng(45)
    m, n, p, k = 4, 5, 6, 2
    q = G3.Problem3(m, n, p, k)
    phi = rng.normal(size=(m, n, p, k))
    st = {"phi": phi, "ux": rng.normal(size=phi.shape), "uy": rng.normal(size=phi.shape),
          "uz": rng.normal(size=phi.shape), "w": np.zeros((m, n, p, 0))}
    st["ux"][-1] = 0
    st["uy"][:, -1] = 0
    st["uz"][:, :, -1] = 0
    # one step from phi = 0 with mu -> 0 is phi1 = tau (div u_bar + f): use the
    # step's div through f = 0, mu tiny, so u1 ~ u and u_bar ~ u
    h = q.h
    gx = np.zeros_like(phi)
    gy = np.zeros_like(phi)
    gz = np.zeros_like(phi)
    gx[:-1] = (phi[1:] - phi[:-1]) / h
    gy[:, :-1] = (phi[:, 1:] - phi[:, :-1]) / h
    gz[:, :, :-1] = (phi[:, :, 1:] - phi[:, :, :-1]) / h
    qq = G3.Problem3(m, n, p, k, tau=1.0, mu=1e-300, h=h)
    zero = dict(st, phi=np.zeros_like(phi))
    div = G3.step(qq, np.zeros_like(phi), zero)["phi"]  # = tau * div(2 u1 - u) with u1 = shrink(u, 1e-300) = u
    lhs = (gx * st["ux"]).sum() + (gy * st["uy"]).sum() + (gz * st["uz"]).sum()
    rhs = -(phi * div).sum()
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_first_iterate_and_monotone_residual(orc):
    r0, r1 = I.random_volume_pair(46, 5, 6, 4, 3)
    q = G3.Problem3(5, 6, 4, 3, edges=I.TRIANGLE, alpha=0.6, tau=2.0)
    f, _ = G3.prepare_f(r0, r1, q.edges)
    s1 = G3.step(q, f, G3.zero_state(q))
    assert np.array_equal(s1["phi"], q.tau * f)
    for key in ("ux", "uy", "uz", "w"):
        assert not s1[key].any()
    met = G3.metrics(q, f, G3.zero_state(q), s1)
    assert met[0] == pytest.approx(q.tau * (f * f).sum(), rel=1e-14)
    res, st = [], None
    for _ in range(8):
        r = G3.solve(q, f, 64, 0.0, 64, st)
        st = r["state"]
        res.append(r["R"])
    assert all(b <= a * (1 + 1e-12) for a, b in zip(res, res[1:]))


@pytest.mark.parametrize("m,n,p", [(4, 4, 4), (5, 3, 6)])
def test_step_rule_margin_on_3d_laplacian(orc, m, n, p):
    # largest eigenvalue of -div_x grad_x (Neumann, App. A) on the 3-D grid,
    # assembled column by column from the oracle's own operators
    q = G3.Problem3(m, n, p, 1, tau=1.0, mu=1e-300)
    N = m * n * p
    A = np.zeros((N, N))
    h = q.h
    for col in range(N):
        e = np.zeros((m, n, p, 1))
        e.reshape(-1)[col] = 1.0
        gx = np.zeros_like(e)
        gy = np.zeros_like(e)
        gz = np.zeros_like(e)
        gx[:-1] = (e[1:] - e[:-1]) / h
        gy[:, :-1] = (e[:, 1:] - e[:, :-1]) / h
        gz[:, :, :-1] = (e[:, :, 1:] - e[:, :, :-1]) / h
        st = {"phi": np.zeros_like(e), "ux": gx, "uy": gy, "uz": gz, "w": np.zeros((m, n, p, 0))}
        A[:, col] = -G3.step(q, np.zeros_like(e), st)["phi"].reshape(-1)  # -(div grad e), tau = 1
    lam = np.linalg.eigvalsh((A + A.T) / 2).max()
    assert lam < 12.0 / h ** 2
    qd = G3.Problem3(m, n, p, 3, edges=I.TRIANGLE, tau=2.5)
    assert qd.tau * qd.mu * lam <= 0.25 + 1e-12  # the 2-D rule's margin
    assert qd.tau * qd.mu * lam + qd.tau * qd.nu * 3.0 < 1.0  # convergence condition (Sec. 7.2)
    qs = G3.Problem3(m, n, p, 1, tau=2.5)
    assert qs.tau * qs.mu * lam <= 0.5 + 1e-12
