"""Independent checks used to pin the oracle (and, through it, the HIP path).

Everything here is written from the mathematics of the discrete problem of
App. A, separately from the oracle's C code:

* ``lp_value``: with the norms ||u||_1 and ||w||_1 the discrete V-OMT problem
  is an uncapacitated min-cost flow on the product graph grid x channel graph
  (spatial arcs cost h, channel arcs cost alpha c_e, supply rho0 - rho1),
  solved exactly by scipy's HiGHS.
* ``lower_bound``: any potential scaled into the dual feasible set of the
  dual problem (Sec. 3.2) gives <phi, rho1 - rho0> <= V.
* ``upper_bound``: any (u, w) repaired to satisfy the constraint exactly gives
  ||u|| + alpha ||w|| >= V.
* closed forms for strips, large alpha and small alpha.
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------ operators

def np_div_x(ux, uy, h):
    """Backward differences with zero flux; ghost entries are ignored."""
    m, n, _ = ux.shape
    x = ux.copy()
    y = uy.copy()
    x[m - 1] = 0.0
    y[:, n - 1] = 0.0
    out = x.copy()
    out[1:] -= x[:-1]
    out += y
    out[:, 1:] -= y[:, :-1]
    return out / h


def np_grad_x(phi, h):
    gx = np.zeros_like(phi)
    gy = np.zeros_like(phi)
    gx[:-1] = (phi[1:] - phi[:-1]) / h
    gy[:, :-1] = (phi[:, 1:] - phi[:, :-1]) / h
    return gx, gy


def np_incidence(k, edges):
    D = np.zeros((k, len(edges)))
    for e, (a, b) in enumerate(edges):
        D[min(a, b), e] = 1.0
        D[max(a, b), e] = -1.0
    return D


def np_div_G(w, k, edges, cost):
    D = np_incidence(k, edges)
    return -(w / cost) @ D.T


def np_grad_G(phi, edges, cost):
    D = np_incidence(phi.shape[2], edges)
    return (phi @ D) / cost


def u_norm_sum(ux, uy, unorm):
    if unorm == 0:
        return np.sqrt(ux ** 2 + uy ** 2).sum()
    if unorm == 1:
        return np.abs(ux).sum() + np.abs(uy).sum()
    return np.sqrt((ux ** 2 + uy ** 2).sum(axis=2)).sum()


def w_norm_sum(w, wnorm):
    if w.size == 0:
        return 0.0
    if wnorm == 0:
        return np.abs(w).sum()
    return np.sqrt((w ** 2).sum(axis=2)).sum()


# -------------------------------------------------------- certificates

def lower_bound(phi, f, h, edges, cost, alpha, unorm=0, wnorm=0):
    """<phi_s, f> for phi_s = phi / s, s the smallest factor making phi_s dual
    feasible (||grad phi||_{u*} <= 1 and ||grad_G phi||_{w*} <= alpha per pixel)."""
    gx, gy = np_grad_x(phi, h)
    if unorm == 0:
        su = np.sqrt(gx ** 2 + gy ** 2).max()
    elif unorm == 1:
        su = max(np.abs(gx).max(), np.abs(gy).max())
    else:
        su = np.sqrt((gx ** 2 + gy ** 2).sum(axis=2)).max()
    sw = 0.0
    if len(edges):
        gG = np_grad_G(phi, edges, cost)
        sw = (np.abs(gG).max() if wnorm == 0 else np.sqrt((gG ** 2).sum(axis=2)).max()) / alpha
    s = max(su, sw)
    if s <= 0:
        return 0.0
    return float((phi * f).sum() / s)


def repair(ux, uy, w, f, h, edges, cost):
    """(ux', uy', w') with div_x u' + div_G w' + f = 0 exactly (up to
    rounding): first the per-channel totals of the residual are moved
    between channels at pixel (0, 0), then every channel's zero-sum residual
    is routed along rows and down the last column."""
    m, n, k = f.shape
    ux = ux.copy()
    uy = uy.copy()
    ux[m - 1] = 0.0
    uy[:, n - 1] = 0.0
    w = w.copy()
    dG = np_div_G(w, k, edges, cost) if len(edges) else np.zeros_like(f)
    r = -(np_div_x(ux, uy, h) + dG + f)
    if len(edges):
        R = r.sum(axis=(0, 1))
        D = np_incidence(k, edges)
        # div_G dw = -D diag(1/c) dw = R  ->  g = -dw / c,  D g = R
        g, *_ = np.linalg.lstsq(D, R, rcond=None)
        dw = -g * cost
        w[0, 0] += dw
        r[0, 0] -= np_div_G(dw[None, None, :], k, edges, cost)[0, 0]
    for c in range(k):
        rc = r[:, :, c]
        cum = np.cumsum(rc, axis=1)          # route along each row (y direction)
        uy[:, : n - 1, c] += h * cum[:, : n - 1]
        rows = cum[:, n - 1]                  # what is left sits in column n-1
        cr = np.cumsum(rows)
        ux[: m - 1, n - 1, c] += h * cr[: m - 1]
    return ux, uy, w


def upper_bound(ux, uy, w, f, h, edges, cost, alpha, unorm=0, wnorm=0):
    ux2, uy2, w2 = repair(ux, uy, w, f, h, edges, cost)
    return float(u_norm_sum(ux2, uy2, unorm) + alpha * w_norm_sum(w2, wnorm)), (ux2, uy2, w2)


# -------------------------------------------------------------- exact LP

def lp_value(rho0, rho1, edges, cost, alpha, h):
    """Exact V for the norms ||u||_1, ||w||_1: min-cost flow on grid x G."""
    from scipy.optimize import linprog
    from scipy.sparse import coo_matrix

    m, n, k = rho0.shape
    node = lambda i, j, c: (i * n + j) * k + c  # noqa: E731
    rows, cols, vals, costs = [], [], [], []
    a = 0

    def arc(s, t, cst):
        nonlocal a
        rows.extend([s, t])
        cols.extend([a, a])
        vals.extend([1.0, -1.0])
        costs.append(cst)
        a += 1

    for i in range(m):
        for j in range(n):
            for c in range(k):
                if i + 1 < m:
                    arc(node(i, j, c), node(i + 1, j, c), h)
                    arc(node(i + 1, j, c), node(i, j, c), h)
                if j + 1 < n:
                    arc(node(i, j, c), node(i, j + 1, c), h)
                    arc(node(i, j + 1, c), node(i, j, c), h)
            for e, (p, q) in enumerate(edges):
                arc(node(i, j, p), node(i, j, q), alpha * cost[e])
                arc(node(i, j, q), node(i, j, p), alpha * cost[e])
    A = coo_matrix((vals, (rows, cols)), shape=(m * n * k, a)).tocsr()
    b = (rho0 - rho1).reshape(-1)
    res = linprog(np.array(costs), A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    assert res.status == 0, res.message
    return float(res.fun)


# ---------------------------------------------------------- closed forms

def strip_value(rho0, rho1, h):
    """Data constant along j, one channel: V = h sum_i |F_i| with F_i the
    cumulative mass difference over rows 0..i (the 1-D W1 distance)."""
    F = np.cumsum((rho0 - rho1).sum(axis=(1, 2)))
    return float(h * np.abs(F[:-1]).sum())


def w1_triangle(a, b):
    """W1 on the unit-cost complete graph on 3 nodes: half the l1 distance."""
    return 0.5 * np.abs(a - b).sum(axis=-1)


def w1_path(a, b):
    """W1 on the unit-cost path graph: sum of |cumulative differences|."""
    return np.abs(np.cumsum(a - b, axis=-1)[..., :-1]).sum(axis=-1)


def lp_value3(rho0, rho1, edges, cost, alpha, h):
    """Exact V for the norms ||u||_1, ||w||_1 on an m x n x p grid: min-cost
    flow on (3-D grid) x G, arcs of cost h between face neighbours along each
    axis and alpha c_e between the channels of an edge at one pixel."""
    from scipy.optimize import linprog
    from scipy.sparse import coo_matrix

    m, n, p, k = rho0.shape
    node = lambda i, j, z, c: ((i * n + j) * p + z) * k + c  # noqa: E731
    rows, cols, vals, costs = [], [], [], []
    a = 0

    def arc(s, t, cst):
        nonlocal a
        rows.extend([s, t])
        cols.extend([a, a])
        vals.extend([1.0, -1.0])
        costs.append(cst)
        a += 1

    for i in range(m):
        for j in range(n):
            for z in range(p):
                for c in range(k):
                    for (di, dj, dz) in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                        if i + di < m and j + dj < n and z + dz < p:
                            arc(node(i, j, z, c), node(i + di, j + dj, z + dz, c), h)
                            arc(node(i + di, j + dj, z + dz, c), node(i, j, z, c), h)
                for e, (q0, q1) in enumerate(edges):
                    arc(node(i, j, z, q0), node(i, j, z, q1), alpha * cost[e])
                    arc(node(i, j, z, q1), node(i, j, z, q0), alpha * cost[e])
    A = coo_matrix((vals, (rows, cols)), shape=(m * n * p * k, a)).tocsr()
    b = (rho0 - rho1).reshape(-1)
    res = linprog(np.array(costs), A_eq=A, b_eq=b, bounds=(0, None), method="highs")
    assert res.status == 0, res.message
    return float(res.fun)
