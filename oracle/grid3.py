"""3-D grids: ctypes wrappers of the FP64 oracle in ``omt3_oracle.c``.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Arrays are
``[i][j][z][c]`` with the channel fastest: ``phi``, ``f``, ``ux``, ``uy``,
``uz`` are ``(m, n, p, k)``, ``w`` is ``(m, n, p, l)``.  The discretisation is
App. A carried to three axes (the paper names 3-D imaging as future work,
Sec. 8.2): see the header of ``omt3_oracle.c`` for the readings.
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass, field

import numpy as np

from . import _d, _f64, _i, _Info, lib, prepare_f as _prepare_f_2d, potential as _potential_2d

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Problem3(C.Structure):
    _fields_ = [("m", C.c_int), ("n", C.c_int), ("p", C.c_int), ("k", C.c_int), ("l", C.c_int),
                ("edges", _ip), ("cost", _dp),
                ("alpha", C.c_double), ("tau", C.c_double), ("mu", C.c_double),
                ("nu", C.c_double), ("h", C.c_double),
                ("unorm", C.c_int), ("wnorm", C.c_int), ("eps", C.c_double)]


@dataclass
class Problem3:
    """Discrete vector-OMT problem on an m x n x p grid."""
    m: int
    n: int
    p: int
    k: int
    edges: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    cost: np.ndarray | None = None
    alpha: float = 1.0
    tau: float = 1.0
    mu: float = 0.0
    nu: float = 0.0
    h: float = 0.0
    unorm: int = 0
    wnorm: int = 0
    eps: float = 0.0

    def __post_init__(self):
        self.edges = np.ascontiguousarray(np.asarray(self.edges, dtype=np.int32).reshape(-1, 2))
        if self.cost is None:
            self.cost = np.ones(len(self.edges))
        self.cost = _f64(self.cost).reshape(-1)
        c = self._c()
        lib().orc3_default_steps(C.byref(c))
        self.h, self.mu, self.nu = c.h, c.mu, c.nu

    @property
    def l(self) -> int:
        return int(self.edges.shape[0])

    def _c(self) -> _Problem3:
        return _Problem3(self.m, self.n, self.p, self.k, self.l, _i(self.edges), _d(self.cost), self.alpha,
                         self.tau, self.mu, self.nu, self.h, self.unorm, self.wnorm, self.eps)


def prepare_f(rho0, rho1, edges):
    """f = rho1 - rho0 minus its mean per mass class (the 2-D routine on the
    pixels laid end to end: only the channel structure matters)."""
    rho0, rho1 = _f64(rho0), _f64(rho1)
    m, n, p, k = rho0.shape
    f, imb = _prepare_f_2d(rho0.reshape(m * n * p, 1, k), rho1.reshape(m * n * p, 1, k), edges)
    return f.reshape(m, n, p, k), imb


def zero_state(q: Problem3):
    z = np.zeros((q.m, q.n, q.p, q.k))
    return {"phi": z.copy(), "ux": z.copy(), "uy": z.copy(), "uz": z.copy(),
            "w": np.zeros((q.m, q.n, q.p, max(q.l, 0)))}


def step(q: Problem3, f, state):
    """One iteration of Sec. 7.2 on the 3-D grid from ``state``."""
    f = _f64(f)
    s = {key: _f64(v) for key, v in state.items()}
    o = {key: np.zeros_like(v) for key, v in s.items()}
    w_in = s["w"] if q.l > 0 else np.zeros(1)
    w_out = o["w"] if q.l > 0 else np.zeros(1)
    c = q._c()
    lib().orc3_step(C.byref(c), _d(f), _d(s["phi"]), _d(s["ux"]), _d(s["uy"]), _d(s["uz"]), _d(w_in),
                    _d(o["phi"]), _d(o["ux"]), _d(o["uy"]), _d(o["uz"]), _d(w_out))
    return o


def metrics(q: Problem3, f, old, new):
    """(R, primal, dual, ||div u + div_G w + f||^2, ||f||^2) of old -> new."""
    f = _f64(f)
    a = {key: _f64(v) for key, v in old.items()}
    b = {key: _f64(v) for key, v in new.items()}
    wa = a["w"] if q.l > 0 else np.zeros(1)
    wb = b["w"] if q.l > 0 else np.zeros(1)
    out = np.zeros(5)
    c = q._c()
    lib().orc3_metrics(C.byref(c), _d(f), _d(a["phi"]), _d(a["ux"]), _d(a["uy"]), _d(a["uz"]), _d(wa),
                       _d(b["phi"]), _d(b["ux"]), _d(b["uy"]), _d(b["uz"]), _d(wb), _d(out))
    return out


def solve(q: Problem3, f, max_iters: int, tol: float = 0.0, check_every: int = 64, state=None):
    """Run the method from ``state`` (zeros if None)."""
    f = _f64(f)
    s = zero_state(q) if state is None else {key: _f64(v).copy() for key, v in state.items()}
    info = _Info()
    w_arr = s["w"] if q.l > 0 else np.zeros(1)
    c = q._c()
    t0 = time.perf_counter()
    lib().orc3_solve(C.byref(c), _d(f), _d(s["phi"]), _d(s["ux"]), _d(s["uy"]), _d(s["uz"]), _d(w_arr),
                     C.c_int64(max_iters), C.c_double(tol), check_every, C.byref(info))
    wall = time.perf_counter() - t0
    if q.l > 0:
        s["w"] = w_arr
    return {"state": s, "iters": int(info.iters), "R": info.R, "residual": info.residual, "primal": info.primal,
            "dual": info.dual, "rel_gap": info.rel_gap, "mass_residual": info.mass_residual,
            "converged": bool(info.converged), "wall_s": wall}


def potential(phi, edges):
    """Phi = -phi with its mean per mass class removed."""
    phi = _f64(phi)
    m, n, p, k = phi.shape
    return _potential_2d(phi.reshape(m * n * p, 1, k), edges).reshape(m, n, p, k)


def solve_pair(rho0, rho1, edges, alpha=1.0, tau=1.0, cost=None, unorm=0, wnorm=0, max_iters=1000, tol=0.0,
               check_every=64, h=0.0, mu=0.0, nu=0.0, eps=0.0, state=None):
    rho0 = _f64(rho0)
    m, n, p, k = rho0.shape
    q = Problem3(m, n, p, k, edges=edges, cost=cost, alpha=alpha, tau=tau, h=h, mu=mu, nu=nu, unorm=unorm,
                 wnorm=wnorm, eps=eps)
    f, _ = prepare_f(rho0, rho1, q.edges)
    r = solve(q, f, max_iters, tol, check_every, state)
    r["problem"] = q
    r["f"] = f
    r["Phi"] = potential(r["state"]["phi"], q.edges)
    return r
