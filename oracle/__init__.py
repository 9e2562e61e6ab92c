"""FP64 CPU oracle of the vector-OMT PDHG method (arXiv 1712.10279).

TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded FP64 C code
(``omt_oracle.c``) reached through ctypes.  Only ``tests/``, the smoke check
and the CPU-baseline leg of the benchmark may import this package; the
product path never does, and shares no code with it.

Arrays use the paper's layout (App. A): ``[i][j][c]`` with the channel index
fastest; ``phi``, ``f``, ``ux``, ``uy`` are ``(m, n, k)``, ``w`` is
``(m, n, l)``.  Norm codes: u -- 0 sum-of-2-norms per channel (L12), 1 L1,
2 Frobenius (L2); w -- 0 L1, 1 L2 (Sec. 6.2).
"""
from __future__ import annotations

import ctypes as C
import os
import time
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("OMT_ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))
_lib = None

U_L12, U_L1, U_L2 = 0, 1, 2
W_L1, W_L2 = 0, 1

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class _Problem(C.Structure):
    _fields_ = [("m", C.c_int), ("n", C.c_int), ("k", C.c_int), ("l", C.c_int),
                ("edges", _ip), ("cost", _dp),
                ("alpha", C.c_double), ("tau", C.c_double), ("mu", C.c_double),
                ("nu", C.c_double), ("h", C.c_double),
                ("unorm", C.c_int), ("wnorm", C.c_int), ("eps", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("iters", C.c_int64), ("R", C.c_double), ("residual", C.c_double),
                ("primal", C.c_double), ("dual", C.c_double), ("rel_gap", C.c_double),
                ("mass_residual", C.c_double), ("converged", C.c_int)]


def lib():
    """Load ``liboracle.so``, building it with gcc if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_graph_lambda_max.restype = C.c_double
        L.orc_sym_lambda_max.restype = C.c_double
        L.orc_shrink1.restype = C.c_double
        L.orc_norm_u.restype = C.c_double
        L.orc_norm_w.restype = C.c_double
        L.orc_prepare_f.restype = C.c_double
        L.orc_solve.restype = C.c_int
        L.orc_mass_classes.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class Problem:
    """Discrete V-OMT problem (App. A) with PDHG steps (Sec. 7.2)."""
    m: int
    n: int
    k: int
    edges: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))
    cost: np.ndarray | None = None
    alpha: float = 1.0
    tau: float = 1.0
    mu: float = 0.0
    nu: float = 0.0
    h: float = 0.0
    unorm: int = U_L12
    wnorm: int = W_L1
    eps: float = 0.0

    def __post_init__(self):
        self.edges = np.ascontiguousarray(np.asarray(self.edges, dtype=np.int32).reshape(-1, 2))
        if self.cost is None:
            self.cost = np.ones(len(self.edges))
        self.cost = _f64(self.cost).reshape(-1)
        self._fill_steps()

    @property
    def l(self) -> int:
        return int(self.edges.shape[0])

    def _c(self) -> _Problem:
        return _Problem(self.m, self.n, self.k, self.l, _i(self.edges), _d(self.cost),
                        self.alpha, self.tau, self.mu, self.nu, self.h, self.unorm, self.wnorm, self.eps)

    def _fill_steps(self):
        p = self._c()
        lib().orc_default_steps(C.byref(p))
        self.h, self.mu, self.nu = p.h, p.mu, p.nu


# ------------------------------------------------------------ operators

def incidence(k: int, edges) -> np.ndarray:
    e = np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2))
    D = np.zeros((k, len(e)))
    lib().orc_incidence(k, len(e), _i(e), _d(D))
    return D


def graph_lambda_max(k: int, edges, cost=None) -> float:
    e = np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2))
    c = _f64(np.ones(len(e)) if cost is None else cost)
    return lib().orc_graph_lambda_max(k, len(e), _i(e), _d(c))


def sym_lambda_max(A) -> float:
    A = _f64(A)
    return lib().orc_sym_lambda_max(A.shape[0], _d(A))


def mass_classes(k: int, edges) -> np.ndarray:
    e = np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2))
    cls = np.zeros(k, np.int32)
    lib().orc_mass_classes(k, len(e), _i(e), _i(cls))
    return cls


def grad_x(phi, h):
    phi = _f64(phi)
    m, n, k = phi.shape
    gx, gy = np.zeros_like(phi), np.zeros_like(phi)
    lib().orc_grad_x(m, n, k, C.c_double(h), _d(phi), _d(gx), _d(gy))
    return gx, gy


def div_x(ux, uy, h):
    ux, uy = _f64(ux), _f64(uy)
    m, n, k = ux.shape
    out = np.zeros_like(ux)
    lib().orc_div_x(m, n, k, C.c_double(h), _d(ux), _d(uy), _d(out))
    return out


def grad_G(phi, edges, cost=None):
    phi = _f64(phi)
    m, n, k = phi.shape
    e = np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2))
    c = _f64(np.ones(len(e)) if cost is None else cost)
    out = np.zeros((m, n, len(e)))
    lib().orc_grad_G(m, n, k, len(e), _i(e), _d(c), _d(phi), _d(out))
    return out


def div_G(w, k, edges, cost=None):
    w = _f64(w)
    m, n, l = w.shape
    e = np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2))
    c = _f64(np.ones(len(e)) if cost is None else cost)
    out = np.zeros((m, n, k))
    lib().orc_div_G(m, n, k, l, _i(e), _d(c), _d(w), _d(out))
    return out


def shrink1(x: float, t: float) -> float:
    return lib().orc_shrink1(C.c_double(x), C.c_double(t))


def shrink2(x, t):
    x = _f64(x).copy()
    lib().orc_shrink2(len(x), _d(x), C.c_double(t))
    return x


def shrink_u(unorm, bx, by, t):
    bx, by = _f64(bx).copy(), _f64(by).copy()
    lib().orc_shrink_u(unorm, len(bx), _d(bx), _d(by), C.c_double(t))
    return bx, by


def shrink_w(wnorm, w, t):
    w = _f64(w).copy()
    lib().orc_shrink_w(wnorm, len(w), _d(w), C.c_double(t))
    return w


def prepare_f(rho0, rho1, edges):
    """f = rho1 - rho0 minus its mean per mass class; also the imbalance."""
    rho0, rho1 = _f64(rho0), _f64(rho1)
    m, n, k = rho0.shape
    e = np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2))
    f = np.zeros_like(rho0)
    imb = lib().orc_prepare_f(m, n, k, len(e), _i(e), _d(rho0), _d(rho1), _d(f))
    return f, imb


def zero_state(p: Problem):
    z = np.zeros((p.m, p.n, p.k))
    return {"phi": z.copy(), "ux": z.copy(), "uy": z.copy(), "w": np.zeros((p.m, p.n, max(p.l, 0)))}


def step(p: Problem, f, state):
    """One PDHG iteration (Sec. 7.2) from ``state``; returns the new state."""
    f = _f64(f)
    s = {key: _f64(v) for key, v in state.items()}
    o = {key: np.zeros_like(v) for key, v in s.items()}
    pc = p._c()
    w_in = s["w"] if p.l > 0 else np.zeros(1)
    w_out = o["w"] if p.l > 0 else np.zeros(1)
    lib().orc_step(C.byref(pc), _d(f), _d(s["phi"]), _d(s["ux"]), _d(s["uy"]), _d(w_in),
                   _d(o["phi"]), _d(o["ux"]), _d(o["uy"]), _d(w_out))
    return o


def metrics(p: Problem, f, old, new):
    """(R, primal, dual, ||div u + div_G w + f||^2, ||f||^2) for the step old -> new."""
    f = _f64(f)
    a = {key: _f64(v) for key, v in old.items()}
    b = {key: _f64(v) for key, v in new.items()}
    out = np.zeros(5)
    pc = p._c()
    wa = a["w"] if p.l > 0 else np.zeros(1)
    wb = b["w"] if p.l > 0 else np.zeros(1)
    lib().orc_metrics(C.byref(pc), _d(f), _d(a["phi"]), _d(a["ux"]), _d(a["uy"]), _d(wa),
                      _d(b["phi"]), _d(b["ux"]), _d(b["uy"]), _d(wb), _d(out))
    return out


def solve(p: Problem, f, max_iters: int, tol: float = 0.0, check_every: int = 64, state=None,
          hist_cap: int = 100000):
    """Run the method from ``state`` (zeros if None).  Returns a dict with the
    final state, the info of the last check, the residual history and the
    wall time of the iteration loop."""
    f = _f64(f)
    s = zero_state(p) if state is None else {key: _f64(v).copy() for key, v in state.items()}
    info = _Info()
    hist = np.zeros(hist_cap)
    pc = p._c()
    w_arr = s["w"] if p.l > 0 else np.zeros(1)
    t0 = time.perf_counter()
    nchk = lib().orc_solve(C.byref(pc), _d(f), _d(s["phi"]), _d(s["ux"]), _d(s["uy"]), _d(w_arr),
                           C.c_int64(max_iters), C.c_double(tol), check_every, C.byref(info),
                           _d(hist), hist_cap)
    wall = time.perf_counter() - t0
    if p.l > 0:
        s["w"] = w_arr
    return {
        "state": s,
        "iters": int(info.iters), "R": info.R, "residual": info.residual,
        "primal": info.primal, "dual": info.dual, "rel_gap": info.rel_gap,
        "mass_residual": info.mass_residual, "converged": bool(info.converged),
        "hist": hist[:min(nchk, hist_cap)].copy(), "wall_s": wall,
    }


def potential(phi, edges):
    """Exported potential: Phi = -phi with its mean over each mass class removed
    (the derivative of V with respect to rho0; dual objective of Sec. 3.2)."""
    phi = _f64(phi)
    k = phi.shape[2]
    cls = mass_classes(k, edges)
    out = -phi.copy()
    for g in np.unique(cls):
        sel = cls == g
        out[:, :, sel] -= out[:, :, sel].mean()
    return out


def solve_pair(rho0, rho1, edges, alpha=1.0, tau=1.0, cost=None, unorm=U_L12, wnorm=W_L1,
               max_iters=1000, tol=0.0, check_every=64, h=0.0, mu=0.0, nu=0.0, eps=0.0):
    """Convenience: problem set-up + f + solve from zeros."""
    rho0 = _f64(rho0)
    m, n, k = rho0.shape
    p = Problem(m, n, k, edges=edges, cost=cost, alpha=alpha, tau=tau, h=h, mu=mu, nu=nu,
                unorm=unorm, wnorm=wnorm, eps=eps)
    f, _ = prepare_f(rho0, rho1, p.edges)
    r = solve(p, f, max_iters, tol, check_every)
    r["problem"] = p
    r["f"] = f
    r["Phi"] = potential(r["state"]["phi"], p.edges)
    return r
