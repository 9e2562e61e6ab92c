"""FP64 CPU oracle of the matrix-OMT PDHG method (arXiv 1712.10279, Sec. 4
and Sec. 7.3).

TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded FP64 C code
(``momt_oracle.c``) reached through ctypes; it works on whole complex k x k
matrices.  Only ``tests/``, the smoke check and the CPU-baseline leg of the
benchmark may import it; the product path never does.

Arrays are numpy ``complex128``: ``Phi``, ``f``, ``Lambda``, ``Ux``, ``Uy``
are ``(m, n, k, k)``, ``W`` is ``(m, n, l, k, k)`` and ``L`` is ``(l, k, k)``.
Norm codes (Sec. 6.2): 0 ``||.||_2`` (Frobenius of the whole block),
1 ``||.||_1`` (sum of the moduli of the entries), 2 ``||.||_{1,nuc}`` (sum of
nuclear norms).
"""
from __future__ import annotations

import ctypes as C
import time
from dataclasses import dataclass

import numpy as np

from . import lib

FRO, L1, NUC = 0, 1, 2

_dp = C.POINTER(C.c_double)


class _MProblem(C.Structure):
    _fields_ = [("m", C.c_int), ("n", C.c_int), ("k", C.c_int), ("l", C.c_int), ("L", _dp),
                ("alpha", C.c_double), ("tau", C.c_double), ("mu", C.c_double),
                ("nu", C.c_double), ("h", C.c_double), ("unorm", C.c_int), ("wnorm", C.c_int)]


class _MInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("R", C.c_double), ("residual", C.c_double),
                ("primal", C.c_double), ("dual", C.c_double), ("rel_gap", C.c_double),
                ("mass_residual", C.c_double), ("converged", C.c_int)]


def _lib():
    L = lib()
    if not getattr(L, "_matrix_ready", False):
        L.morc_lambda_max.restype = C.c_double
        L.morc_norm_block.restype = C.c_double
        L.morc_prepare_f.restype = C.c_double
        L.morc_solve.restype = C.c_int
        L._matrix_ready = True
    return L


def _c(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _p(a):
    return a.ctypes.data_as(_dp)


@dataclass
class MProblem:
    m: int
    n: int
    L: np.ndarray
    alpha: float = 1.0
    tau: float = 1.0
    mu: float = 0.0
    nu: float = 0.0
    h: float = 0.0
    unorm: int = FRO
    wnorm: int = L1

    def __post_init__(self):
        self.L = _c(self.L)
        if self.L.ndim == 2:
            self.L = self.L[None]
        self.l, self.k = self.L.shape[0], self.L.shape[1]
        c = self._c()
        _lib().morc_default_steps(C.byref(c))
        self.h, self.mu, self.nu = c.h, c.mu, c.nu

    def _c(self):
        return _MProblem(self.m, self.n, self.k, self.l, _p(self.L), self.alpha, self.tau, self.mu, self.nu,
                         self.h, self.unorm, self.wnorm)


def grad_L(L, X):
    """(L_s X - X L_s)_s of one k x k matrix (Sec. 4.1)."""
    L, X = _c(L), _c(X)
    Z = np.zeros((L.shape[0],) + X.shape, np.complex128)
    _lib().morc_grad_L(X.shape[0], L.shape[0], _p(L), _p(X), _p(Z))
    return Z


def div_L(L, Z):
    """sum_s (-L_s Z_s + Z_s L_s) (Sec. 4.1)."""
    L, Z = _c(L), _c(Z)
    X = np.zeros(Z.shape[1:], np.complex128)
    _lib().morc_div_L(Z.shape[1], L.shape[0], _p(L), _p(Z), _p(X))
    return X


def lambda_max(L) -> float:
    """lambda_max(-Delta_L) from the k^2 x k^2 matrix of -Delta_L (Sec. 7.3)."""
    L = _c(L)
    return _lib().morc_lambda_max(L.shape[1], L.shape[0], _p(L))


def shrink_block(kind, herm, X, t):
    """Prox of t * norm over a block of matrices (count, k, k) (App. B)."""
    X = _c(X).copy()
    _lib().morc_shrink_block(kind, int(herm), X.shape[1], X.shape[0], _p(X), C.c_double(t))
    return X


def norm_block(kind, herm, X) -> float:
    X = _c(X)
    return _lib().morc_norm_block(kind, int(herm), X.shape[1], X.shape[0], _p(X))


def prepare_f(lam0, lam1):
    """f = Lambda1 - Lambda0 minus its trace mean times I; returns (f, rel. imbalance)."""
    lam0, lam1 = _c(lam0), _c(lam1)
    f = np.zeros_like(lam0)
    m, n, k = lam0.shape[:3]
    imb = _lib().morc_prepare_f(m, n, k, _p(lam0), _p(lam1), _p(f))
    return f, imb


def zero_state(p: MProblem):
    z = np.zeros((p.m, p.n, p.k, p.k), np.complex128)
    return {"phi": z.copy(), "ux": z.copy(), "uy": z.copy(),
            "w": np.zeros((p.m, p.n, p.l, p.k, p.k), np.complex128)}


def step(p: MProblem, f, state):
    """One bare iteration of the M-OMT method (Sec. 7.3)."""
    f = _c(f)
    s = {key: _c(v) for key, v in state.items()}
    out = {key: np.zeros_like(v) for key, v in s.items()}
    pc = p._c()
    _lib().morc_step(C.byref(pc), _p(f), _p(s["phi"]), _p(s["ux"]), _p(s["uy"]), _p(s["w"]),
                     _p(out["phi"]), _p(out["ux"]), _p(out["uy"]), _p(out["w"]))
    return out


def solve(p: MProblem, f, max_iters: int, tol: float = 0.0, check_every: int = 64, state=None, hist_cap=4096):
    f = _c(f)
    s = zero_state(p) if state is None else {key: _c(v).copy() for key, v in state.items()}
    info = _MInfo()
    hist = np.zeros(hist_cap)
    pc = p._c()
    t0 = time.perf_counter()
    nchk = _lib().morc_solve(C.byref(pc), _p(f), _p(s["phi"]), _p(s["ux"]), _p(s["uy"]), _p(s["w"]),
                             C.c_int64(max_iters), C.c_double(tol), check_every, C.byref(info),
                             hist.ctypes.data_as(_dp), hist_cap)
    wall = time.perf_counter() - t0
    return {"state": s, "iters": int(info.iters), "R": info.R, "residual": info.residual,
            "primal": info.primal, "dual": info.dual, "rel_gap": info.rel_gap,
            "mass_residual": info.mass_residual, "converged": bool(info.converged),
            "hist": hist[:min(nchk, hist_cap)].copy(), "wall_s": wall}


def potential(phi):
    """Exported potential -Phi with (mean trace / k) I removed: the derivative
    of M with respect to Lambda0 (dual problem, Sec. 4.2)."""
    phi = _c(phi)
    k = phi.shape[-1]
    out = -phi.copy()
    t = np.trace(out, axis1=-2, axis2=-1).real.mean() / k
    out -= t * np.eye(k)
    return out


def solve_pair(lam0, lam1, L, alpha=1.0, tau=1.0, unorm=FRO, wnorm=L1, max_iters=1000, tol=0.0, check_every=64,
               mu=0.0, nu=0.0, h=0.0):
    lam0 = _c(lam0)
    m, n = lam0.shape[:2]
    p = MProblem(m, n, L, alpha=alpha, tau=tau, mu=mu, nu=nu, h=h, unorm=unorm, wnorm=wnorm)
    f, _ = prepare_f(lam0, lam1)
    r = solve(p, f, max_iters, tol, check_every)
    r["problem"] = p
    r["f"] = f
    r["Phi"] = potential(r["state"]["phi"])
    return r
