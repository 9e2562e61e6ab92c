"""Python binding of ``libomt.so`` (the C ABI of ``include/omt.h``).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  PyTorch provides device memory (the workspace and the caller's
tensors) and the current stream.  The library is loaded on first use; if it
is missing the binding raises instead of computing anything elsewhere.
"""
from __future__ import annotations

import ctypes as C
import os
import warnings
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# OMT_LIB selects another build of the same library (e.g. a variant built
# with different compile-time options); the default is the in-tree build.
LIB_PATH = os.environ.get("OMT_LIB", os.path.join(_HERE, "libomt.so"))

OK, EINVAL, EGRAPH, EMASS, ESTEP, ENOMEM, EDEVICE, ENOTCONV, EDIVERGED, EUNSUPPORTED = range(10)
U_L12, U_L1, U_L2 = 0, 1, 2
W_L1, W_L2 = 0, 1
F32, F64 = 0, 1
FLAG_COMPENSATED_PHI = 1
MAX_CHANNELS = 8


class Params(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("k", C.c_int32), ("n_edges", C.c_int32),
                ("edges", C.POINTER(C.c_int32)), ("edge_cost", C.POINTER(C.c_double)),
                ("alpha", C.c_double), ("tau", C.c_double), ("mu", C.c_double), ("nu", C.c_double),
                ("h", C.c_double), ("unorm", C.c_int32), ("wnorm", C.c_int32), ("dtype", C.c_int32),
                ("flags", C.c_uint32), ("tblock", C.c_int32), ("rows_per_wave", C.c_int32),
                ("reg_eps", C.c_double), ("p", C.c_int32)]


M_FRO, M_L1, M_NUC = 0, 1, 2


class MatrixParams(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("k", C.c_int32), ("n_L", C.c_int32),
                ("L", C.POINTER(C.c_double)), ("real", C.c_int32),
                ("alpha", C.c_double), ("tau", C.c_double), ("mu", C.c_double), ("nu", C.c_double),
                ("h", C.c_double), ("unorm", C.c_int32), ("wnorm", C.c_int32), ("dtype", C.c_int32),
                ("flags", C.c_int32), ("rows_per_wave", C.c_int32), ("tblock", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int64), ("residual", C.c_double), ("primal", C.c_double), ("dual", C.c_double),
                ("rel_gap", C.c_double), ("mass_residual", C.c_double), ("R", C.c_double),
                ("converged", C.c_int32), ("checks", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class OMTError(RuntimeError):
    def __init__(self, status, where, detail):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


_lib = None

# every function the header declares, with its argument and result types
_SIGS = {
    "omt_params_init": (None, [C.POINTER(Params)]),
    "omt_resolve_params": (C.c_int, [C.POINTER(Params)] + [C.POINTER(C.c_double)] * 4),
    "omt_workspace_bytes": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_size_t)]),
    "omt_create": (C.c_int, [C.POINTER(Params), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    "omt_solve": (C.c_int, [C.c_void_p, C.c_int64, C.c_double, C.c_int32, C.POINTER(Info)]),
    "omt_distance": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(Info)]),
    "omt_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "omt_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "omt_set_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "omt_destroy": (C.c_int, [C.c_void_p]),
    "omt_batch_workspace_bytes": (C.c_int, [C.c_int32, C.POINTER(Params), C.POINTER(C.c_size_t)]),
    "omt_batch_create": (C.c_int, [C.c_int32, C.POINTER(Params), C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                   C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "omt_batch_solve": (C.c_int, [C.c_void_p, C.c_int64, C.c_double, C.c_int32, C.POINTER(Info)]),
    "omt_batch_distance": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "omt_batch_grad": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    "omt_batch_get_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "omt_batch_set_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "omt_batch_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "omt_batch_destroy": (C.c_int, [C.c_void_p]),
    "omt_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                               C.POINTER(C.c_double)]),
    "omt_time_steps": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int64, C.POINTER(C.c_double)]),
    "omt_solve_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double, C.c_int32,
                                   C.POINTER(C.c_double), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "omt_matrix_params_init": (C.c_int, [C.POINTER(MatrixParams)]),
    "omt_matrix_resolve": (C.c_int, [C.POINTER(MatrixParams)] + [C.POINTER(C.c_double)] * 4 +
                           [C.POINTER(C.c_int32)] * 2),
    "omt_matrix_workspace_bytes": (C.c_int, [C.POINTER(MatrixParams), C.POINTER(C.c_size_t)]),
    "omt_matrix_create": (C.c_int, [C.POINTER(MatrixParams), C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                    C.c_void_p, C.POINTER(C.c_void_p)]),
    "omt_matrix_solve": (C.c_int, [C.c_void_p, C.c_int64, C.c_double, C.c_int32, C.POINTER(Info)]),
    "omt_matrix_distance": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(Info)]),
    "omt_matrix_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "omt_matrix_get_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "omt_matrix_time_steps": (C.c_int, [C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)]),
    "omt_matrix_destroy": (C.c_int, [C.c_void_p]),
    "omt_strerror": (C.c_char_p, [C.c_int]),
    "omt_last_error": (C.c_char_p, []),
    "omt_version": (C.c_int32, []),
}


def lib():
    """The loaded ``libomt.so``; raises if the HIP library was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1712_10279_amd/build.py "
                               "(the solver has no other implementation)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status, where, allow=()):
    if status != OK and status not in allow:
        detail = lib().omt_last_error().decode()
        raise OMTError(status, where, detail)
    return status


def _torch():
    import torch
    return torch


def _stream_ptr():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


@dataclass
class Config:
    alpha: float = 1.0
    tau: float = 1.0
    cost: object = None
    unorm: int = U_L12
    wnorm: int = W_L1
    mu: float = 0.0
    nu: float = 0.0
    h: float = 0.0
    compensated: bool = False
    tblock: int = 0
    rows_per_wave: int = 0
    eps: float = 0.0


def make_params(m, n, k, edges, cfg: Config, dtype: int, p: int = 0):
    """(Params, keep-alive arrays) for the C ABI; p > 1: a 3-D grid of p slices."""
    depth = p
    e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    p = Params()
    lib().omt_params_init(C.byref(p))
    p.m, p.n, p.k, p.n_edges = int(m), int(n), int(k), int(e.shape[0])
    p.edges = e.ctypes.data_as(C.POINTER(C.c_int32)) if e.size else C.POINTER(C.c_int32)()
    cost = None
    if cfg.cost is not None:
        cost = np.ascontiguousarray(np.asarray(cfg.cost, dtype=np.float64).reshape(-1))
        p.edge_cost = cost.ctypes.data_as(C.POINTER(C.c_double))
    p.alpha, p.tau, p.mu, p.nu, p.h = float(cfg.alpha), float(cfg.tau), float(cfg.mu), float(cfg.nu), float(cfg.h)
    p.unorm, p.wnorm, p.dtype = int(cfg.unorm), int(cfg.wnorm), int(dtype)
    p.flags = FLAG_COMPENSATED_PHI if cfg.compensated else 0
    p.tblock, p.rows_per_wave = int(cfg.tblock), int(cfg.rows_per_wave)
    p.reg_eps = float(cfg.eps)
    p.p = int(depth)
    return p, (e, cost)


def resolve_params(m, n, k, edges, depth=0, **kw):
    """Host-only: validated (h, mu, nu, lambda_max) of a problem (Sec. 7.2);
    depth > 1: a 3-D grid of that many slices."""
    dtype = F64 if kw.pop("dtype", "f32") in ("f64", F64) else F32
    p, keep = make_params(m, n, k, edges, Config(**kw), dtype, depth)
    out = [C.c_double() for _ in range(4)]
    _check(lib().omt_resolve_params(C.byref(p), *[C.byref(o) for o in out]), "omt_resolve_params")
    return tuple(o.value for o in out)


def workspace_bytes(m, n, k, edges, dtype="f32", depth=0, **kw):
    p, keep = make_params(m, n, k, edges, Config(**kw), F64 if dtype in ("f64", F64) else F32, depth)
    b = C.c_size_t()
    _check(lib().omt_workspace_bytes(C.byref(p), C.byref(b)), "omt_workspace_bytes")
    return b.value


class Solver:
    """One transport problem on the GPU (omt_create ... omt_destroy).  rho0,
    rho1: (m, n, k), or (m, n, p, k) for a 3-D grid of p slices."""

    def __init__(self, rho0, rho1, edges=None, **kw):
        torch = _torch()
        if rho0.dim() not in (3, 4) or rho0.shape != rho1.shape:
            raise ValueError("rho0 and rho1 must both be (m, n, k) or (m, n, p, k)")
        if not (rho0.is_cuda and rho1.is_cuda):
            raise ValueError("rho0 and rho1 must be on the GPU")
        if rho0.dtype not in (torch.float32, torch.float64) or rho1.dtype != rho0.dtype:
            raise ValueError("rho0 and rho1 must share dtype float32 or float64")
        self.dtype = rho0.dtype
        if rho0.dim() == 4:
            self.m, self.n, self.p, self.k = (int(s) for s in rho0.shape)
        else:
            self.m, self.n, self.k = (int(s) for s in rho0.shape)
            self.p = 0
        self.grid = (self.m, self.n, self.p) if self.p else (self.m, self.n)
        self.edges = np.zeros((0, 2), np.int32) if edges is None else np.asarray(edges, np.int32).reshape(-1, 2)
        self.l = int(self.edges.shape[0])
        self.cfg = Config(**kw)
        dt = F64 if self.dtype == torch.float64 else F32
        self._p, self._keep = make_params(self.m, self.n, self.k, self.edges, self.cfg, dt, self.p)
        nbytes = C.c_size_t()
        _check(lib().omt_workspace_bytes(C.byref(self._p), C.byref(nbytes)), "omt_workspace_bytes")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=rho0.device)
        self.device = rho0.device
        r0 = rho0.contiguous()
        r1 = rho1.contiguous()
        h = C.c_void_p()
        _check(lib().omt_create(C.byref(self._p), _ptr(r0), _ptr(r1), _ptr(self.workspace), nbytes.value,
                                _stream_ptr(), C.byref(h)), "omt_create")
        self._h = h
        self.info = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.omt_destroy(h)
            self._h = None

    def solve(self, max_iters, tol=0.0, check_every=64, allow_notconv=True):
        info = Info()
        allow = (ENOTCONV,) if allow_notconv else ()
        _check(lib().omt_solve(self._h, int(max_iters), float(tol), int(check_every), C.byref(info)),
               "omt_solve", allow)
        self.info = info.as_dict()
        return self.info

    def distance(self):
        v = C.c_double()
        info = Info()
        _check(lib().omt_distance(self._h, C.byref(v), C.byref(info)), "omt_distance")
        return v.value, info.as_dict()

    def grad(self):
        torch = _torch()
        d0 = torch.empty(self.grid + (self.k,), dtype=self.dtype, device=self.device)
        d1 = torch.empty_like(d0)
        _check(lib().omt_grad(self._h, _ptr(d0), _ptr(d1)), "omt_grad")
        return d0, d1

    def get_state(self):
        """phi (grid x k), u (grid x k x 2, or x 3 on a 3-D grid), w (grid x l)."""
        torch = _torch()
        phi = torch.empty(self.grid + (self.k,), dtype=self.dtype, device=self.device)
        u = torch.empty(self.grid + (self.k, 3 if self.p else 2), dtype=self.dtype, device=self.device)
        w = torch.zeros(self.grid + (max(self.l, 1),), dtype=self.dtype, device=self.device)
        _check(lib().omt_get_state(self._h, _ptr(phi), _ptr(u), _ptr(w) if self.l else C.c_void_p(0)),
               "omt_get_state")
        return {"phi": phi, "u": u, "w": w[..., : self.l]}

    def set_state(self, phi=None, u=None, w=None):
        """Load phi, u, w (shapes of get_state, the solver's dtype; None keeps
        that field) as the current iterate."""
        keep = [t.contiguous() if t is not None else None for t in (phi, u, w)]
        _check(lib().omt_set_state(self._h, *[_ptr(t) for t in keep]), "omt_set_state")

    def time_steps(self, T, rows_per_wave, n):
        us = C.c_double()
        _check(lib().omt_time_steps(self._h, int(T), int(rows_per_wave), int(n), C.byref(us)), "omt_time_steps")
        return us.value

    def autotune(self, iters_per_trial=64):
        t, r, us = C.c_int32(), C.c_int32(), C.c_double()
        _check(lib().omt_autotune(self._h, int(iters_per_trial), C.byref(t), C.byref(r), C.byref(us)),
               "omt_autotune")
        return t.value, r.value, us.value


def distance(rho0, rho1, edges=None, max_iters=10000, tol=0.0, check_every=64, **kw):
    """V(rho0, rho1) of the discrete problem (App. A) after the solve."""
    s = Solver(rho0, rho1, edges, **kw)
    s.solve(max_iters, tol, check_every)
    return s.distance()[0]


def solve_static(rho0, rho1, edges=None, max_iters=10000, tol=0.0, check_every=64, d_rho0=None, d_rho1=None,
                 allow_notconv=True, **kw):
    """One whole solve through omt_solve_static (device workspace inside the
    library; the call allocates nothing).  d_rho0 / d_rho1: optional output
    tensors (m, n, k) of the input dtype on the same device, filled with
    Phi and -Phi.  Returns (V, info)."""
    torch = _torch()
    if rho0.dim() != 3 or rho0.shape != rho1.shape or rho0.dtype != rho1.dtype:
        raise ValueError("rho0 and rho1 must both be (m, n, k) of one dtype")
    if not (rho0.is_cuda and rho1.is_cuda):
        raise ValueError("rho0 and rho1 must be on the GPU")
    for t in (d_rho0, d_rho1):
        if t is not None and (t.shape != rho0.shape or t.dtype != rho0.dtype or not t.is_contiguous()):
            raise ValueError("outputs must be contiguous tensors shaped and typed like rho0")
    m, n, k = (int(x) for x in rho0.shape)
    e = np.zeros((0, 2), np.int32) if edges is None else np.asarray(edges, np.int32).reshape(-1, 2)
    dt = F64 if rho0.dtype == torch.float64 else F32
    p, keep = make_params(m, n, k, e, Config(**kw), dt)
    r0, r1 = rho0.contiguous(), rho1.contiguous()
    V = C.c_double()
    info = Info()
    allow = (ENOTCONV,) if allow_notconv else ()
    _check(lib().omt_solve_static(C.byref(p), _ptr(r0), _ptr(r1), int(max_iters), float(tol), int(check_every),
                                  C.byref(V), _ptr(d_rho0), _ptr(d_rho1), C.byref(info), _stream_ptr()),
           "omt_solve_static", allow)
    return V.value, info.as_dict()


# ----------------------------------------------------------------- autograd

def _autograd_function():
    torch = _torch()

    class OMTDistance(torch.autograd.Function):
        """V(rho0, rho1) as a differentiable loss.

        Forward: solve on the GPU (to ``tol`` or for ``max_iters``) and return
        the transport cost V (the discrete primal objective, App. A).  Backward:
        dV/drho0 = Phi and dV/drho1 = -Phi, with Phi = -phi minus its mean per
        mass class (dual problem, Sec. 3.2); no second solve is needed.
        """

        @staticmethod
        def forward(ctx, rho0, rho1, edges, max_iters, tol, check_every, kw, on_notconv):
            s = Solver(rho0.detach(), rho1.detach(), edges, **kw)
            _notconv([s.solve(max_iters, tol, check_every)], tol, on_notconv)
            V, info = s.distance()
            d0, _ = s.grad()
            ctx.save_for_backward(d0)
            ctx.info = info
            return torch.tensor(V, dtype=rho0.dtype, device=rho0.device)

        @staticmethod
        def backward(ctx, g):
            (d0,) = ctx.saved_tensors
            return g * d0, -g * d0, None, None, None, None, None, None

    class OMTDistanceBatch(torch.autograd.Function):
        """The same for a batch (B, m, n, k) of pairs solved together by the
        batched solver (one launch per iteration for all unfinished pairs);
        returns the (B,) distances."""

        @staticmethod
        def forward(ctx, rho0, rho1, edges, max_iters, tol, check_every, kw, on_notconv):
            probs = [dict(rho0=rho0[b].detach(), rho1=rho1[b].detach(), edges=edges, **kw)
                     for b in range(rho0.shape[0])]
            bs = BatchSolver(probs)
            ctx.infos = bs.solve(max_iters, tol, check_every)
            _notconv(ctx.infos, tol, on_notconv)
            V = bs.distance()
            d0, _ = bs.grad()
            d0 = torch.stack(d0)
            ctx.save_for_backward(d0)
            return torch.tensor(V, dtype=rho0.dtype, device=rho0.device)

        @staticmethod
        def backward(ctx, g):
            (d0,) = ctx.saved_tensors
            gb = g.reshape(-1, 1, 1, 1)
            return gb * d0, -gb * d0, None, None, None, None, None, None

    return OMTDistance, OMTDistanceBatch


_OMT_FN = None


class NotConvergedWarning(UserWarning):
    """A loss value whose solve stopped at max_iters above its tolerance."""


def _notconv(infos, tol, on_notconv):
    if tol <= 0 or on_notconv == "ignore":
        return
    bad = [(b, i["iters"], i["residual"]) for b, i in enumerate(infos) if not i["converged"]]
    if not bad:
        return
    text = (f"{len(bad)} of {len(infos)} solves stopped above tol {tol:g} (pair, iterations, R^k): "
            + ", ".join(f"({b}, {it}, {r:.3g})" for b, it, r in bad[:8]))
    if on_notconv == "raise":
        raise OMTError(ENOTCONV, "omt_loss", text)
    warnings.warn(text, NotConvergedWarning, stacklevel=4)


def omt_loss(rho0, rho1, edges=None, max_iters=100000, tol=1e-6, check_every=64, on_notconv="warn", **kw):
    """Differentiable V(rho0, rho1) (see ``OMTDistance``); rho0 / rho1 may be
    (m, n, k) or a batch (B, m, n, k), which returns a (B,) tensor.

    A solve that reaches max_iters above ``tol`` still gives its value and
    gradient; ``on_notconv`` says what else happens: "warn" (a
    NotConvergedWarning naming the pairs), "raise" (OMTError ENOTCONV) or
    "ignore"."""
    global _OMT_FN
    if on_notconv not in ("warn", "raise", "ignore"):
        raise ValueError(f"on_notconv must be warn, raise or ignore, not {on_notconv!r}")
    if _OMT_FN is None:
        _OMT_FN = _autograd_function()
    single, batched = _OMT_FN
    if rho0.dim() == 4:
        torch = _torch()
        try:
            return batched.apply(rho0, rho1, edges, max_iters, tol, check_every, kw, on_notconv)
        except OMTError as e:
            if e.status != EUNSUPPORTED:
                raise
        # problems the batched kernel does not compile: one solve per pair
        return torch.stack([single.apply(rho0[b], rho1[b], edges, max_iters, tol, check_every, kw, on_notconv)
                            for b in range(rho0.shape[0])])
    return single.apply(rho0, rho1, edges, max_iters, tol, check_every, kw, on_notconv)


class BatchSolver:
    """Many problems solved together by the persistent batched kernel
    (omt_batch_create ... omt_batch_destroy).  ``problems`` is a list of
    dicts with keys rho0, rho1 (GPU tensors, all float32 or all float64),
    edges and any Config field (alpha, tau, compensated, ...)."""

    def __init__(self, problems):
        torch = _torch()
        self.B = len(problems)
        ps = (Params * self.B)()
        self._keep = []
        self.shapes = []
        r0 = (C.c_void_p * self.B)()
        r1 = (C.c_void_p * self.B)()
        dev = None
        self.dtype = problems[0]["rho0"].dtype if problems else torch.float32
        for b, pr in enumerate(problems):
            a0, a1 = pr["rho0"].contiguous(), pr["rho1"].contiguous()
            if a0.dtype not in (torch.float32, torch.float64) or not a0.is_cuda:
                raise ValueError("batched problems must be float32 or float64 GPU tensors")
            if a0.dtype != self.dtype or a1.dtype != self.dtype:
                raise ValueError("every problem of a batch must have the same dtype")
            dev = a0.device
            m, n, k = (int(x) for x in a0.shape)
            edges = np.zeros((0, 2), np.int32) if pr.get("edges") is None else pr["edges"]
            kw = {key: v for key, v in pr.items() if key not in ("rho0", "rho1", "edges")}
            p, keep = make_params(m, n, k, edges, Config(**kw), F64 if self.dtype == torch.float64 else F32)
            ps[b] = p
            self._keep += [keep, a0, a1]
            r0[b], r1[b] = a0.data_ptr(), a1.data_ptr()
            self.shapes.append((m, n, k, int(np.asarray(edges).reshape(-1, 2).shape[0])))
        nbytes = C.c_size_t()
        _check(lib().omt_batch_workspace_bytes(self.B, ps, C.byref(nbytes)), "omt_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        self.device = dev
        h = C.c_void_p()
        _check(lib().omt_batch_create(self.B, ps, r0, r1, _ptr(self.workspace), nbytes.value, _stream_ptr(),
                                      C.byref(h)), "omt_batch_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.omt_batch_destroy(h)
            self._h = None

    def solve(self, max_iters, tol=0.0, check_every=64, allow_notconv=True):
        infos = (Info * self.B)()
        allow = (ENOTCONV,) if allow_notconv else ()
        _check(lib().omt_batch_solve(self._h, int(max_iters), float(tol), int(check_every), infos),
               "omt_batch_solve", allow)
        return [i.as_dict() for i in infos]

    def distance(self):
        V = (C.c_double * self.B)()
        _check(lib().omt_batch_distance(self._h, V), "omt_batch_distance")
        return list(V)

    def grad(self):
        torch = _torch()
        d0 = [torch.empty(s[:3], dtype=self.dtype, device=self.device) for s in self.shapes]
        d1 = [torch.empty_like(x) for x in d0]
        p0 = (C.c_void_p * self.B)(*[x.data_ptr() for x in d0])
        p1 = (C.c_void_p * self.B)(*[x.data_ptr() for x in d1])
        _check(lib().omt_batch_grad(self._h, p0, p1), "omt_batch_grad")
        return d0, d1

    def get_state(self, b):
        torch = _torch()
        m, n, k, l = self.shapes[b]
        phi = torch.empty((m, n, k), dtype=self.dtype, device=self.device)
        u = torch.empty((m, n, k, 2), dtype=self.dtype, device=self.device)
        w = torch.zeros((m, n, max(l, 1)), dtype=self.dtype, device=self.device)
        _check(lib().omt_batch_get_state(self._h, int(b), _ptr(phi), _ptr(u), _ptr(w) if l else C.c_void_p(0)),
               "omt_batch_get_state")
        return {"phi": phi, "u": u, "w": w[:, :, :l]}

    def autotune(self, launches_per_trial=32):
        """Rows per strip for every shape class of the batch (see
        omt_batch_autotune); returns (rows per problem, us per batched
        iteration of all problems)."""
        rows = (C.c_int32 * self.B)()
        us = C.c_double()
        _check(lib().omt_batch_autotune(self._h, int(launches_per_trial), rows, C.byref(us)), "omt_batch_autotune")
        return list(rows), us.value

    def set_state(self, b, phi=None, u=None, w=None):
        """Warm start of problem b (see Solver.set_state)."""
        keep = [t.contiguous() if t is not None else None for t in (phi, u, w)]
        _check(lib().omt_batch_set_state(self._h, int(b), *[_ptr(t) for t in keep]), "omt_batch_set_state")


# ----------------------------------------------------------------- matrix OMT

def make_matrix_params(m, n, L, real, alpha=1.0, tau=1.0, unorm=M_FRO, wnorm=M_L1, mu=0.0, nu=0.0, h=0.0,
                       compensated=False, rows_per_wave=0, tblock=0, dtype=F32):
    """(MatrixParams, keep-alive array) for the matrix C ABI; L is an
    (l, k, k) real or complex array of Hermitian matrices."""
    Lc = np.asarray(L)
    if Lc.ndim == 2:
        Lc = Lc[None]
    Lc = np.ascontiguousarray(Lc.astype(np.complex128))
    p = MatrixParams()
    lib().omt_matrix_params_init(C.byref(p))
    p.m, p.n, p.k, p.n_L = int(m), int(n), int(Lc.shape[1]), int(Lc.shape[0])
    p.L = Lc.ctypes.data_as(C.POINTER(C.c_double))
    p.real = 1 if real else 0
    p.alpha, p.tau, p.mu, p.nu, p.h = float(alpha), float(tau), float(mu), float(nu), float(h)
    p.unorm, p.wnorm, p.dtype = int(unorm), int(wnorm), int(dtype)
    p.flags = FLAG_COMPENSATED_PHI if compensated else 0
    p.rows_per_wave = int(rows_per_wave)
    p.tblock = int(tblock)
    return p, Lc


def matrix_resolve(m, n, L, real, **kw):
    """(h, mu, nu, lambda_max(-Delta_L), coordinates of Phi, coordinates of W)."""
    p, keep = make_matrix_params(m, n, L, real, **kw)
    h, mu, nu, lm = C.c_double(), C.c_double(), C.c_double(), C.c_double()
    K, KW = C.c_int32(), C.c_int32()
    _check(lib().omt_matrix_resolve(C.byref(p), C.byref(h), C.byref(mu), C.byref(nu), C.byref(lm), C.byref(K),
                                    C.byref(KW)), "omt_matrix_resolve")
    return h.value, mu.value, nu.value, lm.value, K.value, KW.value


class MatrixSolver:
    """One matrix-OMT problem (omt_matrix_create ... omt_matrix_destroy).
    Lambda0 / Lambda1: GPU tensors (m, n, k, k), complex64/complex128, or
    float32/float64 in the real mode (real symmetric data and L)."""

    def __init__(self, lam0, lam1, L, **kw):
        torch = _torch()
        a0, a1 = lam0.contiguous(), lam1.contiguous()
        if not a0.is_cuda or a0.dtype != a1.dtype or a0.shape != a1.shape:
            raise ValueError("Lambda0 / Lambda1 must be GPU tensors of one dtype and shape")
        real = not a0.is_complex()
        if a0.dtype in (torch.float64, torch.complex128):
            dtype = F64
        elif a0.dtype in (torch.float32, torch.complex64):
            dtype = F32
        else:
            raise ValueError("unsupported dtype")
        m, n, k = (int(x) for x in a0.shape[:3])
        self.m, self.n, self.k, self.real = m, n, k, real
        self.tdtype = a0.dtype
        self.params, self._keep = make_matrix_params(m, n, L, real, dtype=dtype, **kw)
        self.l = int(self.params.n_L)
        nbytes = C.c_size_t()
        _check(lib().omt_matrix_workspace_bytes(C.byref(self.params), C.byref(nbytes)), "omt_matrix_workspace_bytes")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=a0.device)
        self.device = a0.device
        self._in = (a0, a1)
        h = C.c_void_p()
        _check(lib().omt_matrix_create(C.byref(self.params), _ptr(a0), _ptr(a1), _ptr(self.workspace), nbytes.value,
                                       _stream_ptr(), C.byref(h)), "omt_matrix_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.omt_matrix_destroy(h)
            self._h = None

    def solve(self, max_iters, tol=0.0, check_every=64, allow_notconv=True):
        info = Info()
        allow = (ENOTCONV,) if allow_notconv else ()
        _check(lib().omt_matrix_solve(self._h, int(max_iters), float(tol), int(check_every), C.byref(info)),
               "omt_matrix_solve", allow)
        return info.as_dict()

    def distance(self):
        M, info = C.c_double(), Info()
        _check(lib().omt_matrix_distance(self._h, C.byref(M), C.byref(info)), "omt_matrix_distance")
        return M.value, info.as_dict()

    def _mat(self, count=None):
        torch = _torch()
        shape = (self.m, self.n) + ((count,) if count else ()) + (self.k, self.k)
        return torch.empty(shape, dtype=self.tdtype, device=self.device)

    def grad(self):
        d0, d1 = self._mat(), self._mat()
        _check(lib().omt_matrix_grad(self._h, _ptr(d0), _ptr(d1)), "omt_matrix_grad")
        return d0, d1

    def get_state(self):
        phi, ux, uy, w = self._mat(), self._mat(), self._mat(), self._mat(self.l)
        _check(lib().omt_matrix_get_state(self._h, _ptr(phi), _ptr(ux), _ptr(uy), _ptr(w)), "omt_matrix_get_state")
        return {"phi": phi, "ux": ux, "uy": uy, "w": w}

    def time_steps(self, rows_per_wave, n):
        us = C.c_double()
        _check(lib().omt_matrix_time_steps(self._h, int(rows_per_wave), int(n), C.byref(us)), "omt_matrix_time_steps")
        return us.value
