"""Helpers shared by the GPU tests: device fixture, oracle runs on the same
seeded inputs, comparisons, and the sampled-cone check for full-size grids."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle as O


def cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(torch, a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def cast_inputs(rho0, rho1, dtype_name):
    """The values both sides see: the inputs rounded to the path's dtype."""
    if dtype_name == "f32":
        return rho0.astype(np.float32).astype(np.float64), rho1.astype(np.float32).astype(np.float64)
    return rho0, rho1


def oracle_run(rho0, rho1, edges, iters, tol=0.0, check_every=64, **kw):
    r = O.solve_pair(rho0, rho1, edges, max_iters=iters, tol=tol, check_every=check_every, **kw)
    return r


def gpu_state_np(s):
    st = s.get_state()
    out = {"phi": st["phi"].double().cpu().numpy(), "u": st["u"].double().cpu().numpy(),
           "w": st["w"].double().cpu().numpy()}
    return out


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cone_oracle(f_full, p_full, pix, iters, state=None):
    """Oracle values at pixel ``pix`` after ``iters`` iterations from zeros
    (or from ``state``: full-grid arrays phi (m, n, k), ux, uy (m, n, k) and
    w (m, n, l)), computed on the crop of radius iters+2 around it:
    information moves at most one pixel per iteration, so the crop's
    artificial border cannot reach the centre (where the crop meets the real
    border, the real border is inside the crop)."""
    m, n, k = f_full.shape
    i, j = pix
    rad = iters + 2
    i0, i1 = max(0, i - rad), min(m, i + rad + 1)
    j0, j1 = max(0, j - rad), min(n, j + rad + 1)
    p = O.Problem(i1 - i0, j1 - j0, k, edges=p_full.edges, cost=p_full.cost, alpha=p_full.alpha, tau=p_full.tau,
                  mu=p_full.mu, nu=p_full.nu, h=p_full.h, unorm=p_full.unorm, wnorm=p_full.wnorm, eps=p_full.eps)
    st = None
    if state is not None:
        st = {key: np.array(state[key][i0:i1, j0:j1], dtype=np.float64) for key in ("phi", "ux", "uy", "w")}
        # ghost components of the real border (App. A) are zero on both sides
        if i1 == m:
            st["ux"][-1] = 0.0
        if j1 == n:
            st["uy"][:, -1] = 0.0
    r = O.solve(p, f_full[i0:i1, j0:j1], iters, 0.0, 1 << 30, state=st)
    s = r["state"]
    ci, cj = i - i0, j - j0
    return {"phi": s["phi"][ci, cj], "ux": s["ux"][ci, cj], "uy": s["uy"][ci, cj],
            "w": s["w"][ci, cj] if p.l else np.zeros(0)}


def active_fraction(ux, uy, w):
    """Fractions of pixels whose flux (any channel, either direction) and
    whose transfer (any edge) are non-zero; arrays (..., k) and (..., l)."""
    ux, uy, w = np.asarray(ux), np.asarray(uy), np.asarray(w)
    ua = float(((ux != 0) | (uy != 0)).reshape(-1, ux.shape[-1]).any(axis=1).mean())
    wa = float((w != 0).reshape(-1, w.shape[-1]).any(axis=1).mean()) if w.size else 0.0
    return ua, wa
