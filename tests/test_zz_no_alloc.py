"""omt_solve_static (the entry point for callers that cannot allocate: its
device workspace is a fixed array inside the library) against the handle
path omt_create + omt_solve + omt_distance + omt_grad, through the C ABI.
Same kernels, so the results must agree bit for bit; two calls in a row,
the second on a smaller problem, show that nothing of the first call's state
survives in the shared array."""
import numpy as np
import pytest

from gpu_util import cuda, note, to_dev
from paper_1712_10279_amd import inputs as I

pytestmark = pytest.mark.gpu


def _handle(torch, r0, r1, edges, iters, tol, **kw):
    from paper_1712_10279_amd import omt
    s = omt.Solver(r0, r1, edges, **kw)
    info = s.solve(iters, tol, 64)
    V, _ = s.distance()
    d0, d1 = s.grad()
    return V, info, d0, d1


def _static(torch, r0, r1, edges, iters, tol, **kw):
    from paper_1712_10279_amd import omt
    d0, d1 = torch.empty_like(r0), torch.empty_like(r0)
    V, info = omt.solve_static(r0, r1, edges, iters, tol, 64, d_rho0=d0, d_rho1=d1, **kw)
    return V, info, d0, d1


CASES = [  # (seed, m, n, k, edges, dtype, iters, tol, kw)
    (90, 96, 130, 3, I.TRIANGLE, "f32", 640, 0.0, dict(alpha=0.3, tau=3.0)),
    (91, 40, 70, 3, I.TRIANGLE, "f32", 320, 0.0, dict(alpha=0.3, tau=3.0)),
    (92, 64, 80, 8, I.path_edges(8), "f32", 500, 0.0, dict(alpha=0.1, tau=3.0, compensated=True)),
    (93, 24, 24, 3, I.TRIANGLE, "f64", 200000, 1e-4, {}),
    (94, 150, 40, 1, None, "f64", 300, 0.0, dict(tau=3.0)),
]


def test_static_matches_handle_path_on_consecutive_calls():
    torch = cuda()
    for (seed, m, n, k, edges, dt, iters, tol, kw) in CASES:
        note(f"case: static vs handle {m}x{n} k{k} {dt} {iters} it tol {tol}")
        r0, r1 = I.random_pair(seed, m, n, k)
        tdt = torch.float64 if dt == "f64" else torch.float32
        a, b = to_dev(torch, r0, tdt), to_dev(torch, r1, tdt)
        Vh, ih, h0, h1 = _handle(torch, a, b, edges, iters, tol, **kw)
        Vs, is_, s0, s1 = _static(torch, a, b, edges, iters, tol, **kw)
        note(f"  V handle {Vh!r} static {Vs!r}; iters {ih['iters']} / {is_['iters']}")
        assert Vs == Vh
        assert is_["iters"] == ih["iters"] and is_["converged"] == ih["converged"]
        assert is_["residual"] == ih["residual"] and is_["primal"] == ih["primal"]
        assert torch.equal(s0, h0) and torch.equal(s1, h1)
        if tol > 0:
            assert is_["converged"] == 1


def test_static_second_call_smaller_after_larger():
    """The required pair: a large call, then a smaller one, each checked
    against its own handle-path solve."""
    torch = cuda()
    out = []
    for (seed, m, n) in ((95, 200, 300), (96, 33, 65)):
        r0, r1 = I.random_pair(seed, m, n, 3)
        a, b = to_dev(torch, r0, torch.float32), to_dev(torch, r1, torch.float32)
        kw = dict(alpha=0.5, tau=3.0)
        note(f"case: static {m}x{n} after the previous call")
        Vs, is_, s0, _ = _static(torch, a, b, I.TRIANGLE, 384, 0.0, **kw)
        Vh, ih, h0, _ = _handle(torch, a, b, I.TRIANGLE, 384, 0.0, **kw)
        assert Vs == Vh and is_["residual"] == ih["residual"]
        assert torch.equal(s0, h0)
        out.append(Vs)
    assert out[0] != out[1]


def test_static_rejects_problems_beyond_the_workspace():
    torch = cuda()
    from paper_1712_10279_amd import omt
    r = torch.zeros((1024, 1024, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(omt.OMTError) as e:
        omt.solve_static(r, r, I.TRIANGLE, 10)
    assert e.value.status == omt.ENOMEM
    # a call after the rejected one still works
    r0, r1 = I.random_pair(97, 20, 30, 3)
    a, b = to_dev(torch, r0, torch.float64), to_dev(torch, r1, torch.float64)
    Vs, _, _, _ = _static(torch, a, b, I.TRIANGLE, 100, 0.0)
    Vh, _, _, _ = _handle(torch, a, b, I.TRIANGLE, 100, 0.0)
    assert Vs == Vh
