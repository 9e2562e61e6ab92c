"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times, on sampled pixels the oracle can compute one by one.

After N iterations a pixel depends only on the pixels within N of it, so the
oracle runs on the crop of radius N+2 around each sample (with the full
problem's f, h, mu and nu) and must agree with the GPU there.  FP32 samples
are compared at the FP32 tolerances (1e-4 relative, 1e-3 absolute on the
potential) scaled to the iterate size.
"""
import numpy as np
import pytest

import oracle as O
from gpu_util import cast_inputs, cone_oracle, cuda, gpu_state_np, note, to_dev
from paper_1712_10279_amd import inputs as I

pytestmark = pytest.mark.gpu


def _samples(m, n, rng, count):
    fixed = [(0, 0), (0, n - 1), (m - 1, 0), (m - 1, n - 1), (m // 2, 63), (m // 2, 64), (7, n // 2),
             (m - 2, n - 65)]
    rand = [(int(rng.integers(m)), int(rng.integers(n))) for _ in range(count)]
    return fixed + rand


def _check_cone(torch, d, iters, tblock=0, rows=0, nsamp=8, tol_rel=2e-5, tune=False):
    from paper_1712_10279_amd import omt
    r0, r1 = cast_inputs(d["rho0"], d["rho1"], "f32")
    m, n, k = r0.shape
    s = omt.Solver(to_dev(torch, d["rho0"], torch.float32), to_dev(torch, d["rho1"], torch.float32), d["edges"],
                   alpha=d["alpha"], tau=d["tau"], tblock=tblock, rows_per_wave=rows)
    if tune:
        T, R, us = s.autotune()
        note(f"autotuned shape: T {T}, {R} rows per wave, {us:.2f} us per iteration")
    s.solve(iters, 0.0, 64)
    g = gpu_state_np(s)
    p = O.Problem(m, n, k, edges=d["edges"], alpha=d["alpha"], tau=d["tau"])
    f, _ = O.prepare_f(r0, r1, p.edges)
    rng = np.random.default_rng(7)
    worst = 0.0
    for (i, j) in _samples(m, n, rng, nsamp):
        o = cone_oracle(f, p, (i, j), iters)
        scale_phi = max(np.abs(o["phi"]).max(), 1e-12)
        scale_u = max(np.abs(o["ux"]).max(), np.abs(o["uy"]).max(), 1e-12)
        e_phi = np.abs(g["phi"][i, j] - o["phi"]).max() / scale_phi
        e_u = max(np.abs(g["u"][i, j, :, 0] - o["ux"]).max(), np.abs(g["u"][i, j, :, 1] - o["uy"]).max()) / scale_u
        e_w = 0.0
        if p.l:
            e_w = np.abs(g["w"][i, j] - o["w"]).max() / max(np.abs(o["w"]).max(), 1e-12)
        # a zero oracle u (or w) leaves the floor 1e-12 as the scale, so the
        # kernel's must be zero there too
        worst = max(worst, e_phi, e_u, e_w)
    note(f"worst sampled relative error {worst:.2e}")
    assert worst <= tol_rel


def test_large_grid_sampled_cones():
    """1024x1024, k=8 path, FP32, in the launch shape the benchmark takes
    from the autotuner."""
    torch = cuda()
    d = I.path8_1024()
    note("case: 1024x1024 k8 path, 24 iterations, autotuned shape, sampled cones")
    _check_cone(torch, d, 24, tune=True)


@pytest.mark.parametrize("tblock,rows", [(1, 0), (2, 10)])
def test_large_grid_sampled_cones_fixed_shapes(tblock, rows):
    """1024x1024, k=8 path, FP32: single-iteration launches with the default
    rows, and two iterations per launch with 10 rows per wave (the shape the
    autotuner picks on MI355X)."""
    torch = cuda()
    d = I.path8_1024()
    note(f"case: 1024x1024 k8 path, 24 iterations, T={tblock} rows={rows}, sampled cones")
    _check_cone(torch, d, 24, tblock=tblock, rows=rows)


def test_rgb_grid_sampled_cones_blocked():
    """256x256, k=3 triangle, FP32, pipelined launches (T = 4)."""
    torch = cuda()
    d = I.rgb_256(1.0)
    note("case: 256x256 k3 triangle, 32 iterations, T=4, sampled cones")
    _check_cone(torch, d, 32, tblock=4)


def test_large_grid_invariants():
    """Properties that hold at any size: the mean of phi is conserved, R^k
    decreases, the residual matches its definition from R and f."""
    torch = cuda()
    from paper_1712_10279_amd import omt
    d = I.path8_1024()
    s = omt.Solver(to_dev(torch, d["rho0"], torch.float32), to_dev(torch, d["rho1"], torch.float32), d["edges"],
                   alpha=d["alpha"], tau=d["tau"])
    res = []
    for _ in range(5):
        info = s.solve(640, 0.0, 64)
        res.append(info["R"])
    st = s.get_state()
    phi_mean = st["phi"].double().mean().item()
    note(f"R history {res}, mean phi {phi_mean:.3e}")
    assert abs(phi_mean) < 1e-6 * st["phi"].double().abs().max().item() + 1e-12
    assert all(b <= a * (1 + 1e-6) for a, b in zip(res, res[1:]))
