"""Parity of the 3-D grid kernels (the method of Sec. 7.2 on m x n x p grids,
App. A's discretisation along each axis; 3-D is the paper's future work,
Sec. 8.2) with the FP64 3-D oracle, through the C ABI.

FP64 states match element by element; FP32 runs match V to 1e-4 relative
and Phi to 1e-3; every launch shape (slices per wave) gives the same bits;
the full-size workload is checked on sampled cones from an active state.
Each case asserts on the oracle's side that the shrinks are active."""
import numpy as np
import pytest

import oracle.grid3 as G3
from gpu_util import active_fraction, cast_inputs, cuda, note, to_dev
from paper_1712_10279_amd import inputs as I

pytestmark = pytest.mark.gpu

MIN_ACTIVE = 0.2


def _solver(torch, r0, r1, edges, dtype, **kw):
    from paper_1712_10279_amd import omt
    tdt = torch.float64 if dtype == "f64" else torch.float32
    return omt.Solver(to_dev(torch, r0, tdt), to_dev(torch, r1, tdt), edges, **kw)


def _active(st, what, need_w=True):
    ux, uy, uz, w = st["ux"], st["uy"], st["uz"], st["w"]
    ua = float(((ux != 0) | (uy != 0) | (uz != 0)).reshape(-1, ux.shape[-1]).any(axis=1).mean())
    _, wa = active_fraction(ux, uy, w)
    note(f"{what}: oracle active fraction u {ua:.3f} w {wa:.3f}")
    assert ua >= MIN_ACTIVE
    if need_w:
        assert wa >= MIN_ACTIVE


def _gpu_state(s):
    st = s.get_state()
    u = st["u"].double().cpu().numpy()
    return {"phi": st["phi"].double().cpu().numpy(), "ux": u[..., 0], "uy": u[..., 1], "uz": u[..., 2],
            "w": st["w"].double().cpu().numpy()}


def _cmp(g, o, tol, what):
    errs = {}
    for key in ("phi", "ux", "uy", "uz", "w"):
        b = o[key]
        if b.size == 0:
            continue
        scale = np.abs(b).max()
        errs[key] = np.abs(g[key] - b).max() / scale if scale > 0 else np.abs(g[key]).max()
    note(f"{what}: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    for key, v in errs.items():
        assert v <= tol, (what, key, v)


CASES = [  # m, n, p, k, edges, alpha, tau, iters
    (13, 70, 9, 3, I.TRIANGLE, 0.05, 1.0, 600),    # ragged rows and columns, two strips
    (8, 130, 5, 2, [(0, 1)], 0.05, 3.0, 600),      # three strips
    (17, 64, 3, 1, np.zeros((0, 2)), 1.0, 1.0, 400),
    (6, 40, 40, 3, I.path_edges(3), 0.05, 1.0, 400),  # many slices: several z chunks
    (2, 3, 2, 3, I.TRIANGLE, 0.3, 1.0, 100),       # smallest
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fp64_matches_3d_oracle_elementwise(case):
    torch = cuda()
    m, n, p, k, edges, alpha, tau, iters = CASES[case]
    r0, r1 = I.random_volume_pair(50, m, n, p, k)
    note(f"case: 3-D fp64 {m}x{n}x{p} k{k} l{len(edges)} {iters} it")
    r = G3.solve_pair(r0, r1, edges, alpha=alpha, tau=tau, max_iters=iters, check_every=64)
    if m > 2:
        _active(r["state"], f"{m}x{n}x{p}", need_w=len(edges) > 0)
    s = _solver(torch, r0, r1, edges, "f64", alpha=alpha, tau=tau)
    info = s.solve(iters, 0.0, 64)
    _cmp(_gpu_state(s), r["state"], 1e-10, f"{m}x{n}x{p}")
    V, dinfo = s.distance()
    assert abs(V - r["primal"]) <= 1e-10 * r["primal"]
    assert abs(info["residual"] - r["residual"]) <= 1e-8 * r["residual"]
    assert abs(dinfo["mass_residual"] - r["mass_residual"]) <= 1e-8 * r["mass_residual"]
    Phi = s.grad()[0].cpu().numpy()
    assert np.abs(Phi - r["Phi"]).max() <= 1e-9 * np.abs(r["Phi"]).max()


@pytest.mark.parametrize("unorm,wnorm", [(0, 1), (1, 0), (2, 1)])
@pytest.mark.parametrize("eps", [0.0, 1.5])
def test_fp64_norms_and_regularisation(unorm, wnorm, eps):
    torch = cuda()
    m, n, p = 11, 66, 7
    r0, r1 = I.random_volume_pair(51, m, n, p, 3)
    kw = dict(alpha=0.05, tau=1.0, unorm=unorm, wnorm=wnorm, eps=eps)
    note(f"case: 3-D fp64 norms u{unorm} w{wnorm} eps {eps}")
    r = G3.solve_pair(r0, r1, I.TRIANGLE, max_iters=500, **kw)
    _active(r["state"], f"norms {unorm}{wnorm} eps {eps}")
    s = _solver(torch, r0, r1, I.TRIANGLE, "f64", **kw)
    info = s.solve(500, 0.0, 64)
    _cmp(_gpu_state(s), r["state"], 1e-10, f"norms {unorm}{wnorm} eps {eps}")
    assert abs(info["primal"] - r["primal"]) <= 1e-10 * r["primal"]


def test_fp64_stops_with_the_oracle():
    torch = cuda()
    r0, r1 = I.random_volume_pair(52, 10, 12, 9, 3)
    note("case: 3-D fp64 to tol 1e-4")
    r = G3.solve_pair(r0, r1, I.TRIANGLE, tau=1.0, max_iters=500000, tol=1e-4)
    s = _solver(torch, r0, r1, I.TRIANGLE, "f64", tau=1.0)
    info = s.solve(500000, 1e-4, 64)
    assert r["converged"] and info["converged"]
    assert info["iters"] == r["iters"]
    assert abs(info["residual"] - r["residual"]) <= 1e-6 * r["residual"]


@pytest.mark.parametrize("k,edges", [(3, I.TRIANGLE), (2, [(0, 1)]), (1, np.zeros((0, 2))), (3, [(0, 2), (1, 2)])])
def test_fp32_within_target_tolerances(k, edges):
    torch = cuda()
    m, n, p = 24, 70, 12
    r0, r1 = I.random_volume_pair(53, m, n, p, k)
    r0c, r1c = cast_inputs(r0, r1, "f32")
    note(f"case: 3-D fp32 {m}x{n}x{p} k{k} l{len(edges)} 1500 it")
    r = G3.solve_pair(r0c, r1c, edges, alpha=0.03, tau=1.0, max_iters=1500)
    _active(r["state"], "fp32", need_w=len(edges) > 0)
    s = _solver(torch, r0, r1, edges, "f32", alpha=0.03, tau=1.0)
    s.solve(1500, 0.0, 64)
    V, _ = s.distance()
    Phi = s.grad()[0].double().cpu().numpy()
    relV = abs(V - r["primal"]) / r["primal"]
    ePhi = np.abs(Phi - r["Phi"]).max()
    note(f"3-D fp32: rel V {relV:.2e}, max |dPhi| {ePhi:.2e}")
    assert relV <= 1e-4 and ePhi <= 1e-3


def test_slices_per_wave_do_not_change_bits():
    """Any chunking of the slices (and the autotuned one) gives the same
    iterates, from an active warm state."""
    torch = cuda()
    m, n, p = 21, 130, 17
    r0, r1 = I.random_volume_pair(54, m, n, p, 3)
    q = G3.Problem3(m, n, p, 3, edges=I.TRIANGLE, alpha=1.0, tau=3.0)
    rng = np.random.default_rng(5)
    phi = (np.sin(np.arange(m)[:, None, None, None] / 3.0) + np.cos(np.arange(n)[None, :, None, None] / 5.0)
           + np.sin(np.arange(p)[None, None, :, None] / 2.0)) * 0.05 + np.array([0.0, 1.2, -1.1])
    u = rng.uniform(-q.mu, q.mu, size=(m, n, p, 3, 3))
    w = rng.uniform(-50 * q.nu, 50 * q.nu, size=(m, n, p, 3))
    phi, u, w = (x.astype(np.float32) for x in (phi, u, w))
    out = []
    for zch in (1, 2, 5, 17, 0):
        s = _solver(torch, r0, r1, I.TRIANGLE, "f32", alpha=1.0, tau=3.0, rows_per_wave=zch)
        s.set_state(to_dev(torch, phi, torch.float32), to_dev(torch, u, torch.float32), to_dev(torch, w, torch.float32))
        s.solve(24, 0.0, 8)
        out.append(s.get_state())
    t = _solver(torch, r0, r1, I.TRIANGLE, "f32", alpha=1.0, tau=3.0)
    T, rows, us = t.autotune(16)
    note(f"3-D autotune: T {T}, {rows} slices per wave, {us:.2f} us per iteration")
    assert T == 1
    t.set_state(to_dev(torch, phi, torch.float32), to_dev(torch, u, torch.float32), to_dev(torch, w, torch.float32))
    t.solve(24, 0.0, 8)
    out.append(t.get_state())
    st = out[0]
    g = {"ux": st["u"][..., 0].cpu().numpy(), "uy": st["u"][..., 1].cpu().numpy(),
         "uz": st["u"][..., 2].cpu().numpy(), "w": st["w"].cpu().numpy()}
    _active(g, "warm 3-D state after 24 it")
    for o in out[1:]:
        for key in ("phi", "u", "w"):
            assert torch.equal(out[0][key], o[key]), key


def test_3d_state_roundtrip_and_errors():
    torch = cuda()
    from paper_1712_10279_amd import omt
    r0, r1 = I.random_volume_pair(55, 9, 20, 6, 3)
    s = _solver(torch, r0, r1, I.TRIANGLE, "f64")
    s.solve(100, 0.0, 64)
    st = s.get_state()
    assert st["u"].shape == (9, 20, 6, 3, 3)
    b = _solver(torch, r0, r1, I.TRIANGLE, "f64")
    b.set_state(st["phi"], st["u"], st["w"])
    st2 = b.get_state()
    for key in ("phi", "u", "w"):
        assert torch.equal(st[key], st2[key])
    # ghosts zeroed on set: u_z on the last slice
    ones = torch.ones_like(st["u"])
    b.set_state(st["phi"], ones, st["w"])
    ub = b.get_state()["u"]
    assert torch.all(ub[:, :, -1, :, 2] == 0) and torch.all(ub[:, :, :-1, :, 2] == 1)
    assert torch.all(ub[-1, :, :, :, 0] == 0) and torch.all(ub[:, -1, :, :, 1] == 0)
    with pytest.raises(omt.OMTError) as e:
        _solver(torch, r0, r1 * 1.01, I.TRIANGLE, "f64")
    assert e.value.status == omt.EMASS
    r5a, r5b = I.random_volume_pair(56, 6, 7, 3, 5)
    with pytest.raises(omt.OMTError) as e:
        _solver(torch, r5a, r5b, I.path_edges(5), "f32")
    assert e.value.status == omt.EUNSUPPORTED


def test_full_volume_sampled_cones_from_active_state():
    """256 x 256 x 128, k = 3 triangle (the 3-D workload), FP32, 12
    iterations from a synthetic active state in the default launch shape:
    the oracle on the cube of radius 14 around each sample."""
    torch = cuda()
    d = I.volume_256()
    m, n, p, k = d["rho0"].shape
    r0c, r1c = cast_inputs(d["rho0"], d["rho1"], "f32")
    q = G3.Problem3(m, n, p, k, edges=d["edges"], alpha=d["alpha"], tau=d["tau"])
    rng = np.random.default_rng(6)
    ii = np.arange(m)[:, None, None, None]
    jj = np.arange(n)[None, :, None, None]
    zz = np.arange(p)[None, None, :, None]
    phi = (0.004 * np.sin(2 * np.pi * ii / 24.0) + 0.004 * np.cos(2 * np.pi * jj / 20.0)
           + 0.004 * np.sin(2 * np.pi * zz / 16.0) + np.array([0.0, 0.5 * d["alpha"] + 0.6, -0.6]))
    u = rng.uniform(-q.mu, q.mu, size=(m, n, p, k, 3))
    w = rng.uniform(-50 * d["alpha"] * q.nu, 50 * d["alpha"] * q.nu, size=(m, n, p, 3))
    phi, u, w = (x.astype(np.float32).astype(np.float64) for x in (phi, u, w))
    iters = 12
    note("case: 3-D 256x256x128 k3 fp32, warm active state, 12 it, sampled cones")
    s = _solver(torch, d["rho0"], d["rho1"], d["edges"], "f32", alpha=d["alpha"], tau=d["tau"])
    s.set_state(to_dev(torch, phi, torch.float32), to_dev(torch, u, torch.float32), to_dev(torch, w, torch.float32))
    s.solve(iters, 0.0, 64)
    g = _gpu_state(s)
    f, _ = G3.prepare_f(r0c, r1c, q.edges)
    samples = [(0, 0, 0), (m - 1, n - 1, p - 1), (m // 2, 61, p // 2), (m // 2, 62, 1), (5, 124, p - 2),
               (m - 3, 0, 64)] + [(int(rng.integers(m)), int(rng.integers(n)), int(rng.integers(p))) for _ in range(6)]
    orc, gpu = [], []
    rad = iters + 2
    for (i, j, z) in samples:
        i0, i1 = max(0, i - rad), min(m, i + rad + 1)
        j0, j1 = max(0, j - rad), min(n, j + rad + 1)
        z0, z1 = max(0, z - rad), min(p, z + rad + 1)
        qc = G3.Problem3(i1 - i0, j1 - j0, z1 - z0, k, edges=q.edges, alpha=q.alpha, tau=q.tau, mu=q.mu, nu=q.nu,
                         h=q.h)
        st = {"phi": phi[i0:i1, j0:j1, z0:z1], "ux": u[i0:i1, j0:j1, z0:z1, :, 0].copy(),
              "uy": u[i0:i1, j0:j1, z0:z1, :, 1].copy(), "uz": u[i0:i1, j0:j1, z0:z1, :, 2].copy(),
              "w": w[i0:i1, j0:j1, z0:z1]}
        if i1 == m:
            st["ux"][-1] = 0
        if j1 == n:
            st["uy"][:, -1] = 0
        if z1 == p:
            st["uz"][:, :, -1] = 0
        o = G3.solve(qc, f[i0:i1, j0:j1, z0:z1], iters, 0.0, 1 << 30, st)["state"]
        c = (i - i0, j - j0, z - z0)
        orc.append({key: o[key][c] for key in ("phi", "ux", "uy", "uz", "w")})
        gpu.append({key: g[key][i, j, z] for key in ("phi", "ux", "uy", "uz", "w")})
    cat = lambda lst, key: np.stack([x[key] for x in lst])  # noqa: E731
    _active({key: cat(orc, key) for key in ("ux", "uy", "uz", "w")}, "3-D cones")
    tol = {"phi": 2e-6, "ux": 1e-3, "uy": 1e-3, "uz": 1e-3, "w": 1e-4}
    for key in ("phi", "ux", "uy", "uz", "w"):
        a, b = cat(gpu, key), cat(orc, key)
        err = np.abs(a - b).max() / np.abs(b).max()
        note(f"3-D cones {key}: {err:.2e}")
        assert err <= tol[key], key
