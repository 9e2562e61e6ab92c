"""Parity with the FP64 oracle at states where the shrinks are active.

From the zero start the potential grows as k tau f until the first shrink
fires, so short runs compare nothing but phi = k tau f.  Every test here
reaches (or starts from) a state in which the flux u and the transfer w are
non-zero on a large part of the grid, and asserts that fraction on the
oracle's side, so the comparison cannot slide back to the trivial regime.
Cases:
  * the 8-channel path graph of the large workload on a small grid, solved
    from zero long enough for both shrinks to fire (FP64 element-wise; FP32
    at the target tolerances in one- and two-iteration launches, which must
    agree bit for bit);
  * the full 1024 x 1024 k = 8 grid from a synthetic active state, in the
    benchmark's launch shape, on sampled cones (FP32 and FP64);
  * launches of T = 2, 4, 8 iterations against T = 1 from an active state;
  * the norm ||w||_2, FP32 with w active, the regularised method with w
    active, and the check quantities (constraint residual, gap) against the
    oracle.
"""
import numpy as np
import pytest

import oracle as O
from gpu_util import active_fraction, cast_inputs, cone_oracle, cuda, gpu_state_np, note, to_dev
from paper_1712_10279_amd import inputs as I

pytestmark = pytest.mark.gpu

MIN_ACTIVE = 0.2  # fraction of compared pixels with u != 0, and with w != 0


def _solver(torch, rho0, rho1, edges, dtype, **kw):
    from paper_1712_10279_amd import omt
    tdt = torch.float64 if dtype == "f64" else torch.float32
    return omt.Solver(to_dev(torch, rho0, tdt), to_dev(torch, rho1, tdt), edges, **kw)


def _assert_active(st, what, need_w=True):
    ua, wa = active_fraction(st["ux"], st["uy"], st["w"])
    note(f"{what}: oracle active fraction u {ua:.3f} w {wa:.3f}")
    assert ua >= MIN_ACTIVE, (what, ua)
    if need_w:
        assert wa >= MIN_ACTIVE, (what, wa)


def _cmp_state(g, st, tol, what):
    """Element-wise, relative to each field's largest entry; a field the
    oracle leaves at zero must be zero on the GPU as well."""
    errs = {}
    for key, a, b in (("phi", g["phi"], st["phi"]), ("ux", g["u"][..., 0], st["ux"]),
                      ("uy", g["u"][..., 1], st["uy"]), ("w", g["w"], st["w"])):
        if b.size == 0:
            continue
        scale = np.abs(b).max()
        errs[key] = np.abs(a - b).max() / scale if scale > 0 else np.abs(a).max()
    note(f"{what}: " + " ".join(f"{key} {v:.2e}" for key, v in errs.items()))
    for key, v in errs.items():
        assert v <= tol, (what, key, v)


def _path8_small():
    d = I.path8_1024(m=64, n=80)
    return d["rho0"], d["rho1"], d["edges"]


PATH8_KW = dict(alpha=0.1, tau=3.0)
PATH8_ITERS = 2000


def test_path8_active_fp64_elementwise():
    """k = 8 path, channel masses moved (the large workload's generator on
    64 x 80), alpha 0.1, 2000 iterations: FP64 state element-wise to 1e-10,
    and every check quantity against the oracle's."""
    torch = cuda()
    r0, r1, edges = _path8_small()
    note("case: path8 64x80 fp64 2000 it active")
    r = O.solve_pair(r0, r1, edges, max_iters=PATH8_ITERS, check_every=64, **PATH8_KW)
    _assert_active(r["state"], "path8 64x80")
    s = _solver(torch, r0, r1, edges, "f64", **PATH8_KW)
    info = s.solve(PATH8_ITERS, 0.0, 64)
    _cmp_state(gpu_state_np(s), r["state"], 1e-10, "path8 fp64")
    V, dinfo = s.distance()
    assert abs(V - r["primal"]) <= 1e-10 * r["primal"]
    assert abs(info["dual"] - r["dual"]) <= 1e-10 * abs(r["primal"])
    assert abs(info["rel_gap"] - r["rel_gap"]) <= 1e-8 * max(abs(r["rel_gap"]), 1e-3)
    assert abs(info["mass_residual"] - r["mass_residual"]) <= 1e-8 * r["mass_residual"]
    assert abs(info["residual"] - r["residual"]) <= 1e-8 * r["residual"]
    assert abs(dinfo["mass_residual"] - r["mass_residual"]) <= 1e-8 * r["mass_residual"]
    Phi = s.grad()[0].cpu().numpy()
    assert np.abs(Phi - r["Phi"]).max() <= 1e-9 * np.abs(r["Phi"]).max()


@pytest.mark.parametrize("comp", [False, True])
def test_path8_active_fp32_blocked_and_single(comp):
    """The same problem in FP32: V to 1e-4 relative and Phi to 1e-3 max-abs
    against the oracle, and two-iteration launches (rows 0, 5, 10) give the
    bits of single-iteration launches."""
    torch = cuda()
    r0, r1, edges = _path8_small()
    r0c, r1c = cast_inputs(r0, r1, "f32")
    note(f"case: path8 64x80 fp32 comp={comp} 2000 it, T=1 and T=2")
    r = O.solve_pair(r0c, r1c, edges, max_iters=PATH8_ITERS, check_every=64, **PATH8_KW)
    _assert_active(r["state"], "path8 64x80 fp32")
    ref = _solver(torch, r0, r1, edges, "f32", compensated=comp, tblock=1, **PATH8_KW)
    iref = ref.solve(PATH8_ITERS, 0.0, 64)
    V, _ = ref.distance()
    Phi = ref.grad()[0].double().cpu().numpy()
    relV = abs(V - r["primal"]) / r["primal"]
    ePhi = np.abs(Phi - r["Phi"]).max()
    note(f"fp32 T=1: rel V {relV:.2e} max|dPhi| {ePhi:.2e} (|Phi| max {np.abs(r['Phi']).max():.2e})")
    assert relV <= 1e-4 and ePhi <= 1e-3
    a = ref.get_state()
    for rows in (0, 5, 10):
        s = _solver(torch, r0, r1, edges, "f32", compensated=comp, tblock=2, rows_per_wave=rows, **PATH8_KW)
        i2 = s.solve(PATH8_ITERS, 0.0, 64)
        b = s.get_state()
        for key in ("phi", "u", "w"):
            assert torch.equal(a[key], b[key]), (rows, key)
        assert i2["residual"] == iref["residual"] and i2["primal"] == iref["primal"]


# ------------------------------------------------------ full size, warm state

def _warm(d, p, seed=1):
    """Synthetic active state for the problem (FP32-representable)."""
    m, n, k = d["rho0"].shape
    phi, u, w = I.warm_state(seed, m, n, k, p.l, u_scale=p.mu, w_scale=50.0 * p.alpha * p.nu,
                             offset=p.alpha)
    return tuple(x.astype(np.float32).astype(np.float64) for x in (phi, u, w))


def _samples(m, n, rng, count):
    fixed = [(0, 0), (0, n - 1), (m - 1, 0), (m - 1, n - 1), (m // 2, 63), (m // 2, 64), (7, n // 2),
             (m - 2, n - 65), (m // 3, 59), (m // 3, 60), (m // 4, 119), (m // 4, 120)]
    rand = [(int(rng.integers(m)), int(rng.integers(n))) for _ in range(count)]
    return fixed + rand


def _cones(torch, d, dtype, iters, shapes, tol, nsamp=8):
    """Run each launch shape from the same warm state, require identical bits
    across shapes, and compare sampled cones with the oracle."""
    from paper_1712_10279_amd import omt
    m, n, k = d["rho0"].shape
    r0, r1 = cast_inputs(d["rho0"], d["rho1"], dtype)
    p = O.Problem(m, n, k, edges=d["edges"], alpha=d["alpha"], tau=d["tau"])
    phi, u, w = _warm(d, p)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    states = []
    for (T, rows) in shapes:
        s = omt.Solver(to_dev(torch, d["rho0"], tdt), to_dev(torch, d["rho1"], tdt), d["edges"], alpha=d["alpha"],
                       tau=d["tau"], tblock=max(T, 0), rows_per_wave=rows)
        if T == -1:  # the benchmark's shape: from the autotuner
            T, rows, us = s.autotune()
            note(f"autotuned shape: T {T}, {rows} rows per wave, {us:.2f} us per iteration")
        s.set_state(to_dev(torch, phi, tdt), to_dev(torch, u, tdt), to_dev(torch, w, tdt))
        s.solve(iters, 0.0, 64)
        states.append(gpu_state_np(s))
        del s
    for q in range(1, len(states)):
        for key in ("phi", "u", "w"):
            assert np.array_equal(states[0][key], states[q][key]), (shapes[q], key)
    g = states[0]
    f, _ = O.prepare_f(r0, r1, p.edges)
    full = {"phi": phi, "ux": u[..., 0], "uy": u[..., 1], "w": w}
    rng = np.random.default_rng(7)
    orc, gpu = [], []
    for (i, j) in _samples(m, n, rng, nsamp):
        o = cone_oracle(f, p, (i, j), iters, state=full)
        orc.append(o)
        gpu.append({"phi": g["phi"][i, j], "ux": g["u"][i, j, :, 0], "uy": g["u"][i, j, :, 1], "w": g["w"][i, j]})
    cat = lambda lst, key: np.stack([x[key] for x in lst])
    _assert_active({key: cat(orc, key) for key in ("ux", "uy", "w")}, f"{m}x{n} cones after {iters} it")
    errs = {}
    for key in ("phi", "ux", "uy", "w"):
        a, b = cat(gpu, key), cat(orc, key)
        errs[key] = np.abs(a - b).max() / np.abs(b).max()
    note(f"{dtype} cones: " + " ".join(f"{key} {v:.2e}" for key, v in errs.items()))
    for key, v in errs.items():
        assert v <= tol[key], (key, v)


# FP32: phi's rounding (spacing ~2.4e-7 at |phi| ~ 2) enters the gradient
# divided by h ~ 1e-3 and then the flux through mu / h, so the flux carries
# ~1e-4 of its scale; phi and w carry a few spacings of phi.
FP32_CONE_TOL = {"phi": 2e-6, "ux": 1e-3, "uy": 1e-3, "w": 1e-4}


def test_large_grid_cones_from_active_state_fp32():
    """1024 x 1024, k = 8 path (the benchmark's problem), FP32, 24 iterations
    from a synthetic state with u and w active: the autotuned shape, T = 2
    with 10 rows per wave, and T = 1 give identical bits and match the
    oracle's cones."""
    torch = cuda()
    d = I.path8_1024()
    note("case: 1024x1024 k8 path fp32, warm active state, 24 it, shapes autotuned / T2 r10 / T1")
    _cones(torch, d, "f32", 24, [(-1, 0), (2, 10), (1, 0)], FP32_CONE_TOL)


def test_large_grid_cones_from_active_state_fp64():
    """The same in FP64 (single-iteration launches), element-wise to 1e-10."""
    torch = cuda()
    d = I.path8_1024()
    note("case: 1024x1024 k8 path fp64, warm active state, 24 it")
    tol = {key: 1e-10 for key in ("phi", "ux", "uy", "w")}
    _cones(torch, d, "f64", 24, [(1, 0), (1, 3)], tol)


def test_loss_grid_cones_fp64_two_iterations_per_launch():
    """512 x 512, k = 3 triangle, tau 1024 (the loss workload's problem),
    FP64 from an active state: two iterations per launch (the default strips
    and 5-row strips) and single-iteration launches give identical bits and
    match the oracle's cones to 1e-10."""
    torch = cuda()
    d = I.loss_512(0)
    note("case: 512x512 k3 triangle fp64, warm active state, 24 it, shapes T2 / T2 r5 / T1")
    _cones(torch, d, "f64", 24, [(2, 0), (2, 5), (1, 0)], {key: 1e-10 for key in ("phi", "ux", "uy", "w")})


@pytest.mark.parametrize("k,edges", [(3, I.TRIANGLE), (3, [(0, 1), (1, 2)]), (5, I.path_edges(5)),
                                     (8, I.path_edges(8)), (2, [(0, 1)]), (1, np.zeros((0, 2)))])
@pytest.mark.parametrize("comp", [False, True])
def test_blocking_bit_identical_from_active_state(k, edges, comp):
    """T = 2, 4, 8 iterations per pass against T = 1 from a state with u and
    w active (activity asserted on the oracle's run of the same steps)."""
    torch = cuda()
    from paper_1712_10279_amd import omt
    m, n, iters = 77, 200, 24
    r0, r1 = I.random_pair(27, m, n, k)
    p = O.Problem(m, n, k, edges=edges, alpha=1.0, tau=3.0)
    phi, u, w = I.warm_state(5, m, n, k, p.l, u_scale=p.mu, w_scale=50.0 * p.nu, offset=1.0)
    phi, u, w = (x.astype(np.float32) for x in (phi, u, w))
    f, _ = O.prepare_f(*cast_inputs(r0, r1, "f32"), p.edges)
    o = O.solve(p, f, iters, 0.0, 1 << 30,
                state={"phi": phi, "ux": u[..., 0], "uy": u[..., 1], "w": w})["state"]
    _assert_active(o, f"k{k} l{p.l} warm {iters} it", need_w=p.l > 0)

    def run(T, rows):
        s = _solver(torch, r0, r1, edges, "f32", compensated=comp, tau=3.0)
        s.set_state(to_dev(torch, phi, torch.float32), to_dev(torch, u, torch.float32),
                    to_dev(torch, w, torch.float32) if p.l else None)
        s.time_steps(T, rows, iters)
        return s.get_state()

    a = run(1, 0)
    tested = 0
    for T in (2, 4, 8):
        for rows in (0, 5, 16):
            try:
                b = run(T, rows)
            except omt.OMTError as e:
                assert e.status == omt.EUNSUPPORTED
                continue
            tested += 1
            for key in ("phi", "u", "w"):
                assert torch.equal(a[key], b[key]), (k, T, rows, key)
    note(f"case: k{k} comp{comp}: {tested} blocked shapes bit-identical to T=1")
    assert tested >= 3


# ------------------------------------------------------ other active paths

def test_w_l2_norm_active_fp64():
    """||w||_2 with the transfer active (alpha 0.05): element-wise to 1e-10."""
    torch = cuda()
    r0, r1 = I.random_pair(22, 48, 90, 3)
    kw = dict(alpha=0.05, tau=1.0, unorm=0, wnorm=1)
    note("case: fp64 48x90 ||w||_2 alpha 0.05 1500 it")
    r = O.solve_pair(r0, r1, I.TRIANGLE, max_iters=1500, **kw)
    _assert_active(r["state"], "w l2")
    s = _solver(torch, r0, r1, I.TRIANGLE, "f64", **kw)
    info = s.solve(1500, 0.0, 64)
    _cmp_state(gpu_state_np(s), r["state"], 1e-10, "w l2")
    assert abs(info["primal"] - r["primal"]) <= 1e-10 * r["primal"]
    assert abs(info["mass_residual"] - r["mass_residual"]) <= 1e-8 * r["mass_residual"]


@pytest.mark.parametrize("unorm,wnorm", [(1, 0), (2, 1)])
def test_other_norms_active_fp64(unorm, wnorm):
    """||u||_1 and ||u||_2 (with ||w||_1 / ||w||_2) with both shrinks active."""
    torch = cuda()
    r0, r1 = I.random_pair(22, 48, 90, 3)
    kw = dict(alpha=0.05, tau=1.0, unorm=unorm, wnorm=wnorm)
    note(f"case: fp64 48x90 u{unorm} w{wnorm} alpha 0.05 1500 it")
    r = O.solve_pair(r0, r1, I.TRIANGLE, max_iters=1500, **kw)
    _assert_active(r["state"], f"norms {unorm}{wnorm}")
    s = _solver(torch, r0, r1, I.TRIANGLE, "f64", **kw)
    s.solve(1500, 0.0, 64)
    _cmp_state(gpu_state_np(s), r["state"], 1e-10, f"norms {unorm}{wnorm}")


@pytest.mark.parametrize("comp", [False, True])
def test_fp32_with_transfer_active(comp):
    """FP32 iterates with w active on most pixels (alpha 0.05): V to 1e-4
    relative, Phi to 1e-3 max-abs."""
    torch = cuda()
    r0, r1 = I.random_pair(25, 96, 130, 3, bumps=4)
    r0c, r1c = cast_inputs(r0, r1, "f32")
    note(f"case: fp32 96x130 alpha 0.05 3000 it comp={comp}")
    r = O.solve_pair(r0c, r1c, I.TRIANGLE, max_iters=3000, alpha=0.05, tau=3.0)
    _assert_active(r["state"], "fp32 w active")
    s = _solver(torch, r0, r1, I.TRIANGLE, "f32", alpha=0.05, tau=3.0, compensated=comp)
    s.solve(3000, 0.0, 64)
    V, _ = s.distance()
    Phi = s.grad()[0].double().cpu().numpy()
    relV = abs(V - r["primal"]) / r["primal"]
    ePhi = np.abs(Phi - r["Phi"]).max()
    note(f"fp32 w active: rel V {relV:.2e}, max |dPhi| {ePhi:.2e}")
    assert relV <= 1e-4 and ePhi <= 1e-3


@pytest.mark.parametrize("unorm,wnorm", [(0, 0), (2, 1)])
def test_regularised_with_transfer_active_fp64(unorm, wnorm):
    """Quadratic regularisation (Sec. 9) with u and w active (alpha 0.05,
    eps 2, 1500 iterations): element-wise to 1e-10, and the regularised
    primal objective."""
    torch = cuda()
    r0, r1 = I.random_pair(33, 40, 75, 3)
    kw = dict(alpha=0.05, unorm=unorm, wnorm=wnorm, eps=2.0)
    note(f"case: fp64 regularised eps=2 alpha 0.05 u{unorm} w{wnorm} 1500 it")
    r = O.solve_pair(r0, r1, I.TRIANGLE, max_iters=1500, **kw)
    _assert_active(r["state"], "regularised")
    s = _solver(torch, r0, r1, I.TRIANGLE, "f64", **kw)
    info = s.solve(1500, 0.0, 64)
    _cmp_state(gpu_state_np(s), r["state"], 1e-10, "regularised")
    assert abs(info["primal"] - r["primal"]) <= 1e-10 * r["primal"]
    assert abs(info["mass_residual"] - r["mass_residual"]) <= 1e-8 * r["mass_residual"]


@pytest.mark.parametrize("k,edges", [(3, I.TRIANGLE), (3, [(0, 1), (1, 2)]), (2, [(0, 1)]), (1, np.zeros((0, 2)))])
def test_fp64_two_iterations_per_launch_from_active_state(k, edges):
    """FP64 launches of two iterations (k <= 3) from a state with u and w
    active: bit-identical to single-iteration launches for several strip
    heights, and element-wise to 1e-10 of the oracle started from the same
    state."""
    torch = cuda()
    m, n, iters = 77, 200, 24
    r0, r1 = I.random_pair(28, m, n, k)
    p = O.Problem(m, n, k, edges=edges, alpha=1.0, tau=3.0)
    phi, u, w = I.warm_state(6, m, n, k, p.l, u_scale=p.mu, w_scale=50.0 * p.nu, offset=1.0)
    f, _ = O.prepare_f(r0, r1, p.edges)
    o = O.solve(p, f, iters, 0.0, 1 << 30, state={"phi": phi, "ux": u[..., 0], "uy": u[..., 1], "w": w})["state"]
    _assert_active(o, f"fp64 k{k} l{p.l} warm {iters} it", need_w=p.l > 0)
    note(f"case: fp64 T=2 k{k} l{p.l} from an active state")

    def run(T, rows):
        s = _solver(torch, r0, r1, edges, "f64", tau=3.0)
        s.set_state(to_dev(torch, phi, torch.float64), to_dev(torch, u, torch.float64),
                    to_dev(torch, w, torch.float64) if p.l else None)
        s.time_steps(T, rows, iters)
        return s

    a = run(1, 0)
    sa = a.get_state()
    for rows in (0, 5, 16):
        b = run(2, rows).get_state()
        for key in ("phi", "u", "w"):
            assert torch.equal(sa[key], b[key]), (k, rows, key)
    _cmp_state(gpu_state_np(a), o, 1e-10, f"fp64 T=2 k{k}")
