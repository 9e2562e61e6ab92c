"""Parity of the matrix-OMT HIP path (through the C ABI of
include/omt_matrix.h) with the FP64 whole-matrix oracle (Sec. 4, Sec. 7.3).
The GPU carries the matrices in orthonormal coordinates; the oracle works on
complex k x k matrices, so agreement also checks the packing, the operator
and the grouped norms."""
import numpy as np
import pytest

import oracle.matrix as MO
from gpu_util import cuda, note
from paper_1712_10279_amd import inputs as I

pytestmark = pytest.mark.gpu

rng = np.random.default_rng(44)


def _herm(k):
    A = rng.normal(size=(k, k)) + 1j * rng.normal(size=(k, k))
    return (A + A.conj().T) / 2


CASES = {  # name: (m, n, k, real, L)
    "dti_real_k3": (40, 70, 3, True, I.L_DTI),
    "pauli_real_k2": (21, 130, 2, True, I.L_PAULI_XZ.real.copy()),
    "complex_k2": (33, 65, 2, False, np.stack([I.L_PAULI_XZ[0] + 0.3 * _herm(2), I.L_PAULI_XZ[1]])),
    "dti_plus_one_real_k3": (3, 130, 3, True, np.stack([I.L_DTI[0], I.L_DTI[1], np.diag([0.0, 1.0, -1.0])])),
    "complex_k3": (20, 70, 3, False, np.stack([_herm(3), _herm(3)])),
}


def _dev(torch, a, real, f64):
    if real:
        return torch.as_tensor(np.ascontiguousarray(a.real), dtype=torch.float64 if f64 else torch.float32,
                               device="cuda")
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.complex128 if f64 else torch.complex64,
                           device="cuda")


def _np(t):
    return t.cpu().numpy().astype(np.complex128)


def _solver(torch, case, f64=True, seed=5, **kw):
    from paper_1712_10279_amd import omt
    m, n, k, real, L = CASES[case]
    lam0, lam1 = I.matrix_pair(seed, m, n, k, real)
    if not f64:
        # both sides see the inputs as rounded to the kernel's dtype
        cast = np.float32 if real else np.complex64
        lam0, lam1 = lam0.astype(cast).astype(np.complex128), lam1.astype(cast).astype(np.complex128)
    s = omt.MatrixSolver(_dev(torch, lam0, real, f64), _dev(torch, lam1, real, f64), L, **kw)
    return s, lam0, lam1, L


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("unorm,wnorm", [(MO.FRO, MO.L1), (MO.L1, MO.L1), (MO.FRO, MO.FRO), (MO.L1, MO.FRO)])
def test_fp64_state_matches_oracle(case, unorm, wnorm):
    torch = cuda()
    iters = 150
    note(f"case: matrix fp64 {case} unorm {unorm} wnorm {wnorm} {iters} it")
    s, lam0, lam1, L = _solver(torch, case, alpha=0.8, tau=2.0, unorm=unorm, wnorm=wnorm)
    info = s.solve(iters, 0.0, 50)
    r = MO.solve_pair(lam0, lam1, L, alpha=0.8, tau=2.0, unorm=unorm, wnorm=wnorm, max_iters=iters, check_every=50)
    st = s.get_state()
    for key in ("phi", "ux", "uy", "w"):
        a, b = _np(st[key]), r["state"][key]
        scale = max(np.abs(b).max(), 1e-300)
        assert np.abs(a - b).max() <= 1e-9 * scale, (key, np.abs(a - b).max(), scale)
    M, inf = s.distance()
    assert M == pytest.approx(r["primal"], rel=1e-10)
    assert info["residual"] == pytest.approx(r["residual"], rel=1e-8)
    assert inf["dual"] == pytest.approx(r["dual"], rel=1e-8, abs=1e-14)


# the oracle's nuclear shrinks diagonalise a 2k x 2k real image per matrix,
# so these cases stay small
NUC_CASES = {  # name: (m, n, k, real, L)
    "dti_real_k3": (6, 70, 3, True, I.L_DTI),
    "pauli_real_k2": (9, 66, 2, True, I.L_PAULI_XZ.real.copy()),
    "complex_k2": (7, 65, 2, False, CASES["complex_k2"][4]),
    "dti_plus_one_real_k3": (3, 66, 3, True, CASES["dti_plus_one_real_k3"][4]),
}


@pytest.mark.parametrize("case", list(NUC_CASES))
@pytest.mark.parametrize("unorm,wnorm", [(MO.NUC, MO.NUC), (MO.FRO, MO.NUC), (MO.NUC, MO.L1)])
def test_fp64_nuclear_norms_match_oracle(case, unorm, wnorm):
    """Nuclear norms (per-pixel eigendecompositions on the GPU: closed form
    for 2 x 2, Jacobi for real 3 x 3; the oracle diagonalises the real image
    of each complex matrix)."""
    torch = cuda()
    from paper_1712_10279_amd import omt
    m, n, k, real, L = NUC_CASES[case]
    iters = 60
    note(f"case: matrix fp64 nuclear {case} unorm {unorm} wnorm {wnorm} {iters} it")
    lam0, lam1 = I.matrix_pair(6, m, n, k, real)
    s = omt.MatrixSolver(_dev(torch, lam0, real, True), _dev(torch, lam1, real, True), L, alpha=0.8, tau=2.0,
                         unorm=unorm, wnorm=wnorm)
    info = s.solve(iters, 0.0, 30)
    r = MO.solve_pair(lam0, lam1, L, alpha=0.8, tau=2.0, unorm=unorm, wnorm=wnorm, max_iters=iters, check_every=30)
    st = s.get_state()
    for key in ("phi", "ux", "uy", "w"):
        a, b = _np(st[key]), r["state"][key]
        assert np.abs(a - b).max() <= 1e-9 * max(np.abs(b).max(), 1e-300), key
    M, _ = s.distance()
    assert M == pytest.approx(r["primal"], rel=1e-10)
    assert info["residual"] == pytest.approx(r["residual"], rel=1e-8)


def test_fp32_nuclear_within_tolerance():
    torch = cuda()
    from paper_1712_10279_amd import omt
    note("case: matrix fp32 nuclear dti 8x24, 500 it")
    iters = 500
    lam0, lam1 = I.matrix_pair(7, 8, 24, 3, True)
    lam0, lam1 = lam0.astype(np.float32).astype(np.float64), lam1.astype(np.float32).astype(np.float64)
    s = omt.MatrixSolver(_dev(torch, lam0, True, False), _dev(torch, lam1, True, False), I.L_DTI, alpha=1.0,
                         tau=2.0, unorm=MO.NUC, wnorm=MO.NUC)
    s.solve(iters, 0.0, 64)
    r = MO.solve_pair(lam0, lam1, I.L_DTI, alpha=1.0, tau=2.0, unorm=MO.NUC, wnorm=MO.NUC, max_iters=iters)
    M, _ = s.distance()
    assert abs(M - r["primal"]) <= 1e-4 * r["primal"]


@pytest.mark.parametrize("case", ["dti_real_k3", "pauli_real_k2", "complex_k2", "dti_plus_one_real_k3"])
@pytest.mark.parametrize("comp", [False, True])
def test_two_iterations_per_pass_are_bit_identical(case, comp):
    """FP32 launches of two iterations (T = 2: one HBM pass, halo lanes and
    rows recomputed) give the bits of single-iteration launches, for any
    strip height, in timed launches and in a solve with checks."""
    torch = cuda()
    note(f"case: matrix T=2 bits {case} comp={comp}")
    kw = dict(f64=False, alpha=0.8, tau=2.0, compensated=comp, unorm=MO.FRO, wnorm=MO.L1)
    ref = _solver(torch, case, tblock=1, **kw)[0]
    ref.time_steps(0, 48)
    a = ref.get_state()
    for rows in (0, 5):
        s = _solver(torch, case, tblock=2, rows_per_wave=rows, **kw)[0]
        s.time_steps(rows, 48)
        b = s.get_state()
        for key in ("phi", "ux", "uy", "w"):
            assert torch.equal(a[key], b[key]), (case, comp, rows, key)
    s1 = _solver(torch, case, tblock=1, **kw)[0]
    s2 = _solver(torch, case, tblock=2, **kw)[0]
    i1, i2 = s1.solve(200, 0.0, 32), s2.solve(200, 0.0, 32)
    assert i1["residual"] == i2["residual"] and i1["primal"] == i2["primal"]
    a, b = s1.get_state(), s2.get_state()
    for key in ("phi", "ux", "uy", "w"):
        assert torch.equal(a[key], b[key]), (case, comp, "solve", key)


@pytest.mark.parametrize("case", ["dti_real_k3", "complex_k2", "complex_k3"])
def test_fp64_gradient_is_the_oracle_potential(case):
    torch = cuda()
    note(f"case: matrix gradient {case}")
    s, lam0, lam1, L = _solver(torch, case, alpha=1.3, tau=1.0)
    s.solve(400, 0.0, 64)
    r = MO.solve_pair(lam0, lam1, L, alpha=1.3, tau=1.0, max_iters=400)
    d0, d1 = s.grad()
    assert torch.equal(d0, -d1)
    g = _np(d0)
    assert np.abs(g - r["Phi"]).max() <= 1e-9 * np.abs(r["Phi"]).max()
    # Hermitian with zero total trace
    assert np.allclose(g, np.conj(np.swapaxes(g, -1, -2)), atol=1e-14)
    assert abs(np.trace(g.sum((0, 1)))) < 1e-9


@pytest.mark.parametrize("comp", [False, True])
def test_fp32_within_tolerance(comp):
    torch = cuda()
    note(f"case: matrix fp32 dti comp={comp}")
    iters = 3000
    s, lam0, lam1, L = _solver(torch, "dti_real_k3", f64=False, alpha=1.0, tau=2.0, compensated=comp)
    s.solve(iters, 0.0, 64)
    r = MO.solve_pair(lam0, lam1, L, alpha=1.0, tau=2.0, max_iters=iters)
    M, _ = s.distance()
    assert abs(M - r["primal"]) <= 1e-4 * r["primal"]
    d0, _ = s.grad()
    assert np.abs(_np(d0) - r["Phi"]).max() <= 1e-3


def test_stopping_decision_matches_oracle():
    torch = cuda()
    note("case: matrix tol 3e-3 complex k2")
    s, lam0, lam1, L = _solver(torch, "complex_k2", alpha=0.6, tau=1.0)
    info = s.solve(100000, 3e-3, 32)
    r = MO.solve_pair(lam0, lam1, L, alpha=0.6, tau=1.0, max_iters=100000, tol=3e-3, check_every=32)
    assert info["converged"] and r["converged"]
    assert info["iters"] == r["iters"]


def test_matrix_error_paths():
    torch = cuda()
    from paper_1712_10279_amd import omt
    m, n, k, real, L = CASES["dti_real_k3"]
    lam0, lam1 = I.matrix_pair(9, m, n, k, real)
    note("case: matrix EMASS")
    with pytest.raises(omt.OMTError) as e:
        omt.MatrixSolver(_dev(torch, lam0, True, True), _dev(torch, 1.5 * lam1, True, True), L)
    assert e.value.status == omt.EMASS
    note("case: matrix NaN")
    bad = lam1.copy()
    bad[3, 4, 0, 1] = np.nan
    with pytest.raises(omt.OMTError) as e:
        omt.MatrixSolver(_dev(torch, lam0, True, True), _dev(torch, bad, True, True), L)
    assert e.value.status == omt.EINVAL


def _active(st):
    """Fractions of pixels where the oracle's U (either axis) and W (any
    edge) are non-zero."""
    u = (np.abs(st["ux"]) + np.abs(st["uy"])).reshape(st["ux"].shape[0], st["ux"].shape[1], -1).max(-1)
    w = np.abs(st["w"]).reshape(st["w"].shape[0], st["w"].shape[1], -1).max(-1)
    return (u > 0).mean(), (w > 0).mean()


def _compare_state(st, r, rel):
    for key in ("phi", "ux", "uy", "w"):
        a, b = _np(st[key]), r["state"][key]
        scale = max(np.abs(b).max(), 1e-300)
        assert np.abs(a - b).max() <= rel * scale, (key, np.abs(a - b).max(), scale)
        # where the oracle's shrink returned zero the kernel's must too
        assert np.abs(a[b == 0]).max(initial=0.0) <= rel * scale, key


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("unorm,wnorm", [(MO.FRO, MO.L1), (MO.L1, MO.L1), (MO.FRO, MO.FRO), (MO.L1, MO.FRO)])
def test_fp64_active_state_matches_oracle(case, unorm, wnorm):
    """alpha = 0.1, 1200 iterations: U and W are non-zero on most pixels (the
    test asserts at least 20 % each), so every shrink divides."""
    torch = cuda()
    iters = 1200
    note(f"case: matrix fp64 active {case} unorm {unorm} wnorm {wnorm} {iters} it")
    s, lam0, lam1, L = _solver(torch, case, alpha=0.1, tau=2.0, unorm=unorm, wnorm=wnorm)
    info = s.solve(iters, 0.0, 64)
    r = MO.solve_pair(lam0, lam1, L, alpha=0.1, tau=2.0, unorm=unorm, wnorm=wnorm, max_iters=iters, check_every=64)
    ua, wa = _active(r["state"])
    assert ua >= 0.2 and wa >= 0.2, (ua, wa)
    _compare_state(s.get_state(), r, 1e-9)
    M, inf = s.distance()
    assert M == pytest.approx(r["primal"], rel=1e-10)
    assert info["residual"] == pytest.approx(r["residual"], rel=1e-8)
    assert inf["dual"] == pytest.approx(r["dual"], rel=1e-8, abs=1e-14)
    assert inf["mass_residual"] == pytest.approx(r["mass_residual"], rel=1e-8)


@pytest.mark.parametrize("case", list(NUC_CASES))
@pytest.mark.parametrize("unorm,wnorm", [(MO.NUC, MO.NUC), (MO.FRO, MO.NUC), (MO.NUC, MO.L1)])
def test_fp64_nuclear_active_state_matches_oracle(case, unorm, wnorm):
    """Nuclear norms at alpha = 0.1, 150 iterations, U and W active on at
    least 20 % of pixels each."""
    torch = cuda()
    from paper_1712_10279_amd import omt
    m, n, k, real, L = NUC_CASES[case]
    iters = 150
    note(f"case: matrix fp64 nuclear active {case} unorm {unorm} wnorm {wnorm} {iters} it")
    lam0, lam1 = I.matrix_pair(6, m, n, k, real)
    s = omt.MatrixSolver(_dev(torch, lam0, real, True), _dev(torch, lam1, real, True), L, alpha=0.1, tau=2.0,
                         unorm=unorm, wnorm=wnorm)
    info = s.solve(iters, 0.0, 30)
    r = MO.solve_pair(lam0, lam1, L, alpha=0.1, tau=2.0, unorm=unorm, wnorm=wnorm, max_iters=iters, check_every=30)
    ua, wa = _active(r["state"])
    assert ua >= 0.2 and wa >= 0.2, (ua, wa)
    _compare_state(s.get_state(), r, 1e-9)
    M, _ = s.distance()
    assert M == pytest.approx(r["primal"], rel=1e-10)
    assert info["residual"] == pytest.approx(r["residual"], rel=1e-8)


@pytest.mark.parametrize("case", ["dti_real_k3", "pauli_real_k2", "complex_k2", "dti_plus_one_real_k3"])
def test_two_iterations_per_pass_bit_identical_when_active(case):
    """FP32 solves with one and two iterations per launch give the same bits
    after 1200 iterations at alpha = 0.1, where U and W are non-zero on at
    least 20 % of pixels; the FP32 distance stays within 1e-4 of the FP64
    oracle's."""
    torch = cuda()
    note(f"case: matrix T=2 bits active {case}")
    kw = dict(f64=False, alpha=0.1, tau=2.0, unorm=MO.FRO, wnorm=MO.L1)
    s1, lam0, lam1, L = _solver(torch, case, tblock=1, **kw)
    s2 = _solver(torch, case, tblock=2, **kw)[0]
    i1, i2 = s1.solve(1200, 0.0, 64), s2.solve(1200, 0.0, 64)
    assert i1["residual"] == i2["residual"] and i1["primal"] == i2["primal"]
    a, b = s1.get_state(), s2.get_state()
    for key in ("phi", "ux", "uy", "w"):
        assert torch.equal(a[key], b[key]), (case, key)
    ua, wa = _active({key: _np(a[key]) for key in ("ux", "uy", "w")})
    assert ua >= 0.2 and wa >= 0.2, (ua, wa)
    r = MO.solve_pair(lam0, lam1, L, alpha=0.1, tau=2.0, max_iters=1200, check_every=64)
    M, _ = s2.distance()
    assert abs(M - r["primal"]) <= 1e-4 * r["primal"]
