"""CPU checks of the C ABI library: it loads, exports every symbol
include/omt.h declares, and its host-only calls validate parameters and
compute the step sizes of Sec. 7.2 (no device work is done here)."""
import math
import os
import re

import numpy as np
import pytest

from paper_1712_10279_amd import omt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hdr.endswith(".h"):
            src = open(os.path.join(ROOT, "include", hdr)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(omt_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 20
    L = omt.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(omt._SIGS), set(names) ^ set(omt._SIGS)
    assert omt.lib().omt_version() >= 1


def test_step_sizes_follow_the_rule():
    h, mu, nu, lm = omt.resolve_params(33, 33, 3, [(0, 1), (0, 2), (1, 2)], tau=3.0)
    assert h == pytest.approx(1 / 32)
    assert mu == pytest.approx(1 / (32 * 3 * 32 ** 2))
    assert lm == pytest.approx(3.0, abs=1e-12)
    assert nu == pytest.approx(1 / (4 * 3 * 3.0))
    h, mu, nu, lm = omt.resolve_params(17, 9, 1, np.zeros((0, 2)), tau=1.0)
    assert mu == pytest.approx(1 / (16 * 16 ** 2)) and nu == 0.0 and lm == 0.0
    _, _, _, lm = omt.resolve_params(8, 8, 8, [(c, c + 1) for c in range(7)])
    assert lm == pytest.approx(2 + 2 * math.cos(math.pi / 8), abs=1e-12)


@pytest.mark.parametrize("edges,kw,status", [
    ([(1, 0)], {}, omt.EGRAPH),                  # a >= b
    ([(0, 3)], {}, omt.EGRAPH),                  # node out of range
    ([(0, 1), (0, 1)], {}, omt.EGRAPH),          # duplicate
    ([(0, 1)], {"cost": [0.0]}, omt.EGRAPH),     # c <= 0
    ([(0, 1)], {"alpha": 0.0}, omt.EINVAL),
    ([(0, 1)], {"tau": -1.0}, omt.EINVAL),
    ([(0, 1)], {"unorm": 7}, omt.EINVAL),
    ([(0, 1)], {"mu": 1.0}, omt.ESTEP),          # violates tau mu 8/h^2 + tau nu lmax < 1
    ([(0, 1)], {"nu": 10.0}, omt.ESTEP),
    ([(0, 1)], {"eps": -1.0}, omt.EINVAL),       # regularisation weight must be >= 0
])
def test_invalid_parameters(edges, kw, status):
    with pytest.raises(omt.OMTError) as e:
        omt.resolve_params(10, 12, 3, edges, **kw)
    assert e.value.status == status


def test_size_limits():
    with pytest.raises(omt.OMTError) as e:
        omt.resolve_params(1, 10, 3, [])
    assert e.value.status == omt.EINVAL
    with pytest.raises(omt.OMTError) as e:
        omt.resolve_params(10, 10, 9, [])
    assert e.value.status == omt.EUNSUPPORTED
    with pytest.raises(omt.OMTError) as e:
        omt.resolve_params(10, 10, 0, [])
    assert e.value.status == omt.EINVAL
    # each field (here the 16 flux planes) must stay below 2 GiB: 32-bit
    # byte offsets inside the kernels' row buffers
    path8 = [(c, c + 1) for c in range(7)]
    omt.resolve_params(5760, 5760, 8, path8)
    for m, n, dt in ((5824, 5824, "f32"), (5760, 5760, "f64")):
        with pytest.raises(omt.OMTError) as e:
            omt.resolve_params(m, n, 8, path8, dtype=dt)
        assert e.value.status == omt.EUNSUPPORTED


def test_workspace_size_grows_with_problem():
    a = omt.workspace_bytes(256, 256, 3, [(0, 1), (0, 2), (1, 2)])
    b = omt.workspace_bytes(1024, 1024, 8, [(c, c + 1) for c in range(7)])
    c = omt.workspace_bytes(1024, 1024, 8, [(c, c + 1) for c in range(7)], compensated=True)
    d = omt.workspace_bytes(1024, 1024, 8, [(c, c + 1) for c in range(7)], dtype="f64")
    # f, 2 x phi, 2 x u (2k planes), 2 x w: (7k + 2l) planes
    assert b >= (7 * 8 + 2 * 7) * 1024 * 1024 * 4
    assert a < b < c and d >= 2 * (7 * 8 + 2 * 7) * 1024 * 1024 * 4
    assert omt.workspace_bytes(33, 70, 3, []) % 256 == 0


def test_status_strings():
    L = omt.lib()
    for s in range(10):
        assert L.omt_strerror(s)


L_DTI = np.array([[[1, 0, 0], [0, 2, 0], [0, 0, 0]], [[1, 1, 1], [1, 0, 0], [1, 0, 0]]], float)
PAULI = {"x": np.array([[0, 1], [1, 0]], complex), "y": np.array([[0, -1j], [1j, 0]]),
         "z": np.array([[1, 0], [0, -1]], complex)}


def test_matrix_step_sizes_and_coordinates():
    import oracle.matrix as M
    h, mu, nu, lm, K, KW = omt.matrix_resolve(40, 50, L_DTI, True, tau=3.0)
    # lambda_max(-Delta_L) of the example matrices: the oracle's k^2 x k^2 matrix
    assert lm == pytest.approx(M.lambda_max(L_DTI), rel=1e-12)
    assert (K, KW) == (6, 6) and h == pytest.approx(1 / 49)
    assert mu == pytest.approx(h * h / 96) and nu == pytest.approx(1 / (12 * lm))
    L2 = np.stack([PAULI["x"], PAULI["z"]])
    _, _, _, lm2, K2, KW2 = omt.matrix_resolve(10, 10, L2, False)
    assert (K2, KW2) == (4, 8) and lm2 == pytest.approx(M.lambda_max(L2), rel=1e-12)
    # complex 3 x 3 with two L_s: nine coordinates of Phi, eighteen of W
    Lc = np.stack([PAULI["x"].real, PAULI["z"].real])
    L3 = np.stack([np.array([[1, 1j, 0], [-1j, 0, 2], [0, 2, -1]]), np.diag([1.0, 0.0, -2.0]).astype(complex)])
    _, _, _, lm4, K4, KW4 = omt.matrix_resolve(10, 10, L3, False)
    assert (K4, KW4) == (9, 18) and lm4 == pytest.approx(M.lambda_max(L3), rel=1e-12)
    # a single L_s always commutes with itself, so the real 2 x 2 case takes two
    _, _, _, lm3, K3, KW3 = omt.matrix_resolve(10, 10, np.stack([PAULI["x"].real, PAULI["z"].real]), True)
    assert (K3, KW3) == (3, 2) and lm3 == pytest.approx(M.lambda_max(np.stack([PAULI["x"], PAULI["z"]])), rel=1e-12)


@pytest.mark.parametrize("L,real,kw,status", [
    (PAULI["x"][None], False, {}, omt.EGRAPH),            # sigma_x commutes with itself: ker is span(I, sigma_x)
    (np.array([[[0, 1], [0, 0]]], complex), False, {}, omt.EINVAL),   # not Hermitian
    (PAULI["y"][None], True, {}, omt.EINVAL),             # imaginary L in the real mode
    (np.stack([np.array([[1, 1j, 0], [-1j, 0, 2], [0, 2, -1]]), np.diag([1.0, 0.0, -2.0]).astype(complex)]), False,
     {"unorm": omt.M_NUC}, omt.EUNSUPPORTED),           # nuclear norms of complex 3 x 3
    (np.stack([np.eye(3), np.diag([1.0, 2, 3])]), True, {}, omt.EGRAPH),  # commuting diagonals
    (np.stack([PAULI["x"], PAULI["z"], PAULI["y"]]), False, {}, omt.EUNSUPPORTED),  # 12 transfer coordinates
    (L_DTI, True, {"tau": 0.0}, omt.EINVAL),
    (L_DTI, True, {"mu": 1.0}, omt.ESTEP),
    (L_DTI, True, {"tblock": 3}, omt.EINVAL),              # one or two iterations per pass
    (L_DTI, True, {"tblock": 2, "unorm": omt.M_NUC}, omt.EUNSUPPORTED),   # nuclear: one per pass
    (L_DTI, True, {"tblock": 2, "dtype": omt.F64}, omt.EUNSUPPORTED),     # FP64: one per pass
    (np.stack([np.array([[1, 1j, 0], [-1j, 0, 2], [0, 2, -1]]), np.diag([1.0, 0.0, -2.0]).astype(complex)]), False,
     {"tblock": 2}, omt.EUNSUPPORTED),                   # complex 3 x 3: one per pass
])
def test_matrix_invalid_parameters(L, real, kw, status):
    with pytest.raises(omt.OMTError) as e:
        omt.matrix_resolve(12, 12, L, real, **kw)
    assert e.value.status == status


def test_matrix_two_iterations_per_pass_accepted():
    for L, real in ((L_DTI, True), (np.stack([PAULI["x"], PAULI["z"]]), False)):
        for unorm, wnorm in ((omt.M_FRO, omt.M_L1), (omt.M_L1, omt.M_FRO)):
            omt.matrix_resolve(12, 12, L, real, tblock=2, unorm=unorm, wnorm=wnorm)


def test_static_entry_rejects_oversize_before_device_work():
    """omt_solve_static refuses a problem beyond its fixed workspace with
    OMT_ENOMEM before touching the device (so this runs without a GPU)."""
    import ctypes as C
    p, keep = omt.make_params(1024, 1024, 3, [(0, 1), (0, 2), (1, 2)], omt.Config(), omt.F32)
    need = omt.workspace_bytes(1024, 1024, 3, [(0, 1), (0, 2), (1, 2)])
    assert need > 64 << 20
    st = omt.lib().omt_solve_static(C.byref(p), None, None, 10, 0.0, 64, None, None, None, None, None)
    assert st == omt.ENOMEM
    assert b"static workspace" in omt.lib().omt_last_error()
    p.k = 0
    assert omt.lib().omt_solve_static(C.byref(p), None, None, 10, 0.0, 64, None, None, None, None, None) == omt.EINVAL


def test_loss_reports_unconverged_pairs():
    """omt_loss's policy for solves that stop above tol (host logic only)."""
    import warnings
    ok = {"converged": True, "iters": 64, "residual": 1e-7}
    bad = {"converged": False, "iters": 128, "residual": 3e-4}
    omt._notconv([ok, ok], 1e-6, "raise")
    omt._notconv([ok, bad], 0.0, "raise")          # tol 0: a fixed iteration count, nothing to report
    omt._notconv([ok, bad], 1e-6, "ignore")
    with pytest.raises(omt.OMTError) as e:
        omt._notconv([ok, bad], 1e-6, "raise")
    assert e.value.status == omt.ENOTCONV and "(1, 128," in str(e.value)
    with warnings.catch_warnings(record=True) as got:
        warnings.simplefilter("always")
        omt._notconv([bad, ok, bad], 1e-6, "warn")
    assert len(got) == 1 and issubclass(got[0].category, omt.NotConvergedWarning)
    assert "2 of 3" in str(got[0].message)
