"""Memory outside the grid is never used: with OMT_POISON set, every field's
padding (columns past n of each row, the gaps between planes) holds NaN from
create on, and every launch shape, precision and grid kind must still give
the bits of an unpoisoned run."""
import numpy as np
import pytest

from gpu_util import cuda, note, to_dev
from paper_1712_10279_amd import inputs as I

pytestmark = pytest.mark.gpu


def _run(torch, monkeypatch, poison, make, iters):
    if poison:
        monkeypatch.setenv("OMT_POISON", "1")
    else:
        monkeypatch.delenv("OMT_POISON", raising=False)
    s = make()
    s.solve(iters, 0.0, 32)
    st = s.get_state()
    V, _ = s.distance()
    return st, V


CASES = {  # name: (m, n, k, edges, dtype, kw)
    "k3_triangle_f32_T1": (77, 130, 3, I.TRIANGLE, "f32", dict(tblock=1)),
    "k3_triangle_f32_T2_rows5": (77, 130, 3, I.TRIANGLE, "f32", dict(tblock=2, rows_per_wave=5)),
    "k3_triangle_f32_comp_T2": (45, 70, 3, I.TRIANGLE, "f32", dict(tblock=2, compensated=True)),
    "k8_path_f32_T2": (33, 70, 8, I.path_edges(8), "f32", dict(tblock=2, rows_per_wave=10)),
    "k1_f64": (29, 65, 1, None, "f64", dict()),
    "k3_path_f64": (40, 99, 3, I.path_edges(3), "f64", dict()),
}


@pytest.mark.parametrize("case", list(CASES))
def test_poisoned_padding_changes_nothing(case, monkeypatch):
    torch = cuda()
    from paper_1712_10279_amd import omt
    m, n, k, edges, dt, kw = CASES[case]
    note(f"case: poison {case} {m}x{n} k{k}")
    r0, r1 = I.random_pair(90, m, n, k)
    tdt = torch.float64 if dt == "f64" else torch.float32
    make = lambda: omt.Solver(to_dev(torch, r0, tdt), to_dev(torch, r1, tdt), edges, alpha=0.3, tau=2.0, **kw)  # noqa: E731
    a, Va = _run(torch, monkeypatch, False, make, 300)
    b, Vb = _run(torch, monkeypatch, True, make, 300)
    assert np.isfinite(Vb) and Va == Vb
    for key in ("phi", "u", "w"):
        assert torch.equal(a[key], b[key]), key


def test_poisoned_padding_3d(monkeypatch):
    torch = cuda()
    from paper_1712_10279_amd import omt
    m, n, p = 9, 70, 11
    note(f"case: poison 3-D {m}x{n}x{p} k3")
    r0, r1 = I.random_volume_pair(91, m, n, p, 3)
    make = lambda: omt.Solver(to_dev(torch, r0, torch.float32), to_dev(torch, r1, torch.float32), I.TRIANGLE,  # noqa: E731
                              alpha=0.3, tau=2.0, rows_per_wave=3)
    a, Va = _run(torch, monkeypatch, False, make, 200)
    b, Vb = _run(torch, monkeypatch, True, make, 200)
    assert np.isfinite(Vb) and Va == Vb
    for key in ("phi", "u", "w"):
        assert torch.equal(a[key], b[key]), key


def test_poisoned_padding_matrix_and_batch(monkeypatch):
    torch = cuda()
    from paper_1712_10279_amd import omt
    note("case: poison matrix dti 20x70 and a batch of three")
    lam0, lam1 = I.matrix_pair(92, 20, 70, 3, True)
    mk = lambda: omt.MatrixSolver(to_dev(torch, lam0.real, torch.float32), to_dev(torch, lam1.real, torch.float32),  # noqa: E731
                                  I.L_DTI, alpha=0.5, tau=2.0, tblock=2)
    a, Va = _run(torch, monkeypatch, False, mk, 200)
    b, Vb = _run(torch, monkeypatch, True, mk, 200)
    assert np.isfinite(Vb) and Va == Vb
    for key in ("phi", "ux", "uy", "w"):
        assert torch.equal(a[key], b[key]), key
    shapes = [(64, 64, 1, None), (33, 65, 2, [(0, 1)]), (70, 130, 3, I.TRIANGLE)]
    probs = []
    for q, (m, n, k, e) in enumerate(shapes):
        r0, r1 = I.random_pair(93 + q, m, n, k)
        probs.append(dict(rho0=to_dev(torch, r0, torch.float64), rho1=to_dev(torch, r1, torch.float64), edges=e,
                          alpha=0.5, tau=1.0))
    out = []
    for poison in (False, True):
        if poison:
            monkeypatch.setenv("OMT_POISON", "1")
        else:
            monkeypatch.delenv("OMT_POISON", raising=False)
        bs = omt.BatchSolver(probs)
        bs.solve(200, 0.0, 32)
        out.append([bs.get_state(q) for q in range(len(probs))])
    for q in range(len(probs)):
        for key in ("phi", "u", "w"):
            assert torch.equal(out[0][q][key], out[1][q][key]), (q, key)
