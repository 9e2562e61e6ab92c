"""The persistent batched kernel against per-problem solves (and, through
them, the oracle): every problem of a batch must end with bit-identical
iterates, iteration counts and stopping decisions to its own solve."""
import numpy as np
import pytest

from gpu_util import cuda, note, to_dev
from paper_1712_10279_amd import inputs as I

pytestmark = pytest.mark.gpu

SHAPES = [  # (m, n, k, edges)
    (64, 64, 1, None),
    (70, 130, 3, I.TRIANGLE),
    (33, 65, 2, [(0, 1)]),
    (128, 96, 3, I.path_edges(3)),
    (2, 5, 3, I.TRIANGLE),
    (150, 40, 1, None),
]


def _problems(torch, seed, comp=False, tau=None, dtype=None):
    dtype = dtype or torch.float32
    out = []
    for q, (m, n, k, e) in enumerate(SHAPES):
        r0, r1 = I.random_pair(seed + q, m, n, k)
        out.append(dict(rho0=to_dev(torch, r0, dtype), rho1=to_dev(torch, r1, dtype), edges=e,
                        alpha=0.5 + 0.3 * q, tau=tau or I.default_tau(m, n), compensated=comp))
    return out


def _plain(torch, pr, iters, tol):
    from paper_1712_10279_amd import omt
    kw = {key: v for key, v in pr.items() if key not in ("rho0", "rho1", "edges")}
    s = omt.Solver(pr["rho0"], pr["rho1"], pr["edges"], **kw)
    info = s.solve(iters, tol, 64)
    return s, info


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("mode", ["f32", "f32comp", "f64"])
def test_batch_fixed_iterations_bit_identical(mode, persistent, monkeypatch):
    torch = cuda()
    from paper_1712_10279_amd import omt
    if persistent:
        monkeypatch.setenv("OMT_BATCH_PERSISTENT", "1")
    comp = mode == "f32comp"
    probs = _problems(torch, 40, comp, dtype=torch.float64 if mode == "f64" else torch.float32)
    note(f"case: batch of {len(probs)} fixed 300 iterations mode={mode} persistent={persistent}")
    b = omt.BatchSolver(probs)
    infos = b.solve(300, 0.0, 64)
    Vb = b.distance()
    for q, pr in enumerate(probs):
        s, info = _plain(torch, pr, 300, 0.0)
        assert infos[q]["iters"] == info["iters"] == 300
        gs, bs = s.get_state(), b.get_state(q)
        for key in ("phi", "u", "w"):
            assert torch.equal(gs[key], bs[key]), (q, key)
        assert infos[q]["residual"] == info["residual"]
        assert Vb[q] == s.distance()[0]


@pytest.mark.parametrize("persistent", [False, True])
def test_batch_to_tolerance_same_decisions(persistent, monkeypatch):
    torch = cuda()
    from paper_1712_10279_amd import omt
    if persistent:
        monkeypatch.setenv("OMT_BATCH_PERSISTENT", "1")
    probs = _problems(torch, 50, True)
    note(f"case: batch to tol 1e-3 persistent={persistent}")
    b = omt.BatchSolver(probs)
    infos = b.solve(200000, 1e-3, 64)
    for q, pr in enumerate(probs):
        s, info = _plain(torch, pr, 200000, 1e-3)
        note(f"  problem {q}: batch {infos[q]['iters']} it conv {infos[q]['converged']}, "
             f"plain {info['iters']} it conv {info['converged']}")
        assert infos[q]["iters"] == info["iters"]
        assert infos[q]["converged"] == info["converged"] == 1
        gs, bs = s.get_state(), b.get_state(q)
        for key in ("phi", "u", "w"):
            assert torch.equal(gs[key], bs[key]), (q, key)
    # a second solve continues from where each problem stopped
    infos2 = b.solve(128, 0.0, 64)
    assert all(i["iters"] == 128 for i in infos2)
    d0, d1 = b.grad()
    for q in range(len(probs)):
        assert torch.equal(d0[q], -d1[q])


def test_batch_rejects_unsupported_problem():
    torch = cuda()
    from paper_1712_10279_amd import omt
    r0, r1 = I.random_pair(60, 20, 20, 5)
    with pytest.raises(omt.OMTError) as e:
        omt.BatchSolver([dict(rho0=to_dev(torch, r0, torch.float32), rho1=to_dev(torch, r1, torch.float32),
                              edges=I.path_edges(5))])
    assert e.value.status == omt.EUNSUPPORTED


def test_batch_f64_to_tolerance_matches_oracle():
    """FP64 batch to a tight tolerance: the same decisions as each problem's
    own solve, and the distance of the oracle run for the same count."""
    torch = cuda()
    from paper_1712_10279_amd import omt
    import oracle
    probs = _problems(torch, 70, dtype=torch.float64)[:3]
    note("case: FP64 batch of 3 to tol 1e-6")
    b = omt.BatchSolver(probs)
    infos = b.solve(20000, 1e-6, 64)
    Vb = b.distance()
    for q, pr in enumerate(probs):
        s, info = _plain(torch, pr, 20000, 1e-6)
        assert infos[q]["iters"] == info["iters"] and infos[q]["converged"] == info["converged"]
        gs, bs = s.get_state(), b.get_state(q)
        for key in ("phi", "u", "w"):
            assert torch.equal(gs[key], bs[key]), (q, key)
        m, n, k, e = SHAPES[q]
        r0 = pr["rho0"].cpu().numpy()
        r1 = pr["rho1"].cpu().numpy()
        res = oracle.solve_pair(r0, r1, e if e is not None else np.zeros((0, 2)), alpha=pr["alpha"],
                                tau=pr["tau"], max_iters=infos[q]["iters"])
        note(f"  problem {q}: {infos[q]['iters']} it, V batch {Vb[q]:.12g} oracle {res['primal']:.12g}")
        assert abs(Vb[q] - res["primal"]) <= 1e-9 * max(1.0, abs(res["primal"]))


def test_batch_rejects_mixed_dtypes():
    torch = cuda()
    from paper_1712_10279_amd import omt
    probs = _problems(torch, 80)[:2]
    probs[1] = dict(probs[1], rho0=probs[1]["rho0"].double(), rho1=probs[1]["rho1"].double())
    with pytest.raises(ValueError):
        omt.BatchSolver(probs)


@pytest.mark.parametrize("mode", ["f32", "f64"])
def test_batch_autotune_keeps_bits_and_caches_rows(mode, tmp_path, monkeypatch):
    """omt_batch_autotune picks rows per shape class without changing any
    iterate; the tuned batch stays bit-identical to per-problem solves, a
    caller's fixed rows are kept, and a new batch takes the tuned rows from
    the tuning cache."""
    torch = cuda()
    from paper_1712_10279_amd import omt
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("OMT_TUNE_CACHE", str(cache))
    dt = torch.float64 if mode == "f64" else torch.float32
    probs = _problems(torch, 70, dtype=dt)
    probs[1]["rows_per_wave"] = 3
    note(f"case: batch autotune {mode}, {len(probs)} problems")
    b = omt.BatchSolver(probs)
    b.solve(100, 0.0, 64)
    before = [b.get_state(q) for q in range(len(probs))]
    rows, us = b.autotune(8)
    note(f"  tuned rows {rows}, {us:.2f} us per batched iteration")
    assert len(rows) == len(probs) and all(r >= 1 for r in rows) and us > 0
    assert rows[1] == 3
    for q in range(len(probs)):
        st = b.get_state(q)
        for key in ("phi", "u", "w"):
            assert torch.equal(st[key], before[q][key]), (q, key)
    infos = b.solve(300, 0.0, 64)
    for q, pr in enumerate(probs):
        s, _ = _plain(torch, pr, 100, 0.0)
        info = s.solve(300, 0.0, 64)
        gs, bs = s.get_state(), b.get_state(q)
        for key in ("phi", "u", "w"):
            assert torch.equal(gs[key], bs[key]), (q, key)
        assert infos[q]["residual"] == info["residual"]
    # one cache entry per shape class tuned (problem 1's rows were fixed)
    assert cache.read_text().count('"batch ') == len(SHAPES) - 1
    b2 = omt.BatchSolver(_problems(torch, 71, dtype=dt))
    rows2, us2 = b2.autotune(0)
    assert us2 == 0.0
    assert rows2[:1] + rows2[2:] == rows[:1] + rows[2:]


@pytest.mark.parametrize("check_every,iters", [(7, 23), (8, 30), (5, 11), (2, 9)])
def test_batch_interval_schedules_bit_identical(check_every, iters):
    """Check intervals of every parity (two-iteration launches, an odd
    single one, the checked one; a short last interval): each problem of
    the batch ends with the bits and checks of its own solve."""
    torch = cuda()
    from paper_1712_10279_amd import omt
    probs = _problems(torch, 80, dtype=torch.float64)
    note(f"case: batch intervals of {check_every}, {iters} iterations")
    b = omt.BatchSolver(probs)
    infos = b.solve(iters, 0.0, check_every)
    for q, pr in enumerate(probs):
        kw = {key: v for key, v in pr.items() if key not in ("rho0", "rho1", "edges")}
        s = omt.Solver(pr["rho0"], pr["rho1"], pr["edges"], **kw)
        info = s.solve(iters, 0.0, check_every)
        assert infos[q]["iters"] == info["iters"] == iters and infos[q]["checks"] == info["checks"]
        assert infos[q]["residual"] == info["residual"]
        gs, bs = s.get_state(), b.get_state(q)
        for key in ("phi", "u", "w"):
            assert torch.equal(gs[key], bs[key]), (q, key)
