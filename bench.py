"""Throughput of the fused PDHG path on one MI355X.

Workload: vector OMT on a 1024 x 1024 grid, k = 8 channels on a path graph
(7 edges), alpha 1, tau 3, FP32 iterates with FP64 reductions, seeded
16-bump Gaussian mixtures with mass moved between channels (see
``paper_1712_10279_amd/inputs.py``), 20,000 iterations.  One step is one
whole solve: the set-up (mass check, source term, zero state), the 20,000
iterations (gradient, both shrinks, extrapolation, divergences, dual ascent)
with the residual/objective check every 64 iterations, then the distance and
the gradient potential.

Prints one JSON line.  ``value`` is cell-iterations/s (cells = grid pixels,
each carrying all k channels and l edges) with the inputs resident in HBM.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
import warnings

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed steps; a step is one whole solve of the workload")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--iters", type=int, default=0, help="iterations per solve (0: the workload's 20,000)")
    ap.add_argument("--tau", type=float, default=0.0, help="dual step (0: the workload's)")
    ap.add_argument("--no-fp64-check", action="store_true", help="skip the FP64 run that states the FP32 error")
    ap.add_argument("--size", type=int, default=1024, help="grid side (default: the 1024 x 1024 workload)")
    ap.add_argument("--tblock", type=int, default=0, help="iterations per HBM pass (0: library default)")
    ap.add_argument("--rows", type=int, default=0, help="rows per wavefront (0: library default)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=0, help="oracle iterations for the CPU baseline (0: auto)")
    ap.add_argument("--timing-launches", type=int, default=200,
                    help="iterations of step launches timed for the roofline (launches of T iterations each: "
                         "T = 2 times half as many launches)")
    ap.add_argument("--workload", default="large", choices=["large", "batched", "rgb", "loss", "matrix", "volume"],
                    help="large: 1024x1024 k=8 throughput (default); batched: 96 pairs to 1e-5, batched vs "
                         "plain; rgb: 256x256 k=3 time to 1e-5; loss: 8 pairs of 512x512 forward+backward; "
                         "matrix: 3x3 matrix OMT, 256x256 time to a 1e-3 gap and 1024x1024 step roofline; "
                         "volume: 3-D grid 256x256x128, k=3 throughput")
    ap.add_argument("--pairs", type=int, default=96, help="batched workload: number of pairs")
    ap.add_argument("--tol", type=float, default=0.0, help="time-to-tolerance workloads: tolerance (0: workload's)")
    ap.add_argument("--cap", type=int, default=0,
                    help="time-to-tolerance workloads: iteration cap (0: 10 million for the loss workload, whose "
                         "slowest pair needs 6.9 million to reach 1e-6; 3 million otherwise)")
    ap.add_argument("--batch-tune", action="store_true",
                    help="batched workload: rows per strip from omt_batch_autotune instead of the default rule")
    ap.add_argument("--floor-iters", type=int, default=0,
                    help="loss workload: FP64 iterations before the FP32 floors are measured (0: skip)")
    ap.add_argument("--leg", default="both", choices=["both", "plain", "batched"],
                    help="batched workload: time both legs (ratio) or one of them")
    ap.add_argument("--plain-range", default="", metavar="A:B",
                    help="batched workload, plain leg: solve only pairs A..B-1 (the per-pair solves are independent, "
                         "so the leg can be timed in parts)")
    ap.add_argument("--precision", default="auto", choices=["auto", "f32comp", "f64"],
                    help="time-to-tolerance workloads: iterate precision (auto: the workload's)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run plain device-to-device copies of MIB MiB (counter calibration) and exit")
    a = ap.parse_args()
    if a.cap == 0 and a.workload != "loss":
        a.cap = 3_000_000
    return a


def copy_calibration(mib):
    """Plain copies of a known size: the reference for scaling the HBM byte
    counters (FETCH_SIZE, WRITE_SIZE) of the profiler."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 5}), flush=True)


STEP_SOURCES = ("step.hip", "step_device.h", "omt_kernels.h")
STEP3_SOURCES = ("step3.hip", "grid3.h", "step_device.h", "omt_kernels.h")


def _kernel_hash(files=STEP_SOURCES):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1712_10279_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(key, rows=0, files=STEP_SOURCES):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source and the same launch shape."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    e = t.get(key)
    if not e or e.get("kernel_sha") != _kernel_hash(files):
        return None
    if rows and e.get("rows") not in (None, rows):
        return None
    return e.get("bytes_per_launch")


def _timed_from_active_state(s, edges, alpha, tau, T, rows, iters, chunk_iters=32):
    """Time the step kernel (HIP events on the solver's stream, omt_time_steps)
    from a seeded synthetic state in which the flux and transfer shrinks are
    active on most pixels (inputs.warm_state, scaled by the resolved mu and
    nu), so that the measurement never sits in the regime where every shrink
    returns zero.  The iteration relaxes the channel differences of such a
    state within a few hundred iterations (w returns to zero where the data
    need no transfer), so the state is loaded again before every chunk of
    chunk_iters // T iterations (one graph replay of chunk_iters // T^2
    launches); about ``iters`` iterations are timed in all (iters / T
    launches).  Returns (mean us per launch, activity of the state after the
    last timed launch)."""
    import torch
    from paper_1712_10279_amd import inputs as I
    from paper_1712_10279_amd import omt
    m, n, p, k, l = s.m, s.n, s.p, s.k, s.l
    _, mu, nu, _ = omt.resolve_params(m, n, k, edges, depth=p, alpha=alpha, tau=tau)
    kw = dict(u_scale=mu, w_scale=50.0 * alpha * nu, offset=alpha)
    phi, u, w = I.warm_state3(1, m, n, p, k, l, **kw) if p else I.warm_state(1, m, n, k, l, **kw)
    dev = lambda x: torch.as_tensor(x, dtype=s.dtype, device=s.device)  # noqa: E731
    phi, u, w = dev(phi), dev(u), dev(w) if l else None
    per = max(1, chunk_iters // T)
    times = []
    for _ in range(max(1, iters // per)):
        s.set_state(phi, u, w)
        times.append(s.time_steps(T, rows, per))
    return sum(times) / len(times), _activity(s)


def _activity(s):
    """Fractions of cells where the current u (any channel, any axis) and w
    (any edge) are non-zero."""
    st = s.get_state()
    cells = s.m * s.n * max(s.p, 1)
    u = float(((st["u"] != 0).reshape(cells, -1).any(dim=1)).double().mean())
    w = float(((st["w"] != 0).reshape(cells, -1).any(dim=1)).double().mean()) if s.l else 0.0
    return {"u_active": u, "w_active": w}


def _fp32_floor(r0, r1, edges, alpha, tau, state64, V64, g64, iters=2048):
    """What FP32 iterates give on a problem solved in FP64: plain and
    compensated FP32 solves start from the FP64 iterate (rounded to FP32)
    and run ``iters`` iterations; the largest relative residual of their
    last four 512-iteration solves is the floor they sustain there (a
    tolerance below it is out of reach in that precision), and V and Phi are
    compared with the FP64 run's."""
    import torch
    from paper_1712_10279_amd import omt
    out = {}
    for comp in (False, True):
        s = omt.Solver(r0.float(), r1.float(), edges, alpha=alpha, tau=tau, compensated=comp)
        w = state64["w"].float() if state64["w"].shape[-1] else None
        s.set_state(state64["phi"].float(), state64["u"].float(), w)
        res = [s.solve(512, 0.0, 64)["residual"] for _ in range(max(4, iters // 512))]
        V, _ = s.distance()
        g, _ = s.grad()
        out["compensated" if comp else "plain"] = {
            "residual_floor": max(res[-4:]), "rel_V_vs_fp64": abs(V - V64) / V64 if V64 else abs(V),
            "max_abs_Phi_vs_fp64": float((g.double() - g64).abs().max())}
        del s
    torch.cuda.synchronize()
    return out


def cpu_baseline(d, iters):
    """The FP64 oracle, single-threaded, on the same grid for a few iterations."""
    import oracle as O
    p = O.Problem(d["rho0"].shape[0], d["rho0"].shape[1], d["rho0"].shape[2], edges=d["edges"],
                  alpha=d["alpha"], tau=d["tau"])
    f, _ = O.prepare_f(d["rho0"].astype("float32").astype("float64"), d["rho1"].astype("float32").astype("float64"),
                       p.edges)
    r = O.solve(p, f, iters, 0.0, 1 << 30)
    cells = p.m * p.n * iters
    return {"value": cells / r["wall_s"], "unit": "cell-iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} FP64 iterations of the same {p.m}x{p.n}x{p.k} grid, single thread, "
                      f"{r['wall_s']:.1f} s"}


def _line(metric, value, unit, steps, warmup, ms, config, dtype="f32", **extra):
    d = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
         "ms_per_step": ms, "higher_is_better": unit.endswith("/s") or unit == "x", "scaling": "weak",
         "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    d.update(extra)
    return d


def _precision(a, default):
    """(torch dtype, compensated flag, label) of a time-to-tolerance run."""
    import torch
    p = default if a.precision == "auto" else a.precision
    if p == "f64":
        return torch.float64, False, "FP64"
    return torch.float32, True, "compensated FP32"


def _dtype_name(dt):
    import torch
    return "f64" if dt == torch.float64 else "f32"


def _floor_summary(floors, tol):
    """Per precision: how many pairs sustain a residual below tol, the
    largest floor, and the largest V and Phi errors against FP64."""
    out = {}
    for key in ("plain", "compensated"):
        fl = [f[key] for f in floors]
        out[key] = {"pairs_below_tol": sum(f["residual_floor"] <= tol for f in fl), "pairs": len(fl),
                    "max_residual_floor": max(f["residual_floor"] for f in fl),
                    "median_residual_floor": sorted(f["residual_floor"] for f in fl)[len(fl) // 2],
                    "max_rel_V_vs_fp64": max(f["rel_V_vs_fp64"] for f in fl),
                    "max_abs_Phi_vs_fp64": max(f["max_abs_Phi_vs_fp64"] for f in fl)}
    return out


def bench_batched(a):
    """96 pairs (sides 64..512, k in {1, 3}) to a relative residual of 1e-5:
    the batched solve against the per-pair solves, same tau, K, tol and
    precision (identical iteration counts).  FP64 by default: FP32 iterates,
    even with the compensated potential, stall above 1e-5 on some pairs."""
    import torch
    from paper_1712_10279_amd import inputs as I
    from paper_1712_10279_amd import omt
    tol = a.tol or 1e-5
    dt, comp, label = _precision(a, "f64")
    specs = I.batch_spec(a.pairs)
    probs = []
    for sp in specs:
        d = I.batch_pair(sp)
        probs.append(dict(rho0=torch.as_tensor(d["rho0"], dtype=dt, device="cuda"),
                          rho1=torch.as_tensor(d["rho1"], dtype=dt, device="cuda"),
                          edges=d["edges"], alpha=d["alpha"], tau=I.tuned_tau(sp["side"], sp["side"]),
                          compensated=comp, tblock=a.tblock))
    print(f"# batched: {len(probs)} pairs, {label}, tol {tol}", file=sys.stderr, flush=True)
    plain = batch = None
    t_plain = t_batch = None
    if a.leg in ("both", "plain"):
        # plain: one solve after another on one stream
        lo, hi = (int(x) for x in a.plain_range.split(":")) if a.plain_range else (0, len(probs))
        solvers = [omt.Solver(p["rho0"], p["rho1"], p["edges"], alpha=p["alpha"], tau=p["tau"], compensated=comp,
                              tblock=p["tblock"]) for p in probs[lo:hi]]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain = []
        for q, s in enumerate(solvers, start=lo):
            plain.append(s.solve(a.cap, tol, 64))
            sp = specs[q]
            print(f"# plain {q}: side {sp['side']} k {sp['k']} {plain[-1]['iters']} it "
                  f"(residual {plain[-1]['residual']:.2e}), {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        del solvers
    if a.leg in ("both", "batched"):
        os.environ["OMT_VERBOSE"] = "1"
        b = omt.BatchSolver(probs)
        tuned_rows = None
        if a.batch_tune:
            # untimed: rows per strip for every shape class (iterates unchanged)
            tuned_rows, tuned_us = b.autotune()
            print(f"# batched: tuned rows {sorted(set(tuned_rows))}, {tuned_us:.1f} us per all-active iteration",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch = b.solve(a.cap, tol, 64)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        print(f"# batched: {t_batch:.1f} s", file=sys.stderr, flush=True)
    ref = batch if batch is not None else plain
    floors = None
    if batch is not None and dt == torch.float64:
        # FP32 floors of every pair at its FP64 solution
        Vb = b.distance()
        gb, _ = b.grad()
        floors = []
        for q, p in enumerate(probs):
            fl = _fp32_floor(p["rho0"], p["rho1"], p["edges"], p["alpha"], p["tau"], b.get_state(q), Vb[q], gb[q])
            floors.append({"pair": q, "side": specs[q]["side"], "k": specs[q]["k"], **fl})
        print(f"# batched: FP32 floors measured", file=sys.stderr, flush=True)
    its = [i["iters"] for i in ref]
    if batch is None and a.plain_range:
        specs = specs[lo:hi]
    cells = sum(sp["side"] ** 2 * i for sp, i in zip(specs, its))
    extra = dict(converged=sum(i["converged"] for i in ref),
                 iterations={"min": min(its), "median": sorted(its)[len(its) // 2], "max": max(its),
                             "total": sum(its)}, per_pair_iterations=its)
    if plain is not None:
        extra.update(plain_s=t_plain, plain_cell_iter_per_s=cells / t_plain)
    if batch is not None:
        extra.update(batched_s=t_batch, batched_cell_iter_per_s=cells / t_batch, batched_rows=tuned_rows)
    if floors is not None:
        extra["fp32"] = _floor_summary(floors, tol)
        extra["fp32_per_pair"] = floors
    if plain is not None and batch is not None:
        extra["same_iterations"] = all(p["iters"] == q["iters"] for p, q in zip(plain, batch))
        value, unit, metric = t_plain / t_batch, "x", "time to 1e-5 relative residual, batched vs plain"
    else:
        value, unit = (t_plain if batch is None else t_batch), "s"
        metric = f"time to 1e-5 relative residual, {a.leg} leg"
    return _line(metric, value, unit, sum(its), 0, value * 1e3 / max(its) if unit == "s" else t_batch * 1e3 / max(its),
                 dtype=_dtype_name(dt),
                 config={"workload": f"batched_{a.pairs}_pairs_side64-512_k1or3", "pairs": a.pairs, "tol": tol,
                         "check_every": 64, "precision": label, "leg": a.leg, "tblock": a.tblock or "default",
                         "plain_range": a.plain_range or None, "parallelism": "single-gpu"},
                 **extra)


def bench_rgb(a):
    """256x256, k=3 triangle, alpha in {0.5, 1, 4}: time to 1e-5 per pair."""
    import torch
    from paper_1712_10279_amd import inputs as I
    from paper_1712_10279_amd import omt
    tol = a.tol or 1e-5
    # FP64 by default: with FP32 iterates (even the compensated potential)
    # the alpha = 4 pair stalls above 1e-5
    dt, comp, label = _precision(a, "f64")
    out = []
    total_t, total_it = 0.0, 0
    for alpha in (0.5, 1.0, 4.0):
        d = I.rgb_256(alpha)
        s_r0 = torch.as_tensor(d["rho0"], dtype=dt, device="cuda")
        s_r1 = torch.as_tensor(d["rho1"], dtype=dt, device="cuda")
        s = omt.Solver(s_r0, s_r1, d["edges"], alpha=alpha, tau=I.tuned_tau(256, 256), compensated=comp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s.solve(a.cap, tol, 64)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        total_t += el
        total_it += info["iters"]
        print(f"# rgb alpha {alpha}: {info['iters']} it, {el:.2f} s", file=sys.stderr, flush=True)
        V = s.distance()[0]
        row = {"alpha": alpha, "seconds": el, "iterations": info["iters"], "converged": info["converged"],
               "residual": info["residual"], "V": V, "rel_gap": info["rel_gap"]}
        if dt == torch.float64:
            row["fp32"] = _fp32_floor(s_r0, s_r1, d["edges"], alpha, I.tuned_tau(256, 256), s.get_state(), V,
                                      s.grad()[0])
            print(f"# rgb alpha {alpha}: FP32 floors plain {row['fp32']['plain']['residual_floor']:.2e} "
                  f"compensated {row['fp32']['compensated']['residual_floor']:.2e}", file=sys.stderr, flush=True)
        out.append(row)
    return _line("time to 1e-5 relative residual", total_t, "s", total_it, 0, total_t * 1e3 / total_it,
                 dtype=_dtype_name(dt), config={"workload": "vomt_256x256_k3_triangle_3alphas", "tol": tol,
                                                "precision": label, "tau": I.tuned_tau(256, 256),
                                                "parallelism": "single-gpu"}, pairs=out)


def bench_loss(a):
    """8 pairs of 512x512, k=3: forward to 1e-6 and backward (+-Phi)."""
    import torch
    from paper_1712_10279_amd import inputs as I
    from paper_1712_10279_amd import omt
    tol = a.tol or 1e-6
    dt, comp, label = _precision(a, "f64")
    ds = [I.loss_512(q) for q in range(8)]
    r0 = torch.stack([torch.as_tensor(d["rho0"], dtype=dt, device="cuda") for d in ds]).requires_grad_(True)
    r1 = torch.stack([torch.as_tensor(d["rho1"], dtype=dt, device="cuda") for d in ds])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tau = a.tau or ds[0]["tau"]
    cap = a.cap or 10_000_000
    with warnings.catch_warnings(record=True) as caught:
        warnings.simplefilter("always")
        V = omt.omt_loss(r0, r1, I.TRIANGLE, max_iters=cap, tol=tol, tau=tau, compensated=comp)
        V.sum().backward()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    notconv = [str(w.message) for w in caught if issubclass(w.category, omt.NotConvergedWarning)]
    extra = {}
    if dt == torch.float64 and a.floor_iters > 0:
        # untimed: the same pairs solved by the batched FP64 solver for
        # floor_iters iterations (or to tol), then the FP32 floors at that
        # iterate, pair by pair
        b = omt.BatchSolver([dict(rho0=r0[q].detach(), rho1=r1[q], edges=I.TRIANGLE, tau=tau) for q in range(len(ds))])
        infos = b.solve(a.floor_iters, tol, 64)
        Vb = b.distance()
        gb, _ = b.grad()
        rows = []
        for q, info in enumerate(infos):
            rows.append({"pair": q, "iterations": info["iters"], "converged": info["converged"],
                         "residual": info["residual"],
                         **_fp32_floor(r0[q].detach(), r1[q], I.TRIANGLE, 1.0, tau, b.get_state(q), Vb[q], gb[q])})
            print(f"# loss pair {q}: {info['iters']} it, residual {info['residual']:.2e}, FP32 floors "
                  f"{rows[-1]['plain']['residual_floor']:.2e} / {rows[-1]['compensated']['residual_floor']:.2e}",
                  file=sys.stderr, flush=True)
        del b
        extra = {"fp32": _floor_summary(rows, tol), "fp32_floor_iterate": f"FP64 after up to {a.floor_iters} iterations",
                 "per_pair": rows}
    return _line("forward+backward time, 8 pairs to 1e-6", el, "s", 8, 0, el * 1e3 / 8, dtype=_dtype_name(dt),
                 config={"workload": "loss_8x512x512_k3_triangle", "tol": tol, "tau": tau, "cap": cap,
                         "precision": label, "parallelism": "single-gpu"}, V=[float(v) for v in V.detach().cpu()],
                 not_converged=notconv, **extra)


def bench_matrix(a):
    """Matrix OMT (Sec. 7.3) on diffusion-tensor-like real 3 x 3 fields with
    the two matrices L_1, L_2 of the paper's example, ||U||_2 and ||W||_1:
    time to |relative duality gap| <= 1e-3 on 256 x 256 with tau = 60 (the
    precision measure, grid and tau of the paper's matrix table), and the
    step kernel against the HBM roofline on 1024 x 1024."""
    import torch
    from paper_1712_10279_amd import inputs as I
    from paper_1712_10279_amd import omt
    gap = a.tol or 1e-3
    dt, comp, label = _precision(a, "f32comp")
    D = I.dti_like(256)
    dev = lambda x: torch.as_tensor(x, dtype=dt, device="cuda")
    s = omt.MatrixSolver(dev(D["lam0"]), dev(D["lam1"]), D["L"], alpha=1.0, tau=60.0, compensated=comp,
                         tblock=a.tblock)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it, info = 0, None
    while it < a.cap:
        info = s.solve(1024, 0.0, 64)
        it += 1024
        # the gap of an iterate that is not yet feasible can have either sign
        if abs(info["rel_gap"]) <= gap:
            break
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    M01, _ = s.distance()
    print(f"# matrix 256: {it} it, {el:.2f} s, M {M01:.6g}, gap {info['rel_gap']:.2e}", file=sys.stderr, flush=True)
    # throughput of the step kernel on a 1024 x 1024 field
    # (two iterations per launch in FP32, the library's default at this size)
    T = a.tblock if a.tblock > 0 else (2 if dt == torch.float32 else 1)
    B = I.dti_like(1024)
    s2 = omt.MatrixSolver(dev(B["lam0"]), dev(B["lam1"]), B["L"], alpha=1.0, tau=60.0, compensated=comp, tblock=T)
    s2.solve(64, 0.0, 64)
    us = s2.time_steps(0, max(1, a.timing_launches // T) * T)
    K, KW = 6, 6
    per_px = (7 * K + 2 * KW) * (8 if dt == torch.float64 else 4) + (2 * K * 4 if comp else 0)
    bytes_launch = per_px * 1024 * 1024 * T
    ach = bytes_launch / us / 1e3
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": f"pdhg_step_kernel (matrix kind, K=6 coordinates, 6 transfer coordinates, T = {T})",
            "bytes_per_launch": bytes_launch, "us_per_launch": us}
    return _line("matrix OMT time to 1e-3 relative duality gap", el, "s", it, 0, el * 1e3 / it, dtype=_dtype_name(dt),
                 config={"workload": "momt_256x256_real3x3_dti_L", "gap": gap, "tau": 60.0, "alpha": 1.0,
                         "precision": label, "parallelism": "single-gpu"},
                 roofline=roof, M=M01, rel_gap=info["rel_gap"], iterations=it,
                 cell_iter_per_s=1024 * 1024 * T / (us * 1e-6))


def bench_volume(a):
    """3-D grid (256 x 256 x 128 cells, k = 3 triangle, alpha 1, FP32): one
    step is a whole solve of 2,000 iterations with checks every 64; the step
    kernel against the HBM roofline."""
    import torch
    from paper_1712_10279_amd import inputs as I
    from paper_1712_10279_amd import omt
    d = I.volume_256()
    m, n, p, k = d["rho0"].shape
    l = len(d["edges"])
    iters = a.iters or d["iters"]
    r0 = torch.as_tensor(d["rho0"], dtype=torch.float32, device="cuda")
    r1 = torch.as_tensor(d["rho1"], dtype=torch.float32, device="cuda")
    rows = a.rows
    if rows == 0:
        s = omt.Solver(r0, r1, d["edges"], alpha=d["alpha"], tau=d["tau"])
        _, rows, _ = s.autotune()
        del s

    def one_solve():
        s = omt.Solver(r0, r1, d["edges"], alpha=d["alpha"], tau=d["tau"], rows_per_wave=rows)
        info = s.solve(iters, 0.0, 64)
        V, _ = s.distance()
        s.grad()
        return s, info, V

    for _ in range(a.warmup):
        one_solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s, info, V = one_solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cells = m * n * p
    value = cells * iters * a.steps / dt
    act = _activity(s)
    us, timed_act = _timed_from_active_state(s, d["edges"], d["alpha"], d["tau"], 1, rows,
                                             max(1, a.timing_launches))
    alg = (9 * k + 2 * l) * 4 * cells  # reads phi k, u 3k, w l, f k; writes phi k, u 3k, w l
    ach = alg / (us * 1e-6) / 1e9
    traffic = _traffic(f"step3_{m}x{n}x{p}_k{k}", rows, STEP3_SOURCES)
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": traffic, "kernel": "pdhg_step3_kernel (one iteration per launch)", "us_per_launch": us,
            "bytes_per_launch": alg, "timed_from": "seeded active state (inputs.warm_state3)", **timed_act}
    if traffic:
        roof["counted_gbs"] = traffic / (us * 1e-6) / 1e9
        roof["counted_frac"] = roof["counted_gbs"] / HBM_PEAK_GBS
    line = _line("PDHG cell-iterations/s, 3-D grid", value, "cell-iter/s", a.steps, a.warmup, dt * 1e3 / a.steps,
                 config={"workload": d["name"], "grid": [m, n, p], "channels": k, "edges": l, "graph": "triangle",
                         "alpha": d["alpha"], "tau": d["tau"], "iterations_per_step": iters, "check_every": 64,
                         "slices_per_wave": rows, "parallelism": "single-gpu"},
                 roofline=roof, solve={"primal": V, "residual": info["residual"], "rel_gap": info["rel_gap"], **act})
    if not a.no_cpu:
        import oracle.grid3 as G3
        q = G3.Problem3(m, n, p, k, edges=d["edges"], alpha=d["alpha"], tau=d["tau"])
        f, _ = G3.prepare_f(d["rho0"].astype("float32").astype("float64"),
                            d["rho1"].astype("float32").astype("float64"), q.edges)
        ci = a.cpu_iters or 8
        r = G3.solve(q, f, ci, 0.0, 1 << 30)
        line["cpu_baseline"] = {"value": cells * ci / r["wall_s"], "unit": "cell-iter/s", "cores": 1, "kind": "oracle",
                                "sample": f"{ci} FP64 iterations of the same {m}x{n}x{p}x{k} grid, single thread, "
                                          f"{r['wall_s']:.1f} s"}
    return line


def main():
    a = _parse()
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    if a.workload != "large":
        if a.gpus != 1:
            print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus})", file=sys.stderr)
            sys.exit(2)
        fn = {"batched": bench_batched, "rgb": bench_rgb, "loss": bench_loss, "matrix": bench_matrix,
              "volume": bench_volume}[a.workload]
        print(json.dumps(fn(a)), flush=True)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for --gpus {a.gpus})",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_1712_10279_amd import inputs as I
    from paper_1712_10279_amd import omt

    d = I.path8_1024(m=a.size, n=a.size)
    if a.tau > 0:
        d["tau"] = a.tau
    iters = a.iters or d["iters"]
    m, n, k = d["rho0"].shape
    l = len(d["edges"])
    dev = torch.device("cuda:0")
    r0 = torch.as_tensor(d["rho0"], dtype=torch.float32, device=dev)
    r1 = torch.as_tensor(d["rho1"], dtype=torch.float32, device=dev)
    T, rows = a.tblock, a.rows
    if T == 0 and rows == 0:
        # launch shape (iterations per HBM pass, rows per wave) from the
        # library's autotuner, untimed; every shape gives the same iterates
        # bit for bit
        s = omt.Solver(r0, r1, d["edges"], alpha=d["alpha"], tau=d["tau"])
        T, rows, _ = s.autotune()
        del s
    T = T if T > 0 else 1

    def one_solve():
        """One step: the whole path once -- set-up (mass check, source term,
        zero state), the iterations with their checks, then the distance
        and the gradient potential."""
        s = omt.Solver(r0, r1, d["edges"], alpha=d["alpha"], tau=d["tau"], tblock=T, rows_per_wave=rows)
        info = s.solve(iters, 0.0, 64)
        V, _ = s.distance()
        g0, _ = s.grad()
        return s, info, V, g0

    for _ in range(a.warmup):
        one_solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s, info, V, g0 = one_solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cells = m * n
    value = cells * iters * a.steps / dt

    # activity of the final iterate: where the shrinks returned non-zero
    act = _activity(s)

    # dominant kernel: the fused step, timed with HIP events on its own
    # stream, from a seeded state with u and w active
    launches = max(1, a.timing_launches // T) * T
    us, timed_act = _timed_from_active_state(s, d["edges"], d["alpha"], d["tau"], T, rows, launches)
    alg_bytes = (7 * k + 2 * l) * 4 * cells * T
    achieved = alg_bytes / (us * 1e-6) / 1e9
    traffic = _traffic(f"T{T}_n{a.size}", rows)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": f"pdhg_step_kernel (T = {T} iterations per launch)", "us_per_launch": us,
            "bytes_per_launch": alg_bytes, "timed_from": "seeded active state (inputs.warm_state)", **timed_act}
    if traffic:
        # what the memory system moved (counted bytes) at the same launch time
        roof["counted_gbs"] = traffic / (us * 1e-6) / 1e9
        roof["counted_frac"] = roof["counted_gbs"] / HBM_PEAK_GBS

    # error of this FP32 run against an FP64 run of the same problem (the
    # FP64 path follows the oracle element by element in the tests)
    fp64 = None
    if not a.no_fp64_check:
        s64 = omt.Solver(r0.double(), r1.double(), d["edges"], alpha=d["alpha"], tau=d["tau"])
        s64.solve(iters, 0.0, 64)
        V64, _ = s64.distance()
        g64, _ = s64.grad()
        fp64 = {"rel_V": abs(V - V64) / V64 if V64 else abs(V), "max_abs_Phi": float((g0.double() - g64).abs().max()),
                "max_abs_Phi_fp64": float(g64.abs().max()), "V_fp64": V64}
        del s64

    line = {
        "metric": "PDHG cell-iterations/s",
        "value": value,
        "unit": "cell-iter/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt * 1e3 / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": d["name"], "grid": [m, n], "channels": k, "edges": l, "graph": "path",
                   "alpha": d["alpha"], "tau": d["tau"], "iterations_per_step": iters, "check_every": 64,
                   "step": "one whole solve: set-up, iterations with checks, distance and gradient",
                   "tblock": T, "rows_per_wave": rows, "parallelism": "single-gpu"},
        "roofline": roof,
        "pixel_channel_iter_per_s": value * k,
        "solve": {"primal": V, "residual": info["residual"], "rel_gap": info["rel_gap"],
                  "mass_residual": info["mass_residual"], **act},
        "fp32_vs_fp64": fp64,
    }
    if not a.no_cpu:
        cpu_iters = a.cpu_iters or max(2, int(60 * (1024 * 1024 * 8) / (cells * k)))
        line["cpu_baseline"] = cpu_baseline(d, cpu_iters)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
