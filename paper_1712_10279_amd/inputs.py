"""Seeded synthetic workloads for the vector-OMT solver.

This module holds no arithmetic of the transport method: it only draws the
input densities (cell masses, App. A) and names the channel graphs and
parameters of each workload.  Both the HIP path and the oracle are fed from
here, so it imports nothing else from this package.

The paper's own inputs (colour images of Sec. 8.1) are not available; smooth
Gaussian-mixture fields of the same kind stand in for them:

* for every channel ``c`` and bump ``b``: centre uniform over the grid,
  width ``sigma`` uniform in ``[sig_lo, sig_hi]`` pixels, amplitude uniform in
  ``[0.5, 1.5]``; the channel is the sum of its bumps plus a constant floor;
* the whole density is rescaled to unit total mass (Sec. 3.2), or, when
  ``channel_mass`` is given, channel ``c`` is rescaled to carry
  ``channel_mass[c] / sum(channel_mass)``;
* the generator is numpy's PCG64 seeded by ``SeedSequence([cfg, pair, side])``
  with ``side`` 0 for rho0 and 1 for rho1.
"""
from __future__ import annotations

import numpy as np

TRIANGLE = np.array([[0, 1], [0, 2], [1, 2]], dtype=np.int32)


def path_edges(k: int) -> np.ndarray:
    """Edges (c, c+1) of the path graph on k channels."""
    return np.array([[c, c + 1] for c in range(k - 1)], dtype=np.int32).reshape(-1, 2)


def complete_edges(k: int) -> np.ndarray:
    """All pairs a < b in lexicographic order (the triangle for k = 3)."""
    return np.array([[a, b] for a in range(k) for b in range(a + 1, k)], dtype=np.int32).reshape(-1, 2)


def default_tau(m: int, n: int) -> float:
    """Dual step used for a grid: 1 up to side 64, 3 above (the values the
    paper tuned for its V-OMT grids, Table 'vecgrid1')."""
    return 1.0 if max(m, n) <= 64 else 3.0


def tuned_tau(m: int, n: int) -> float:
    """Dual step for the time-to-tolerance workloads (the paper tunes tau for
    the fastest convergence): grows with the grid side because the cell
    masses, and so the per-iteration dual increments, shrink with the grid."""
    return max(1.0, max(m, n) / 8.0)


def gaussian_mixture(m: int, n: int, k: int, bumps: int, sig_lo: float, sig_hi: float,
                     floor: float, rng: np.random.Generator, channel_mass=None) -> np.ndarray:
    """(m, n, k) float64 cell masses, unit total mass."""
    ii = np.arange(m, dtype=np.float64)
    jj = np.arange(n, dtype=np.float64)
    out = np.zeros((m, n, k), dtype=np.float64)
    for c in range(k):
        acc = np.full((m, n), floor, dtype=np.float64)
        for _ in range(bumps):
            x0 = rng.uniform(0.0, m)
            y0 = rng.uniform(0.0, n)
            sig = rng.uniform(sig_lo, sig_hi)
            amp = rng.uniform(0.5, 1.5)
            gi = np.exp(-((ii - x0) ** 2) / (2.0 * sig * sig))
            gj = np.exp(-((jj - y0) ** 2) / (2.0 * sig * sig))
            acc += amp * np.outer(gi, gj)
        out[:, :, c] = acc
    if channel_mass is None:
        out /= out.sum()
    else:
        cm = np.asarray(channel_mass, dtype=np.float64)
        cm = cm / cm.sum()
        for c in range(k):
            out[:, :, c] *= cm[c] / out[:, :, c].sum()
    return out


def pair(cfg: int, pair_id: int, m: int, n: int, k: int, bumps: int, sig_lo: float, sig_hi: float,
         floor: float, channel_mass0=None, channel_mass1=None):
    """(rho0, rho1) for one workload pair, drawn as described above."""
    r0 = np.random.default_rng(np.random.SeedSequence([cfg, pair_id, 0]))
    r1 = np.random.default_rng(np.random.SeedSequence([cfg, pair_id, 1]))
    rho0 = gaussian_mixture(m, n, k, bumps, sig_lo, sig_hi, floor, r0, channel_mass0)
    rho1 = gaussian_mixture(m, n, k, bumps, sig_lo, sig_hi, floor, r1, channel_mass1)
    return rho0, rho1


# ------------------------------------------------------------- workloads

def small_fp64(pair_id: int = 0, m: int = 32, n: int = 32):
    """32x32, k=3 triangle, alpha 1, FP64, 4 bumps per channel with sigma in
    [2, 6] px and no floor; 10,000 iterations."""
    rho0, rho1 = pair(1, pair_id, m, n, 3, 4, 2.0, 6.0, 0.0)
    return dict(name=f"vomt_{m}x{n}_k3_triangle_fp64", rho0=rho0, rho1=rho1, edges=TRIANGLE,
                alpha=1.0, tau=default_tau(m, n), iters=10000, dtype="f64")


def rgb_256(alpha: float = 1.0, pair_id: int = None, m: int = 256, n: int = 256):
    """256x256, k=3 triangle, 8 bumps per channel, sigma in [8, 32] px, floor
    1e-3; one pair per alpha in {0.5, 1, 4}; solved to 1e-5 residual."""
    if pair_id is None:
        pair_id = {0.5: 0, 1.0: 1, 4.0: 2}.get(float(alpha), 0)
    rho0, rho1 = pair(2, pair_id, m, n, 3, 8, 8.0 * m / 256, 32.0 * m / 256, 1e-3)
    return dict(name=f"vomt_{m}x{n}_k3_triangle_a{alpha:g}", rho0=rho0, rho1=rho1, edges=TRIANGLE,
                alpha=float(alpha), tau=default_tau(m, n), tol=1e-5, dtype="f32")


def path8_1024(m: int = 1024, n: int = 1024, k: int = 8):
    """1024x1024, k=8 path graph (7 edges), alpha 1, 16 bumps per channel,
    sigma in [16, 64] px, floor 1e-3.  rho0 puts mass proportional to c+1 in
    channel c and rho1 mass proportional to k-c, so the transfer w between
    channels is active; 20,000 iterations."""
    s = m / 1024.0
    rho0, rho1 = pair(3, 0, m, n, k, 16, max(16.0 * s, 1.0), max(64.0 * s, 2.0), 1e-3,
                      channel_mass0=[c + 1 for c in range(k)],
                      channel_mass1=[k - c for c in range(k)])
    return dict(name=f"vomt_{m}x{n}_k{k}_path", rho0=rho0, rho1=rho1, edges=path_edges(k),
                alpha=1.0, tau=default_tau(m, n), iters=20000, dtype="f32")


BATCH_SIDES = (64, 128, 192, 256, 384, 512)


def batch_spec(n_pairs: int = 96, sides=BATCH_SIDES):
    """Shapes and parameters of the batched workload: side uniform over
    ``sides``, k uniform over {1, 3} (triangle for 3), alpha uniform in
    [0.5, 4]."""
    specs = []
    for p in range(n_pairs):
        rng = np.random.default_rng(np.random.SeedSequence([4, p, 2]))
        side = int(rng.choice(sides))
        k = int(rng.choice([1, 3]))
        alpha = float(rng.uniform(0.5, 4.0))
        specs.append(dict(pair=p, side=side, k=k, alpha=alpha))
    return specs


def batch_pair(spec):
    """(rho0, rho1, edges, alpha, tau) of one batched pair: 8 bumps with sigma
    in [side/32, side/8], floor 1e-3."""
    side, k = spec["side"], spec["k"]
    rho0, rho1 = pair(4, spec["pair"], side, side, k, 8, side / 32.0, side / 8.0, 1e-3)
    edges = TRIANGLE if k == 3 else np.zeros((0, 2), np.int32)
    return dict(name=f"batch{spec['pair']}_{side}_k{k}", rho0=rho0, rho1=rho1, edges=edges,
                alpha=spec["alpha"], tau=default_tau(side, side), tol=1e-5, dtype="f32")


def loss_512(pair_id: int, m: int = 512, n: int = 512):
    """512x512, k=3 triangle, alpha 1 pair for the differentiable loss (8 per
    batch), 8 bumps, sigma in [16, 64] px, floor 1e-3; solved to 1e-6 with
    tau = 2 x side (fastest to 1e-6 in a sweep at 512x512)."""
    s = m / 512.0
    rho0, rho1 = pair(5, pair_id, m, n, 3, 8, 16.0 * s, 64.0 * s, 1e-3)
    return dict(name=f"loss_{m}x{n}_k3_{pair_id}", rho0=rho0, rho1=rho1, edges=TRIANGLE,
                alpha=1.0, tau=2.0 * max(m, n), tol=1e-6, dtype="f32")


def random_pair(seed: int, m: int, n: int, k: int, bumps: int = 3, floor: float = 1e-3):
    """Small generic pair for tests (cfg id 100)."""
    lo = max(1.0, min(m, n) / 12.0)
    hi = max(2.0, min(m, n) / 4.0)
    return pair(100, seed, m, n, k, bumps, lo, hi, floor)


# ------------------------------------------------------------- matrix method
#
# The paper's diffusion-tensor densities (Sec. 8.2) are not available.
# Stand-ins of the same kind: every pixel carries a positive semidefinite
# k x k matrix, the sum of a few Gaussian bumps, each bump with its own
# "ellipsoid" (a random positive definite matrix of unit trace: Q diag(d) Q^*
# with Q from the QR factorisation of a Gaussian matrix, real or complex,
# and d uniform in [0.1, 1] normalised), plus floor * I; the whole field has
# unit total trace (Sec. 4.2).

# the two 3 x 3 matrices of the diffusion-tensor example (Sec. 8.2)
L_DTI = np.array([[[1, 0, 0], [0, 2, 0], [0, 0, 0]], [[1, 1, 1], [1, 0, 0], [1, 0, 0]]], dtype=np.float64)
# a pair of Hermitian 2 x 2 matrices whose commutant is the multiples of I
L_PAULI_XZ = np.array([[[0, 1], [1, 0]], [[1, 0], [0, -1]]], dtype=np.complex128)


def _ellipsoid(rng, k, real):
    X = rng.normal(size=(k, k)) + (0 if real else 1j * rng.normal(size=(k, k)))
    Q, _ = np.linalg.qr(X)
    d = rng.uniform(0.1, 1.0, size=k)
    d /= d.sum()
    return (Q * d) @ Q.conj().T


def matrix_field(rng, m, n, k, bumps, sig_lo, sig_hi, real, floor=1e-3, centres=None, shapes=None):
    ii, jj = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    out = np.zeros((m, n, k, k), dtype=np.complex128)
    for b in range(bumps):
        ci, cj = centres[b] if centres is not None else (rng.uniform(0, m - 1), rng.uniform(0, n - 1))
        sig = rng.uniform(sig_lo, sig_hi)
        amp = rng.uniform(0.5, 1.5)
        A = shapes[b] if shapes is not None else _ellipsoid(rng, k, real)
        g = amp * np.exp(-((ii - ci) ** 2 + (jj - cj) ** 2) / (2.0 * sig * sig))
        out += g[:, :, None, None] * A
    out += floor * np.eye(k)
    out /= np.trace(out.sum((0, 1))).real
    return out.real.copy() if real else out


def matrix_pair(seed, m, n, k, real, bumps=3, floor=1e-3):
    """Two independent unit-trace matrix fields (small parity cases)."""
    r0 = np.random.default_rng(np.random.SeedSequence([7, seed, 0]))
    r1 = np.random.default_rng(np.random.SeedSequence([7, seed, 1]))
    s = max(m, n)
    return (matrix_field(r0, m, n, k, bumps, s / 12, s / 5, real, floor),
            matrix_field(r1, m, n, k, bumps, s / 12, s / 5, real, floor))


def dti_like(side=128, seed=0, bumps=6):
    """Three real 3 x 3 fields in the manner of the paper's Lambda0, Lambda1,
    Lambda2: Lambda1 has Lambda0's bump centres and widths with other
    ellipsoids; Lambda2 has Lambda0's ellipsoids at other centres."""
    rng = np.random.default_rng(np.random.SeedSequence([8, seed, side]))
    cen0 = [(rng.uniform(side * 0.2, side * 0.8), rng.uniform(side * 0.2, side * 0.8)) for _ in range(bumps)]
    cen2 = [(rng.uniform(side * 0.2, side * 0.8), rng.uniform(side * 0.2, side * 0.8)) for _ in range(bumps)]
    sh0 = [_ellipsoid(rng, 3, True) for _ in range(bumps)]
    sh1 = [_ellipsoid(rng, 3, True) for _ in range(bumps)]
    state = rng.bit_generator.state

    def field(cen, sh):
        r = np.random.default_rng()
        r.bit_generator.state = state  # same widths and amplitudes for all three
        return matrix_field(r, side, side, 3, bumps, side / 32, side / 12, True, 1e-3, centres=cen, shapes=sh)

    return {"lam0": field(cen0, sh0), "lam1": field(cen0, sh1), "lam2": field(cen2, sh0), "L": L_DTI}


# ------------------------------------------------------------- warm starts

def warm_state(seed: int, m: int, n: int, k: int, l: int, u_scale: float, w_scale: float,
               offset: float, slope: float = 2.5, period: float = 32.0):
    """A seeded synthetic iterate (phi, u, w) in the caller's layout (phi
    m x n x k, u m x n x k x 2, w m x n x l), for starting both sides from a
    state in which the shrinks are active.

    Channel c of phi is ``a_c sin(2 pi (i cos t_c + j sin t_c) / period +
    p_c) + (-1)^c offset / 2`` with the amplitude a_c chosen so that the
    per-pixel slope (in units of the grid spacing h = 1/(max(m,n)-1)) is
    ``slope`` times a factor uniform in [0.5, 1.5]: slopes above 1 make
    the flux shrink return non-zero values, and neighbouring channels apart
    by more than alpha make the transfer shrink do so.  u and w are uniform
    in [-u_scale, u_scale] and [-w_scale, w_scale]."""
    rng = np.random.default_rng(np.random.SeedSequence([200, seed, m, n, k]))
    h = 1.0 / (max(m, n) - 1)
    ii = np.arange(m, dtype=np.float64)[:, None]
    jj = np.arange(n, dtype=np.float64)[None, :]
    phi = np.zeros((m, n, k))
    for c in range(k):
        t = rng.uniform(0.0, 2.0 * np.pi)
        p = rng.uniform(0.0, 2.0 * np.pi)
        s = slope * rng.uniform(0.5, 1.5)
        amp = s * h * period / (2.0 * np.pi)
        phi[:, :, c] = amp * np.sin(2.0 * np.pi * (ii * np.cos(t) + jj * np.sin(t)) / period + p) \
            + (0.5 if c % 2 == 0 else -0.5) * offset
    u = rng.uniform(-u_scale, u_scale, size=(m, n, k, 2))
    w = rng.uniform(-w_scale, w_scale, size=(m, n, l))
    return phi, u, w


# ------------------------------------------------------------- 3-D grids
#
# The same generator on an m x n x p grid (centres uniform over the volume,
# isotropic 3-D Gaussian bumps): there are no 3-D images in the paper, whose
# Sec. 8.2 names 3-D imaging as future work.

def gaussian_mixture3(m: int, n: int, p: int, k: int, bumps: int, sig_lo: float, sig_hi: float, floor: float,
                      rng: np.random.Generator, channel_mass=None) -> np.ndarray:
    """(m, n, p, k) float64 cell masses, unit total mass (or the given
    split over the channels)."""
    ii = np.arange(m, dtype=np.float64)
    jj = np.arange(n, dtype=np.float64)
    zz = np.arange(p, dtype=np.float64)
    out = np.zeros((m, n, p, k), dtype=np.float64)
    for c in range(k):
        acc = np.full((m, n, p), floor, dtype=np.float64)
        for _ in range(bumps):
            x0, y0, z0 = rng.uniform(0.0, m), rng.uniform(0.0, n), rng.uniform(0.0, p)
            sig = rng.uniform(sig_lo, sig_hi)
            amp = rng.uniform(0.5, 1.5)
            gi = np.exp(-((ii - x0) ** 2) / (2.0 * sig * sig))
            gj = np.exp(-((jj - y0) ** 2) / (2.0 * sig * sig))
            gz = np.exp(-((zz - z0) ** 2) / (2.0 * sig * sig))
            acc += amp * gi[:, None, None] * gj[None, :, None] * gz[None, None, :]
        out[..., c] = acc
    if channel_mass is None:
        out /= out.sum()
    else:
        cm = np.asarray(channel_mass, dtype=np.float64)
        cm = cm / cm.sum()
        for c in range(k):
            out[..., c] *= cm[c] / out[..., c].sum()
    return out


def pair3(cfg: int, pair_id: int, m: int, n: int, p: int, k: int, bumps: int, sig_lo: float, sig_hi: float,
          floor: float, channel_mass0=None, channel_mass1=None):
    """(rho0, rho1) of a 3-D workload pair, seeded like ``pair``."""
    r0 = np.random.default_rng(np.random.SeedSequence([cfg, pair_id, 0, p]))
    r1 = np.random.default_rng(np.random.SeedSequence([cfg, pair_id, 1, p]))
    rho0 = gaussian_mixture3(m, n, p, k, bumps, sig_lo, sig_hi, floor, r0, channel_mass0)
    rho1 = gaussian_mixture3(m, n, p, k, bumps, sig_lo, sig_hi, floor, r1, channel_mass1)
    return rho0, rho1


def random_volume_pair(seed: int, m: int, n: int, p: int, k: int, bumps: int = 3, floor: float = 1e-3):
    """Small generic 3-D pair for tests (cfg id 101)."""
    lo = max(1.0, min(m, n, p) / 12.0)
    hi = max(2.0, min(m, n, p) / 4.0)
    return pair3(101, seed, m, n, p, k, bumps, lo, hi, floor)


def warm_state3(seed: int, m: int, n: int, p: int, k: int, l: int, u_scale: float, w_scale: float,
                offset: float, slope: float = 2.5, period: float = 32.0):
    """``warm_state`` on an m x n x p grid: phi (m, n, p, k) plane waves
    along a random 3-D direction per channel with per-cell slope ``slope``
    times a factor uniform in [0.5, 1.5] (in units of h = 1/(max(m,n,p)-1)),
    channels alternately offset by +-offset/2; u (m, n, p, k, 3) and w
    (m, n, p, l) uniform in [-u_scale, u_scale] and [-w_scale, w_scale]."""
    rng = np.random.default_rng(np.random.SeedSequence([201, seed, m, n, p, k]))
    h = 1.0 / (max(m, n, p) - 1)
    ii = np.arange(m, dtype=np.float64)[:, None, None]
    jj = np.arange(n, dtype=np.float64)[None, :, None]
    zz = np.arange(p, dtype=np.float64)[None, None, :]
    phi = np.zeros((m, n, p, k))
    for c in range(k):
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        s = slope * rng.uniform(0.5, 1.5)
        amp = s * h * period / (2.0 * np.pi)
        phi[..., c] = amp * np.sin(2.0 * np.pi * (ii * v[0] + jj * v[1] + zz * v[2]) / period + ph) \
            + (0.5 if c % 2 == 0 else -0.5) * offset
    u = rng.uniform(-u_scale, u_scale, size=(m, n, p, k, 3))
    w = rng.uniform(-w_scale, w_scale, size=(m, n, p, l))
    return phi, u, w


def volume_256(m: int = 256, n: int = 256, p: int = 128, k: int = 3):
    """3-D workload: 256 x 256 x 128 cells, k = 3 triangle, alpha 0.1, 16
    bumps per channel with sigma in [8, 32] cells, floor 1e-3, unit mass,
    2,000 iterations; the 8.4-million-cell volume is the size of the 2-D
    large workload's 1024 x 1024 x 8 pixel-channels.  tau = 4 x side = 1024:
    the 3-D cell masses are small, so with smaller tau the 2,000 iterations
    end before any flux or transfer shrink returns non-zero (tau 32: none;
    tau 1024: u non-zero on 91 % of cells and w on 54 %)."""
    s = min(m, n, p) / 128.0
    rho0, rho1 = pair3(6, 0, m, n, p, k, 16, max(8.0 * s, 1.0), max(32.0 * s, 2.0), 1e-3)
    return dict(name=f"vomt3_{m}x{n}x{p}_k{k}_triangle", rho0=rho0, rho1=rho1, edges=TRIANGLE, alpha=0.1,
                tau=4.0 * max(m, n, p), iters=2000, dtype="f32")
