"""Pins of the matrix-OMT oracle (Sec. 4, Sec. 7.3, App. B) to facts other
than itself: operator identities of Sec. 4.1, the spectrum of -Delta_L from
an independent superoperator, the reduction of diagonal problems to the
vector method (itself pinned by exact LPs and closed forms), unitary
covariance, transport of one fixed matrix shape, per-pixel optima in closed
form or by LP, and the prox conditions of the shrinks."""
import numpy as np
import pytest

import oracle
import oracle.matrix as M

rng = np.random.default_rng(20171227)

PAULI_X = np.array([[[0, 1], [1, 0]]], float)
# the two 3 x 3 matrices of the diffusion-tensor example (Sec. 8.2)
L_DTI = np.array([[[1, 0, 0], [0, 2, 0], [0, 0, 0]], [[1, 1, 1], [1, 0, 0], [1, 0, 0]]], float)


def herm(k, real=False):
    A = rng.normal(size=(k, k)) + (0 if real else 1j * rng.normal(size=(k, k)))
    return (A + A.conj().T) / 2


def skew(k, real=False):
    A = rng.normal(size=(k, k)) + (0 if real else 1j * rng.normal(size=(k, k)))
    return (A - A.conj().T) / 2


def hs(A, B):
    return float(np.real(np.sum(A * B.conj())))


def unitary(k):
    Q, R = np.linalg.qr(rng.normal(size=(k, k)) + 1j * rng.normal(size=(k, k)))
    return Q * (np.diag(R) / abs(np.diag(R)))


# ------------------------------------------------------------- operators

@pytest.mark.parametrize("k,l", [(2, 1), (3, 2), (4, 3)])
def test_quantum_gradient_identities(k, l):
    L = np.stack([herm(k) for _ in range(l)])
    X, Z = herm(k), np.stack([skew(k) for _ in range(l)])
    g, d = M.grad_L(L, X), M.div_L(L, Z)
    # div_L = -grad_L^* in the Hilbert-Schmidt inner product (Sec. 4.1)
    assert hs(g, Z) == pytest.approx(-hs(X, d), rel=1e-12, abs=1e-12)
    # grad_L maps H to skew-Hermitian matrices, div_L maps S^l to H
    assert np.allclose(g, -np.conj(np.swapaxes(g, -1, -2)), atol=1e-13)
    assert np.allclose(d, d.conj().T, atol=1e-13)
    # div_L ranges in the trace-free matrices; grad_L kills the identity
    assert abs(np.trace(d)) < 1e-12
    assert np.abs(M.grad_L(L, np.eye(k))).max() < 1e-13
    # the commutator written out with numpy
    assert np.allclose(g, np.stack([Ls @ X - X @ Ls for Ls in L]), atol=1e-13)


def _superop_lmax(L):
    """lambda_max of sum_s ad_{L_s}^2 on C^{k x k} (row-major vec), which
    equals lambda_max(-Delta_L) on H: ad is complex-linear and maps H to iS."""
    k = L.shape[1]
    T = 0
    for Ls in L:
        A = np.kron(Ls, np.eye(k)) - np.kron(np.eye(k), Ls.T)
        T = T + A.conj().T @ A
    return float(np.linalg.eigvalsh(T).max())


@pytest.mark.parametrize("case", ["pauli", "dti", "rand3", "rand4real"])
def test_lambda_max_of_minus_laplacian(case):
    L = {"pauli": PAULI_X, "dti": L_DTI, "rand3": np.stack([herm(3), herm(3)]),
         "rand4real": np.stack([herm(4, True) for _ in range(3)])}[case]
    assert M.lambda_max(L) == pytest.approx(_superop_lmax(L), rel=1e-12)
    if case == "pauli":
        # ad_L has eigenvalues l_a - l_b = 0, 0, +-2 for L = sigma_x
        assert M.lambda_max(L) == pytest.approx(4.0, rel=1e-14)


def test_standing_assumption_holds_for_the_example_matrices():
    # ker grad_L = span(I) (Sec. 4.1) for the two matrices of the DTI example:
    # exactly one zero eigenvalue of sum ad^2.  A single sigma_x also
    # commutes with itself, so its kernel is span(I, sigma_x); the diagonal
    # problems below have no sigma_x component, so nothing changes for them.
    for L, nker in ((L_DTI, 1), (PAULI_X, 2), (np.stack([PAULI_X[0], np.diag([1.0, -1.0])]), 1)):
        k = L.shape[1]
        T = 0
        for Ls in L:
            A = np.kron(Ls, np.eye(k)) - np.kron(np.eye(k), Ls.T)
            T = T + A.conj().T @ A
        ev = np.linalg.eigvalsh(T)
        assert np.sum(ev < 1e-10) == nker


# --------------------------------------------------------------- shrinks

def _svd_shrink(X, t):
    U, s, Vh = np.linalg.svd(X)
    return (U * np.maximum(s - t, 0)) @ Vh


@pytest.mark.parametrize("herm_kind", [True, False])
def test_nuclear_shrink_is_svd_soft_threshold(herm_kind):
    for k in (2, 3, 4):
        X = np.stack([herm(k) if herm_kind else skew(k) for _ in range(2)])
        t = 0.4
        Y = M.shrink_block(M.NUC, herm_kind, X, t)
        for s in range(2):
            assert np.allclose(Y[s], _svd_shrink(X[s], t), atol=1e-12)
            # the result stays Hermitian / skew-Hermitian (App. B lemma)
            sgn = 1 if herm_kind else -1
            assert np.allclose(Y[s], sgn * Y[s].conj().T, atol=1e-12)
        nuc = sum(np.linalg.svd(X[s], compute_uv=False).sum() for s in range(2))
        assert M.norm_block(M.NUC, herm_kind, X) == pytest.approx(nuc, rel=1e-12)


def test_frobenius_and_entrywise_shrinks():
    X = np.stack([herm(3), herm(3)])
    t = 0.7
    r = np.sqrt(np.sum(abs(X) ** 2))
    assert np.allclose(M.shrink_block(M.FRO, True, X, t), X * max(0.0, 1 - t / r), atol=1e-14)
    Y = M.shrink_block(M.L1, True, X, t)
    ref = np.where(abs(X) >= t, X * (1 - t / np.maximum(abs(X), 1e-300)), 0)
    assert np.allclose(Y, ref, atol=1e-14)
    assert M.norm_block(M.FRO, True, X) == pytest.approx(r, rel=1e-14)
    assert M.norm_block(M.L1, True, X) == pytest.approx(np.abs(X).sum(), rel=1e-14)
    # prox optimality of the block shrink: X - Y = t * (unit vector of Y)
    Yf = M.shrink_block(M.FRO, True, X, t)
    assert np.allclose(X - Yf, t * Yf / np.sqrt(np.sum(abs(Yf) ** 2)), atol=1e-13)


# ------------------------------------------------------------- reductions

def _diag_pair(m, n, seed):
    from paper_1712_10279_amd import inputs as I
    r0, r1 = I.random_pair(seed, m, n, 2)
    lam0 = np.zeros((m, n, 2, 2), complex)
    lam1 = np.zeros((m, n, 2, 2), complex)
    for c in range(2):
        lam0[:, :, c, c] = r0[:, :, c]
        lam1[:, :, c, c] = r1[:, :, c]
    return r0, r1, lam0, lam1


@pytest.mark.parametrize("unorm,wnorm,vu,vw,ascale", [
    (M.FRO, M.L1, oracle.U_L2, oracle.W_L1, 1.0),
    (M.L1, M.L1, oracle.U_L1, oracle.W_L1, 1.0),
    (M.NUC, M.NUC, oracle.U_L1, oracle.W_L1, 1.0),
    (M.FRO, M.FRO, oracle.U_L2, oracle.W_L1, 2 ** -0.5),
    (M.L1, M.NUC, oracle.U_L1, oracle.W_L1, 1.0),
])
def test_diagonal_problems_are_vector_omt(unorm, wnorm, vu, vw, ascale):
    """With L = sigma_x and diagonal densities, Phi stays diagonal and the
    method is the two-channel vector method on one edge: W = [[0, w], [-w, 0]]
    carries w_vec = -2 w, div_L W = diag(2w, -2w) = div_G w_vec, and
    lambda_max(-Delta_L) = 4 = 2 lambda_max(-Delta_G) so that nu halves
    exactly as w doubles.  ||W||_1 and ||W||_nuc are |w_vec|, ||W||_2 is
    |w_vec|/sqrt2 (hence alpha/sqrt2 on the vector side)."""
    m, n = 9, 11
    r0, r1, lam0, lam1 = _diag_pair(m, n, 3)
    rm = M.solve_pair(lam0, lam1, PAULI_X, alpha=0.7, tau=2.0, unorm=unorm, wnorm=wnorm, max_iters=300)
    rv = oracle.solve_pair(r0, r1, [(0, 1)], alpha=0.7 * ascale, tau=2.0, unorm=vu, wnorm=vw, max_iters=300)
    ph = rm["state"]["phi"]
    for c in range(2):
        assert np.allclose(ph[:, :, c, c], rv["state"]["phi"][:, :, c], rtol=0, atol=1e-13)
        assert np.allclose(rm["state"]["ux"][:, :, c, c], rv["state"]["ux"][:, :, c], rtol=0, atol=1e-13)
    assert np.abs(ph[:, :, 0, 1]).max() == 0.0
    assert np.allclose(rm["state"]["w"][:, :, 0, 0, 1], -0.5 * rv["state"]["w"][:, :, 0], rtol=0, atol=1e-13)
    assert rm["primal"] == pytest.approx(rv["primal"], rel=1e-12)
    assert rm["residual"] == pytest.approx(rv["residual"], rel=1e-10)


@pytest.mark.parametrize("unorm,wnorm", [(M.FRO, M.FRO), (M.NUC, M.NUC), (M.FRO, M.NUC)])
def test_unitary_covariance(unorm, wnorm):
    """For unitarily invariant norms the method commutes with X -> Q X Q^*
    applied to L and to the data (complex Q): every iterate transforms the
    same way.  Catches transposes and missing conjugations."""
    m, n, k = 6, 7, 3
    L = np.stack([herm(k), herm(k)])
    lam0 = np.zeros((m, n, k, k), complex)
    lam1 = np.zeros((m, n, k, k), complex)
    for i in range(m):
        for j in range(n):
            A = rng.normal(size=(k, k)) + 1j * rng.normal(size=(k, k))
            B = rng.normal(size=(k, k)) + 1j * rng.normal(size=(k, k))
            lam0[i, j] = A @ A.conj().T
            lam1[i, j] = B @ B.conj().T
    lam1 *= np.trace(lam0.sum((0, 1))).real / np.trace(lam1.sum((0, 1))).real
    Q = unitary(k)
    tr = lambda X: Q @ X @ Q.conj().T
    r = M.solve_pair(lam0, lam1, L, alpha=0.9, tau=1.5, unorm=unorm, wnorm=wnorm, max_iters=120)
    rq = M.solve_pair(tr(lam0), tr(lam1), np.stack([tr(x) for x in L]), alpha=0.9, tau=1.5, unorm=unorm,
                      wnorm=wnorm, max_iters=120)
    for key in ("phi", "ux", "uy"):
        assert np.allclose(rq["state"][key], tr(r["state"][key]), atol=1e-11), key
    assert np.allclose(rq["state"]["w"], tr(r["state"]["w"]), atol=1e-11)
    assert rq["primal"] == pytest.approx(r["primal"], rel=1e-11)


@pytest.mark.parametrize("unorm", [M.FRO, M.NUC])
def test_transport_of_one_matrix_shape_is_scalar_omt(unorm):
    """Lambda = A rho with a fixed complex A of unit norm (rank one for the
    nuclear norm) and alpha large enough that W stays zero: every iterate is
    A times the scalar method's iterate, and M equals the scalar distance
    (||u||_2 for the Frobenius norm, ||u||_1 for the nuclear norm)."""
    from paper_1712_10279_amd import inputs as I
    m, n, k = 10, 8, 3
    r0, r1 = I.random_pair(11, m, n, 1)
    if unorm == M.NUC:
        q = rng.normal(size=k) + 1j * rng.normal(size=k)
        q /= np.linalg.norm(q)
        A = np.outer(q, q.conj())
    else:
        A = herm(k)
        A /= np.sqrt(np.sum(abs(A) ** 2))
    lam0 = r0[:, :, 0, None, None] * A
    lam1 = r1[:, :, 0, None, None] * A
    L = np.stack([herm(k), herm(k)])
    rm = M.solve_pair(lam0, lam1, L, alpha=1e4, tau=1.0, unorm=unorm, wnorm=M.L1, max_iters=200)
    p = M.MProblem(m, n, L, tau=1.0)
    rv = oracle.solve_pair(r0, r1, np.zeros((0, 2), int), tau=1.0, unorm=oracle.U_L2 if unorm == M.FRO else oracle.U_L1,
                           max_iters=200, mu=p.mu)
    assert np.abs(rm["state"]["w"]).max() == 0.0
    assert np.allclose(rm["state"]["phi"], rv["state"]["phi"][:, :, 0, None, None] * A, atol=1e-12)
    assert rm["primal"] == pytest.approx(rv["primal"], rel=1e-11)


def _coord_basis_skew(k, real):
    """Orthonormal real basis of the skew-Hermitian k x k matrices."""
    out = []
    if not real:
        for a in range(k):
            E = np.zeros((k, k), complex)
            E[a, a] = 1j
            out.append(E)
    for a in range(k):
        for b in range(a + 1, k):
            E = np.zeros((k, k), complex)
            E[a, b], E[b, a] = 2 ** -0.5, -2 ** -0.5
            out.append(E)
            if not real:
                E = np.zeros((k, k), complex)
                E[a, b] = E[b, a] = 1j * 2 ** -0.5
                out.append(E)
    return out


def _uniform(k, L, seed):
    r = np.random.default_rng(seed)
    A = r.normal(size=(k, k))
    B = r.normal(size=(k, k))
    A, B = A @ A.T + 0.1 * np.eye(k), B @ B.T + 0.1 * np.eye(k)
    B *= np.trace(A) / np.trace(B)
    return A, B


@pytest.mark.parametrize("wnorm", [M.FRO, M.L1])
def test_same_difference_at_every_pixel_is_a_per_pixel_problem(wnorm):
    """Lambda0 - Lambda1 = D at every pixel: averaging any feasible W over the
    grid (the zero-flux divergence sums to zero) shows U = 0 and a constant W
    are optimal, so M = alpha * (number of pixels) * min{||W||_w : div_L W = D}.
    The per-pixel minimum: least-norm solution (Frobenius) or an exact LP
    (entry-wise, real data)."""
    from scipy.optimize import linprog
    k, m, n, alpha = 3, 3, 4, 0.8
    L = L_DTI
    A, B = _uniform(k, L, 5)
    D = A - B
    lam0 = np.broadcast_to(A, (m, n, k, k)).astype(complex)
    lam1 = np.broadcast_to(B, (m, n, k, k)).astype(complex)
    # the per-pixel problem in real coordinates (real skew W_s, real symmetric D)
    basis = [(s, E) for s in range(L.shape[0]) for E in _coord_basis_skew(k, real=True)]
    rows = [(a, b) for a in range(k) for b in range(a, k)]
    Amat = np.zeros((len(rows), len(basis)))
    for c, (s, E) in enumerate(basis):
        Z = np.zeros((L.shape[0], k, k), complex)
        Z[s] = E
        dv = (-(L @ Z) + Z @ L).sum(0)
        for r_, (a, b) in enumerate(rows):
            Amat[r_, c] = dv[a, b].real
    d = np.array([D[a, b] for a, b in rows])
    if wnorm == M.FRO:
        x = np.linalg.lstsq(Amat, d, rcond=None)[0]
        assert np.allclose(Amat @ x, d, atol=1e-12)
        per = np.linalg.norm(x)
    else:
        # ||W||_1 = sum over entries = 2 sum_{a<b} |W_ab| = sqrt2 sum |x_c|
        nb = len(basis)
        res = linprog(np.full(2 * nb, np.sqrt(2)), A_eq=np.hstack([Amat, -Amat]), b_eq=d, bounds=(0, None),
                      method="highs")
        assert res.status == 0
        per = res.fun
    expect = alpha * m * n * per
    r = M.solve_pair(lam0, lam1, L, alpha=alpha, tau=1.0, unorm=M.FRO, wnorm=wnorm, max_iters=200000, tol=1e-9)
    assert r["converged"]
    assert r["primal"] == pytest.approx(expect, rel=1e-6)
    assert r["dual"] == pytest.approx(expect, rel=1e-6)


# ------------------------------------------------------------- invariants

def test_first_step_residual_and_conserved_trace():
    m, n, k = 7, 5, 3
    L = L_DTI
    lam0 = np.zeros((m, n, k, k), complex)
    lam1 = np.zeros((m, n, k, k), complex)
    for i in range(m):
        for j in range(n):
            A, B = rng.normal(size=(k, k)), rng.normal(size=(k, k))
            lam0[i, j], lam1[i, j] = A @ A.T, B @ B.T
    lam1 *= np.trace(lam0.sum((0, 1))) / np.trace(lam1.sum((0, 1)))
    f, imb = M.prepare_f(lam0, lam1)
    assert imb < 1e-14 and abs(np.trace(f.sum((0, 1)))) < 1e-12
    # unequal trace mass: reported, and removed from f as a multiple of I
    fu, imbu = M.prepare_f(lam0, 1.25 * lam1)
    assert imbu == pytest.approx(0.25 / 1.25, rel=1e-12)
    assert abs(np.trace(fu.sum((0, 1)))) < 1e-10
    assert np.allclose(fu - f, 0.25 * lam1 - (0.25 * np.trace(lam1.sum((0, 1))) / (m * n * k)) * np.eye(k),
                       atol=1e-12)
    p = M.MProblem(m, n, L, tau=2.0)
    r1 = M.solve(p, f, 1)
    # from zero: U1 = 0, W1 = 0, Phi1 = tau f, so R^1 = tau ||f||^2 (Sec. 6.1)
    assert r1["residual"] == pytest.approx(1.0, rel=1e-13)
    assert np.allclose(r1["state"]["phi"], 2.0 * f, atol=1e-15)
    r = M.solve(p, f, 400, check_every=20)
    # the trace of Phi summed over the grid never moves (both divergences
    # have zero total trace and f has none)
    assert abs(np.trace(r["state"]["phi"].sum((0, 1)))) < 1e-10
    # real data stays real, exactly
    assert np.abs(r["state"]["phi"].imag).max() == 0.0
    # the PDHG fixed-point residual is nonincreasing
    h = r["hist"]
    assert np.all(np.diff(h) <= 1e-12 * h[:-1])


def test_symmetry_and_zero_distance():
    m, n, k = 5, 6, 2
    L = np.stack([herm(k)])
    lam0 = np.zeros((m, n, k, k), complex)
    lam1 = np.zeros((m, n, k, k), complex)
    for i in range(m):
        for j in range(n):
            A = rng.normal(size=(k, k)) + 1j * rng.normal(size=(k, k))
            B = rng.normal(size=(k, k)) + 1j * rng.normal(size=(k, k))
            lam0[i, j], lam1[i, j] = A @ A.conj().T, B @ B.conj().T
    lam1 *= np.trace(lam0.sum((0, 1))).real / np.trace(lam1.sum((0, 1))).real
    a = M.solve_pair(lam0, lam1, L, max_iters=150)
    b = M.solve_pair(lam1, lam0, L, max_iters=150)
    # swapping the densities flips every iterate's sign
    assert np.allclose(b["state"]["phi"], -a["state"]["phi"], atol=1e-13)
    assert b["primal"] == pytest.approx(a["primal"], rel=1e-13)
    z = M.solve_pair(lam0, lam0, L, max_iters=20)
    assert z["primal"] == 0.0
