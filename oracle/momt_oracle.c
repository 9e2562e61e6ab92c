/*
 * Oracle for the matrix optimal mass transport (M-OMT) first-order method of
 * Ryu, Chen, Li and Osher, "Vector and Matrix Optimal Mass Transport:
 * Theory, Algorithm, and Applications" (arXiv 1712.10279).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * FP64 single-threaded reference that the HIP path is checked against.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no code, header, table or constant with the HIP path.
 * It works on whole complex k x k matrices, exactly as the method is stated,
 * with no change of coordinates.
 *
 * Every routine follows one passage of the paper:
 *   - quantum gradient grad_L X = (L_s X - X L_s)_s and divergence
 *     div_L Z = sum_s (-L_s Z_s + Z_s L_s)                         Sec. 4.1
 *   - Hilbert-Schmidt inner product <X, Y> = Re tr(X Y^*)            Sec. 4
 *   - spatial divergence applied entry by entry                       Sec. 4.2
 *     (with the staggered grid and ghost cells of the vector case)   App. A
 *   - norms ||.||_2, ||.||_1, ||.||_{1,nuc} on H^d and S^l            Sec. 6.2
 *   - shrinks: complex soft threshold, Frobenius block shrink, nuclear
 *     shrink; their Hermitian / skew-Hermitian results (lemma)        App. B
 *   - the M-OMT first-order method, its step-size rule and
 *     lambda_max(-Delta_L) from the k^2 x k^2 matrix of -Delta_L      Sec. 7.3
 *   - the fixed-point residual R^k of PDHG                            Sec. 6.1
 *
 * Readings where the paper is silent (each is also listed in the design
 * notes):
 *   - grid spacing, mu = h^2/(32 tau), the residual R^k (1/nu on the W
 *     block), R^0 = tau ||f||^2 and the check cadence are those of the
 *     vector method; nu = 1/(4 tau lambda_max(-Delta_L)).
 *   - mass: div_L maps into the trace-free matrices and the zero-flux
 *     spatial divergence sums to zero over the grid, so the data must have
 *     tr sum_x (Lambda0 - Lambda1) = 0.  f = Lambda1 - Lambda0 has
 *     (tr sum_x f / (m n k)) I removed, in FP64.
 *   - at a pixel U = (U_x, U_y): ||U||_2 is one Frobenius block over both
 *     directions, ||U||_1 the sum of the moduli of all complex entries,
 *     ||U||_{1,nuc} the sum over the two directions of the nuclear norm; W
 *     likewise over its l matrices.
 *   - the nuclear shrink of a Hermitian matrix soft-thresholds the moduli
 *     of its eigenvalues and keeps their signs; that of a skew-Hermitian N
 *     is -i times the shrink of the Hermitian matrix iN.
 *
 * Layout: every complex entry is a (re, im) pair of doubles, matrices are
 * row-major:
 *   Phi, f, Lambda, U_x, U_y : [i][j][a][b]     m*n*k*k entries
 *   W                        : [i][j][s][a][b]  m*n*l*k*k entries
 *   L                        : [s][a][b]        l*k*k entries
 * U_x is zero on the ghost row i = m-1 and U_y on the ghost column j = n-1.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double _Complex cx;

#define MORC_FRO 0 /* ||.||_2 : Frobenius norm of the whole block          */
#define MORC_L1 1  /* ||.||_1 : sum of moduli of all complex entries       */
#define MORC_NUC 2 /* ||.||_{1,nuc} : sum of the matrices' nuclear norms    */

#define MORC_KMAX 8
#define MORC_RSQRT2 0.70710678118654752440 /* 1/sqrt(2) */

typedef struct {
    int m, n, k, l;
    const double *L; /* l Hermitian k x k matrices                      */
    double alpha, tau, mu, nu, h;
    int unorm, wnorm;
} morc_problem;

typedef struct {
    int64_t iters;
    double R;             /* fixed-point residual of the last step          */
    double residual;      /* sqrt(R / R0)                                   */
    double primal;        /* ||U||_u + alpha ||W||_w                        */
    double dual;          /* <Phi, f>                                       */
    double rel_gap;       /* (primal - dual) / primal                       */
    double mass_residual; /* ||div_x U + div_L W + f|| / ||f||             */
    int converged;
} morc_info;

/* The staggered gradient and divergence of App. A act on every channel
 * independently; a complex k x k matrix is 2 k^2 real channels. */
void orc_grad_x(int m, int n, int k, double h, const double *phi, double *gx, double *gy);
void orc_div_x(int m, int n, int k, double h, const double *ux, const double *uy, double *out);

/* ------------------------------------------------------- small matrices */

static void mat_mul(int k, const cx *A, const cx *B, cx *C)
{
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            cx s = 0.0;
            for (int q = 0; q < k; ++q) s += A[a * k + q] * B[q * k + b];
            C[a * k + b] = s;
        }
}

/* Hilbert-Schmidt inner product Re tr(X Y^*) of count k x k matrices. */
static double hs_dot(int k, int count, const cx *X, const cx *Y)
{
    double s = 0.0;
    for (int q = 0; q < count * k * k; ++q) s += creal(X[q] * conj(Y[q]));
    return s;
}

/* grad_L X = (L_s X - X L_s), s = 1..l (Sec. 4.1). */
void morc_grad_L(int k, int l, const double *Ld, const double *Xd, double *Zd)
{
    const cx *L = (const cx *)Ld, *X = (const cx *)Xd;
    cx *Z = (cx *)Zd;
    cx LX[MORC_KMAX * MORC_KMAX], XL[MORC_KMAX * MORC_KMAX];
    for (int s = 0; s < l; ++s) {
        mat_mul(k, L + s * k * k, X, LX);
        mat_mul(k, X, L + s * k * k, XL);
        for (int q = 0; q < k * k; ++q) Z[s * k * k + q] = LX[q] - XL[q];
    }
}

/* div_L Z = sum_s (-L_s Z_s + Z_s L_s) (Sec. 4.1). */
void morc_div_L(int k, int l, const double *Ld, const double *Zd, double *Xd)
{
    const cx *L = (const cx *)Ld, *Z = (const cx *)Zd;
    cx *X = (cx *)Xd;
    cx LZ[MORC_KMAX * MORC_KMAX], ZL[MORC_KMAX * MORC_KMAX];
    for (int q = 0; q < k * k; ++q) X[q] = 0.0;
    for (int s = 0; s < l; ++s) {
        mat_mul(k, L + s * k * k, Z + s * k * k, LZ);
        mat_mul(k, Z + s * k * k, L + s * k * k, ZL);
        for (int q = 0; q < k * k; ++q) X[q] += -LZ[q] + ZL[q];
    }
}

/* Cyclic Jacobi on a real symmetric n x n matrix A (destroyed):
 * A = V diag(ev) V^T, V row-major with the eigenvectors as columns. */
static void jacobi_eig(int n, double *A, double *V, double *ev)
{
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) V[p * n + q] = (p == q) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) {
                tot += A[p * n + q] * A[p * n + q];
                if (p != q) off += A[p * n + q] * A[p * n + q];
            }
        if (off <= 1e-32 * (tot > 0 ? tot : 1.0)) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (apq == 0.0) continue;
                double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int r = 0; r < n; ++r) {
                    double arp = A[r * n + p], arq = A[r * n + q];
                    A[r * n + p] = cs * arp - sn * arq;
                    A[r * n + q] = sn * arp + cs * arq;
                }
                for (int r = 0; r < n; ++r) {
                    double apr = A[p * n + r], aqr = A[q * n + r];
                    A[p * n + r] = cs * apr - sn * aqr;
                    A[q * n + r] = sn * apr + cs * aqr;
                }
                for (int r = 0; r < n; ++r) {
                    double vrp = V[r * n + p], vrq = V[r * n + q];
                    V[r * n + p] = cs * vrp - sn * vrq;
                    V[r * n + q] = sn * vrp + cs * vrq;
                }
            }
    }
    for (int p = 0; p < n; ++p) ev[p] = A[p * n + p];
}

/* Spectral function of a Hermitian H = A + iB through its real symmetric
 * image [[A, -B], [B, A]] (same eigenvalues, each twice): g(H) is read off
 * the left blocks of V g(ev) V^T.  mode 0: out = H with every eigenvalue
 * soft-thresholded by t, keeping its sign; mode 1: out[0] = sum |ev|
 * (the nuclear norm of H). */
static void herm_spectral(int k, const cx *H, int mode, double t, cx *out, double *nuc)
{
    const int n = 2 * k;
    double S[4 * MORC_KMAX * MORC_KMAX], V[4 * MORC_KMAX * MORC_KMAX], ev[2 * MORC_KMAX];
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            const double A = creal(H[a * k + b]), B = cimag(H[a * k + b]);
            S[a * n + b] = A;
            S[a * n + (k + b)] = -B;
            S[(k + a) * n + b] = B;
            S[(k + a) * n + (k + b)] = A;
        }
    jacobi_eig(n, S, V, ev);
    if (mode == 1) {
        double s = 0.0;
        for (int p = 0; p < n; ++p) s += fabs(ev[p]);
        *nuc = 0.5 * s;
        return;
    }
    double g[2 * MORC_KMAX];
    for (int p = 0; p < n; ++p) {
        const double r = fabs(ev[p]) - t;
        g[p] = r > 0.0 ? (ev[p] > 0.0 ? r : -r) : 0.0;
    }
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
            double re = 0.0, im = 0.0;
            for (int p = 0; p < n; ++p) {
                re += V[a * n + p] * g[p] * V[b * n + p];
                im += V[(k + a) * n + p] * g[p] * V[b * n + p];
            }
            out[a * k + b] = re + I * im;
        }
}

/* --------------------------------------------------------------- shrinks */

/* shrink_1 of App. B on one complex number: (1 - t/|x|) x for |x| >= t. */
static cx shrink_c(cx x, double t)
{
    const double r = cabs(x);
    return (r >= t && r > 0.0) ? (1.0 - t / r) * x : 0.0;
}

/* Shrink of the norm `kind` with threshold t on a block of count k x k
 * matrices (U: count = 2 directions; W: count = l).  herm = 1 for Hermitian
 * matrices, 0 for skew-Hermitian ones (only the nuclear shrink needs it). */
void morc_shrink_block(int kind, int herm, int k, int count, double *Xd, double t)
{
    cx *X = (cx *)Xd;
    const int kk = k * k;
    if (kind == MORC_FRO) {
        double r2 = 0.0;
        for (int q = 0; q < count * kk; ++q) r2 += creal(X[q] * conj(X[q]));
        const double r = sqrt(r2);
        const double s = (r >= t && r > 0.0) ? 1.0 - t / r : 0.0;
        for (int q = 0; q < count * kk; ++q) X[q] *= s;
    } else if (kind == MORC_L1) {
        for (int q = 0; q < count * kk; ++q) X[q] = shrink_c(X[q], t);
    } else {
        cx H[MORC_KMAX * MORC_KMAX], G[MORC_KMAX * MORC_KMAX];
        for (int s = 0; s < count; ++s) {
            cx *Xs = X + s * kk;
            if (herm) {
                herm_spectral(k, Xs, 0, t, G, NULL);
                for (int q = 0; q < kk; ++q) Xs[q] = G[q];
            } else {
                for (int q = 0; q < kk; ++q) H[q] = I * Xs[q];
                herm_spectral(k, H, 0, t, G, NULL);
                for (int q = 0; q < kk; ++q) Xs[q] = -I * G[q];
            }
        }
    }
}

/* The norm `kind` of a block of count k x k matrices (Sec. 6.2). */
double morc_norm_block(int kind, int herm, int k, int count, const double *Xd)
{
    const cx *X = (const cx *)Xd;
    const int kk = k * k;
    if (kind == MORC_FRO) {
        double r2 = 0.0;
        for (int q = 0; q < count * kk; ++q) r2 += creal(X[q] * conj(X[q]));
        return sqrt(r2);
    }
    if (kind == MORC_L1) {
        double s = 0.0;
        for (int q = 0; q < count * kk; ++q) s += cabs(X[q]);
        return s;
    }
    double s = 0.0, nuc = 0.0;
    cx H[MORC_KMAX * MORC_KMAX];
    for (int c = 0; c < count; ++c) {
        for (int q = 0; q < kk; ++q) H[q] = herm ? X[c * kk + q] : I * X[c * kk + q];
        herm_spectral(k, H, 1, 0.0, NULL, &nuc);
        s += nuc;
    }
    return s;
}

/* ------------------------------------------------------------ step sizes */

/* lambda_max(-Delta_L) (Sec. 7.3): the k^2 x k^2 matrix of -Delta_L =
 * -div_L grad_L on the Hermitian matrices, in the orthonormal basis
 * E_aa, (E_ab + E_ba)/sqrt2, i(E_ab - E_ba)/sqrt2 (a < b), and its largest
 * eigenvalue by cyclic Jacobi. */
double morc_lambda_max(int k, int l, const double *L)
{
    const int K = k * k;
    cx *basis = (cx *)calloc((size_t)K * (size_t)K, sizeof(cx));
    int q = 0;
    for (int a = 0; a < k; ++a) basis[(size_t)q++ * K + a * k + a] = 1.0;
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b) {
            basis[(size_t)q * K + a * k + b] = MORC_RSQRT2;
            basis[(size_t)q * K + b * k + a] = MORC_RSQRT2;
            ++q;
            basis[(size_t)q * K + a * k + b] = I * MORC_RSQRT2;
            basis[(size_t)q * K + b * k + a] = -I * MORC_RSQRT2;
            ++q;
        }
    cx *Z = (cx *)malloc(sizeof(cx) * (size_t)l * (size_t)K), *Y = (cx *)malloc(sizeof(cx) * (size_t)K);
    double *A = (double *)malloc(sizeof(double) * (size_t)K * (size_t)K);
    double *V = (double *)malloc(sizeof(double) * (size_t)K * (size_t)K), *ev = (double *)malloc(sizeof(double) * K);
    for (int c = 0; c < K; ++c) {
        morc_grad_L(k, l, L, (const double *)(basis + (size_t)c * K), (double *)Z);
        morc_div_L(k, l, L, (const double *)Z, (double *)Y);
        for (int r = 0; r < K; ++r) A[r * K + c] = -hs_dot(k, 1, basis + (size_t)r * K, Y);
    }
    jacobi_eig(K, A, V, ev);
    double mx = 0.0;
    for (int r = 0; r < K; ++r)
        if (ev[r] > mx) mx = ev[r];
    free(basis);
    free(Z);
    free(Y);
    free(A);
    free(V);
    free(ev);
    return mx;
}

/* Fills h, mu, nu where they are zero: h = 1/(max(m,n)-1),
 * mu = h^2/(32 tau), nu = 1/(4 tau lambda_max(-Delta_L)) (Sec. 7.3). */
void morc_default_steps(morc_problem *p)
{
    const int side = p->m > p->n ? p->m : p->n;
    if (p->h <= 0.0) p->h = 1.0 / (double)(side - 1);
    if (p->mu <= 0.0) p->mu = p->h * p->h / (32.0 * p->tau);
    if (p->nu <= 0.0) {
        const double lm = morc_lambda_max(p->k, p->l, p->L);
        p->nu = lm > 0.0 ? 1.0 / (4.0 * p->tau * lm) : 0.0;
    }
}

/* f = Lambda1 - Lambda0 with (tr sum f / (m n k)) I removed.  Returns
 * |tr sum (Lambda0 - Lambda1)| / max(|tr sum Lambda0|, |tr sum Lambda1|). */
double morc_prepare_f(int m, int n, int k, const double *lam0d, const double *lam1d, double *fd)
{
    const cx *l0 = (const cx *)lam0d, *l1 = (const cx *)lam1d;
    cx *f = (cx *)fd;
    const size_t P = (size_t)m * (size_t)n, kk = (size_t)k * (size_t)k;
    double t0 = 0.0, t1 = 0.0, tf = 0.0;
    for (size_t q = 0; q < P; ++q)
        for (int a = 0; a < k; ++a) {
            t0 += creal(l0[q * kk + a * k + a]);
            t1 += creal(l1[q * kk + a * k + a]);
        }
    for (size_t q = 0; q < P * kk; ++q) f[q] = l1[q] - l0[q];
    for (size_t q = 0; q < P; ++q)
        for (int a = 0; a < k; ++a) tf += creal(f[q * kk + a * k + a]);
    const double mean = tf / ((double)P * (double)k);
    for (size_t q = 0; q < P; ++q)
        for (int a = 0; a < k; ++a) f[q * kk + a * k + a] -= mean;
    const double sc = fmax(fabs(t0), fabs(t1));
    return sc > 0.0 ? fabs(t0 - t1) / sc : fabs(t0 - t1);
}

/* --------------------------------------------------------------- method */

typedef struct {
    double *gx, *gy, *bx, *by, *dx; /* 2 k^2 real channels per pixel       */
    cx *gL, *bw, *dL;
} mwork_t;

static void mwork_alloc(const morc_problem *p, mwork_t *W)
{
    const size_t P = (size_t)p->m * (size_t)p->n, kk = (size_t)p->k * (size_t)p->k;
    W->gx = (double *)calloc(2 * P * kk, sizeof(double));
    W->gy = (double *)calloc(2 * P * kk, sizeof(double));
    W->bx = (double *)calloc(2 * P * kk, sizeof(double));
    W->by = (double *)calloc(2 * P * kk, sizeof(double));
    W->dx = (double *)calloc(2 * P * kk, sizeof(double));
    W->gL = (cx *)calloc(P * kk * (size_t)p->l, sizeof(cx));
    W->bw = (cx *)calloc(P * kk * (size_t)p->l, sizeof(cx));
    W->dL = (cx *)calloc(P * kk, sizeof(cx));
}

static void mwork_free(mwork_t *W)
{
    free(W->gx);
    free(W->gy);
    free(W->bx);
    free(W->by);
    free(W->dx);
    free(W->gL);
    free(W->bw);
    free(W->dL);
}

/* div_L of every pixel's W. */
static void div_L_field(const morc_problem *p, const cx *W, cx *out)
{
    const size_t P = (size_t)p->m * (size_t)p->n, kk = (size_t)p->k * (size_t)p->k;
    for (size_t q = 0; q < P; ++q)
        morc_div_L(p->k, p->l, p->L, (const double *)(W + q * kk * (size_t)p->l), (double *)(out + q * kk));
}

/* One iteration of the first-order method for M-OMT (Sec. 7.3):
 *   U1   = shrink_u(U + mu grad_x Phi, mu)
 *   W1   = shrink_w(W + nu grad_L Phi, alpha nu)
 *   Phi1 = Phi + tau (div_x(2 U1 - U) + div_L(2 W1 - W) + f)             */
static void mpdhg_step(const morc_problem *p, const cx *f, const cx *phi, const cx *ux, const cx *uy, const cx *w,
                       cx *phi1, cx *ux1, cx *uy1, cx *w1, mwork_t *Wk)
{
    const int m = p->m, n = p->n, k = p->k, l = p->l;
    const size_t P = (size_t)m * (size_t)n, kk = (size_t)k * (size_t)k;
    const int ch = 2 * k * k;

    orc_grad_x(m, n, ch, p->h, (const double *)phi, Wk->gx, Wk->gy);
    const cx *gx = (const cx *)Wk->gx, *gy = (const cx *)Wk->gy;
    cx blk[2 * MORC_KMAX * MORC_KMAX];
    for (size_t q = 0; q < P; ++q) {
        const int i = (int)(q / (size_t)n), j = (int)(q % (size_t)n);
        for (size_t e = 0; e < kk; ++e) {
            blk[e] = (i < m - 1) ? ux[q * kk + e] + p->mu * gx[q * kk + e] : 0.0;
            blk[kk + e] = (j < n - 1) ? uy[q * kk + e] + p->mu * gy[q * kk + e] : 0.0;
        }
        morc_shrink_block(p->unorm, 1, k, 2, (double *)blk, p->mu);
        for (size_t e = 0; e < kk; ++e) {
            ux1[q * kk + e] = blk[e];
            uy1[q * kk + e] = blk[kk + e];
        }
    }

    for (size_t q = 0; q < P; ++q) {
        cx *b = w1 + q * kk * (size_t)l;
        morc_grad_L(k, l, p->L, (const double *)(phi + q * kk), (double *)(Wk->gL + q * kk * (size_t)l));
        for (size_t e = 0; e < kk * (size_t)l; ++e) b[e] = w[q * kk * (size_t)l + e] + p->nu * Wk->gL[q * kk * (size_t)l + e];
        morc_shrink_block(p->wnorm, 0, k, l, (double *)b, p->alpha * p->nu);
    }

    cx *bx = (cx *)Wk->bx, *by = (cx *)Wk->by;
    for (size_t q = 0; q < P * kk; ++q) {
        bx[q] = 2.0 * ux1[q] - ux[q];
        by[q] = 2.0 * uy1[q] - uy[q];
    }
    orc_div_x(m, n, ch, p->h, Wk->bx, Wk->by, Wk->dx);
    for (size_t q = 0; q < P * kk * (size_t)l; ++q) Wk->bw[q] = 2.0 * w1[q] - w[q];
    div_L_field(p, Wk->bw, Wk->dL);
    const cx *dx = (const cx *)Wk->dx;
    for (size_t q = 0; q < P * kk; ++q) phi1[q] = phi[q] + p->tau * (dx[q] + Wk->dL[q] + f[q]);
}

/* Check quantities: out[0] = R^k, out[1] = primal, out[2] = <Phi1, f>,
 * out[3] = ||div_x U1 + div_L W1 + f||^2, out[4] = ||f||^2 (all in the
 * Hilbert-Schmidt inner product). */
static void mmetrics(const morc_problem *p, const cx *f, const cx *phi, const cx *ux, const cx *uy, const cx *w,
                     const cx *phi1, const cx *ux1, const cx *uy1, const cx *w1, double *out)
{
    const int m = p->m, n = p->n, k = p->k, l = p->l;
    const size_t P = (size_t)m * (size_t)n, kk = (size_t)k * (size_t)k, Pk = P * kk, Pl = Pk * (size_t)l;
    const int ch = 2 * k * k;
    cx *dux = (cx *)malloc(sizeof(cx) * Pk), *duy = (cx *)malloc(sizeof(cx) * Pk);
    cx *dw = (cx *)malloc(sizeof(cx) * Pl), *t1 = (cx *)malloc(sizeof(cx) * Pk), *t2 = (cx *)malloc(sizeof(cx) * Pk);
    cx *dphi = (cx *)malloc(sizeof(cx) * Pk);
    for (size_t q = 0; q < Pk; ++q) {
        dux[q] = ux1[q] - ux[q];
        duy[q] = uy1[q] - uy[q];
        dphi[q] = phi1[q] - phi[q];
    }
    for (size_t q = 0; q < Pl; ++q) dw[q] = w1[q] - w[q];
    const double su = hs_dot(k, (int)P, dux, dux) + hs_dot(k, (int)P, duy, duy);
    const double sw = hs_dot(k, (int)(P * (size_t)l), dw, dw);
    const double sp = hs_dot(k, (int)P, dphi, dphi);
    orc_div_x(m, n, ch, p->h, (const double *)dux, (const double *)duy, (double *)t1);
    div_L_field(p, dw, t2);
    for (size_t q = 0; q < Pk; ++q) t1[q] += t2[q];
    const double cross = hs_dot(k, (int)P, dphi, t1);

    double prim = 0.0;
    cx blk[2 * MORC_KMAX * MORC_KMAX];
    for (size_t q = 0; q < P; ++q) {
        for (size_t e = 0; e < kk; ++e) {
            blk[e] = ux1[q * kk + e];
            blk[kk + e] = uy1[q * kk + e];
        }
        prim += morc_norm_block(p->unorm, 1, k, 2, (const double *)blk);
        prim += p->alpha * morc_norm_block(p->wnorm, 0, k, l, (const double *)(w1 + q * kk * (size_t)l));
    }
    orc_div_x(m, n, ch, p->h, (const double *)ux1, (const double *)uy1, (double *)t1);
    div_L_field(p, w1, t2);
    for (size_t q = 0; q < Pk; ++q) t1[q] += t2[q] + f[q];
    out[0] = su / p->mu + sw / p->nu + sp / p->tau - 2.0 * cross;
    out[1] = prim;
    out[2] = hs_dot(k, (int)P, phi1, f);
    out[3] = hs_dot(k, (int)P, t1, t1);
    out[4] = hs_dot(k, (int)P, f, f);
    free(dux);
    free(duy);
    free(dw);
    free(t1);
    free(t2);
    free(dphi);
}

/* Runs the method from the state (Phi, U_x, U_y, W), overwritten with the
 * last iterate.  Stopping, checks and hist as in the vector oracle: a check
 * every check_every iterations and after the last; stop at the first check
 * with sqrt(R/R0) <= tol when tol > 0.  Returns the number of checks. */
int morc_solve(const morc_problem *pin, const double *fd, double *phid, double *uxd, double *uyd, double *wd,
               int64_t max_iters, double tol, int check_every, morc_info *info, double *hist, int hist_cap)
{
    morc_problem p = *pin;
    const int m = p.m, n = p.n, k = p.k;
    const size_t P = (size_t)m * (size_t)n, kk = (size_t)k * (size_t)k, Pk = P * kk, Pl = Pk * (size_t)p.l;
    const cx *f = (const cx *)fd;
    cx *phi = (cx *)phid, *ux = (cx *)uxd, *uy = (cx *)uyd, *w = (cx *)wd;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j)
            for (size_t e = 0; e < kk; ++e) {
                const size_t q = ((size_t)i * (size_t)n + (size_t)j) * kk + e;
                if (i == m - 1) ux[q] = 0.0;
                if (j == n - 1) uy[q] = 0.0;
            }
    cx *phi1 = (cx *)malloc(sizeof(cx) * Pk), *ux1 = (cx *)malloc(sizeof(cx) * Pk);
    cx *uy1 = (cx *)malloc(sizeof(cx) * Pk), *w1 = (cx *)malloc(sizeof(cx) * Pl);
    mwork_t Wk;
    mwork_alloc(&p, &Wk);
    const double ff = hs_dot(k, (int)P, f, f), R0 = p.tau * ff;
    if (check_every <= 0) check_every = 64;
    memset(info, 0, sizeof(*info));
    int nchecks = 0;
    for (int64_t it = 1; it <= max_iters; ++it) {
        mpdhg_step(&p, f, phi, ux, uy, w, phi1, ux1, uy1, w1, &Wk);
        const int check = (it % check_every == 0) || (it == max_iters);
        if (check) {
            double met[5];
            mmetrics(&p, f, phi, ux, uy, w, phi1, ux1, uy1, w1, met);
            info->iters = it;
            info->R = met[0];
            info->residual = R0 > 0 ? sqrt(fmax(met[0], 0.0) / R0) : 0.0;
            info->primal = met[1];
            info->dual = met[2];
            info->rel_gap = met[1] > 0 ? (met[1] - met[2]) / met[1] : 0.0;
            info->mass_residual = ff > 0 ? sqrt(met[3] / ff) : 0.0;
            if (hist && nchecks < hist_cap) hist[nchecks] = info->residual;
            ++nchecks;
        }
        memcpy(phi, phi1, sizeof(cx) * Pk);
        memcpy(ux, ux1, sizeof(cx) * Pk);
        memcpy(uy, uy1, sizeof(cx) * Pk);
        memcpy(w, w1, sizeof(cx) * Pl);
        if (check && tol > 0.0 && info->residual <= tol) {
            info->converged = 1;
            break;
        }
    }
    mwork_free(&Wk);
    free(phi1);
    free(ux1);
    free(uy1);
    free(w1);
    return nchecks;
}

/* One bare iteration (for first-iterate and operator tests). */
void morc_step(const morc_problem *p, const double *f, const double *phi, const double *ux, const double *uy,
               const double *w, double *phi1, double *ux1, double *uy1, double *w1)
{
    mwork_t Wk;
    mwork_alloc(p, &Wk);
    mpdhg_step(p, (const cx *)f, (const cx *)phi, (const cx *)ux, (const cx *)uy, (const cx *)w, (cx *)phi1,
               (cx *)ux1, (cx *)uy1, (cx *)w1, &Wk);
    mwork_free(&Wk);
}
