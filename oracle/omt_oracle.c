/*
 * Oracle for the vector optimal mass transport (V-OMT) PDHG method of
 * Ryu, Chen, Li and Osher, "Vector and Matrix Optimal Mass Transport:
 * Theory, Algorithm, and Applications" (arXiv 1712.10279).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * FP64 single-threaded reference that the HIP path is checked against.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * load it.  It shares no code, header, table or constant with the HIP path.
 *
 * Every routine follows one passage of the paper:
 *   - incidence matrix D, graph gradient / divergence     Sec. 3.1
 *   - staggered spatial gradient / divergence, ghosts       App. A
 *   - shrink operators and their component-wise use         App. B
 *   - the V-OMT / S-OMT first-order method and step sizes   Sec. 7.1, 7.2
 *   - the fixed-point residual R^k of PDHG                  Sec. 6.1
 *   - duality gap / primal objective as precision           Sec. 8.1
 *
 * Readings where the paper is silent or garbled (each is also listed in the
 * design notes):
 *   - R^k: the second term carries 1/nu (the step of the second primal
 *     block), not 1/mu as printed in Sec. 6.1.
 *   - grid spacing h = 1/(max(m,n)-1) unless given; mu = h^2/(32 tau)
 *     (h^2/(16 tau) when the graph has no edges), nu = 1/(4 tau lmax).
 *   - the source term f = lambda1 - lambda0 has its mean over every mass
 *     class (connected component of the channel graph) removed in FP64.
 *   - the relative residual is sqrt(R^k / R^0) with R^0 = tau ||f||^2, the
 *     value of R for the first step taken from the all-zero start.
 *   - quadratic regularisation (Sec. 9) adds eps (|u|^2 + |w|^2) with the
 *     Euclidean square of all components, so each shrink result is divided
 *     by 1 + 2 t eps (t the step of that block): the prox of
 *     t ||.|| + t eps |.|^2.
 *
 * Layout (paper order): arrays indexed [i][j][c], channel fastest:
 *   phi, lambda, f, u_x, u_y : m*n*k      w : m*n*l
 * u_x is zero on the ghost row i = m-1 and u_y on the ghost column j = n-1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_U_L12 0 /* sum over channels of the Euclidean norm of (u_x,u_y) */
#define ORC_U_L1 1  /* sum of absolute values of all components            */
#define ORC_U_L2 2  /* Euclidean norm of all 2k components of a pixel       */
#define ORC_W_L1 0  /* sum of absolute values                               */
#define ORC_W_L2 1  /* Euclidean norm of the l components of a pixel        */

typedef struct {
    int m, n, k, l;
    const int *edges;    /* 2*l node indices (a_e, b_e), a_e < b_e          */
    const double *cost;  /* l edge costs c_e > 0                            */
    double alpha, tau, mu, nu, h;
    int unorm, wnorm;
    double eps;          /* quadratic regularisation weight (Sec. 9), >= 0  */
} orc_problem;

typedef struct {
    int64_t iters;
    double R;             /* fixed-point residual of the last step          */
    double residual;      /* sqrt(R / R0)                                   */
    double primal;        /* ||u||_u + alpha ||w||_w                        */
    double dual;          /* <phi, f>                                       */
    double rel_gap;       /* (primal - dual) / primal                       */
    double mass_residual; /* ||div_x u + div_G w + f|| / ||f||             */
    int converged;
} orc_info;

#define I3(i, j, c, n, k) ((((size_t)(i)) * (size_t)(n) + (size_t)(j)) * (size_t)(k) + (size_t)(c))

/* ---------------------------------------------------------------- graph -- */

/* Incidence matrix of Sec. 3.1: column e has +1 at the lower-numbered node
 * a_e and -1 at the higher-numbered node b_e.  D is k x l, row-major. */
void orc_incidence(int k, int l, const int *edges, double *D)
{
    for (int c = 0; c < k; ++c)
        for (int e = 0; e < l; ++e) D[c * l + e] = 0.0;
    for (int e = 0; e < l; ++e) {
        int a = edges[2 * e], b = edges[2 * e + 1];
        int lo = a < b ? a : b, hi = a < b ? b : a;
        D[lo * l + e] = 1.0;
        D[hi * l + e] = -1.0;
    }
}

/* (grad_G x)_e = (1/c_e) (D^T x)_e  on one pixel (Sec. 3.1). */
static void graph_grad(int k, int l, const double *D, const double *cost, const double *x, double *y)
{
    for (int e = 0; e < l; ++e) {
        double s = 0.0;
        for (int c = 0; c < k; ++c) s += D[c * l + e] * x[c];
        y[e] = s / cost[e];
    }
}

/* (div_G y)_c = -(D diag(1/c) y)_c  on one pixel (Sec. 3.1). */
static void graph_div(int k, int l, const double *D, const double *cost, const double *y, double *x)
{
    for (int c = 0; c < k; ++c) {
        double s = 0.0;
        for (int e = 0; e < l; ++e) s += D[c * l + e] * (y[e] / cost[e]);
        x[c] = -s;
    }
}

/* Largest eigenvalue of a symmetric k x k matrix by the cyclic Jacobi
 * method (a standard eigenvalue routine, as Sec. 7.2 asks for). */
double orc_sym_lambda_max(int k, const double *Ain)
{
    double *A = (double *)malloc(sizeof(double) * (size_t)k * (size_t)k);
    memcpy(A, Ain, sizeof(double) * (size_t)k * (size_t)k);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int p = 0; p < k; ++p)
            for (int q = 0; q < k; ++q) {
                tot += A[p * k + q] * A[p * k + q];
                if (p != q) off += A[p * k + q] * A[p * k + q];
            }
        if (off <= 1e-30 * (tot > 0 ? tot : 1.0)) break;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                double apq = A[p * k + q];
                if (apq == 0.0) continue;
                double theta = (A[q * k + q] - A[p * k + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int r = 0; r < k; ++r) { /* A <- A J */
                    double arp = A[r * k + p], arq = A[r * k + q];
                    A[r * k + p] = cs * arp - sn * arq;
                    A[r * k + q] = sn * arp + cs * arq;
                }
                for (int r = 0; r < k; ++r) { /* A <- J^T A */
                    double apr = A[p * k + r], aqr = A[q * k + r];
                    A[p * k + r] = cs * apr - sn * aqr;
                    A[q * k + r] = sn * apr + cs * aqr;
                }
            }
    }
    double mx = -INFINITY;
    for (int p = 0; p < k; ++p)
        if (A[p * k + p] > mx) mx = A[p * k + p];
    free(A);
    return k > 0 ? mx : 0.0;
}

/* lambda_max(-Delta_G) with -Delta_G = D diag(1/c^2) D^T (Sec. 3.1, 7.2). */
double orc_graph_lambda_max(int k, int l, const int *edges, const double *cost)
{
    if (l == 0 || k == 0) return 0.0;
    double *D = (double *)malloc(sizeof(double) * (size_t)k * (size_t)l);
    double *L = (double *)malloc(sizeof(double) * (size_t)k * (size_t)k);
    orc_incidence(k, l, edges, D);
    for (int p = 0; p < k; ++p)
        for (int q = 0; q < k; ++q) {
            double s = 0.0;
            for (int e = 0; e < l; ++e) s += D[p * l + e] * D[q * l + e] / (cost[e] * cost[e]);
            L[p * k + q] = s;
        }
    double lm = orc_sym_lambda_max(k, L);
    free(D);
    free(L);
    return lm;
}

/* Mass classes: connected components of the channel graph.  cls[c] gets a
 * component id in [0, k); returns the number of components. */
int orc_mass_classes(int k, int l, const int *edges, int *cls)
{
    for (int c = 0; c < k; ++c) cls[c] = c;
    for (int changed = 1; changed;) { /* label propagation: smallest id wins */
        changed = 0;
        for (int e = 0; e < l; ++e) {
            int a = edges[2 * e], b = edges[2 * e + 1];
            int lo = cls[a] < cls[b] ? cls[a] : cls[b];
            if (cls[a] != lo || cls[b] != lo) {
                cls[a] = cls[b] = lo;
                changed = 1;
            }
        }
    }
    int nc = 0;
    int *map = (int *)malloc(sizeof(int) * (size_t)(k > 0 ? k : 1));
    for (int c = 0; c < k; ++c) map[c] = -1;
    for (int c = 0; c < k; ++c) {
        if (map[cls[c]] < 0) map[cls[c]] = nc++;
        cls[c] = map[cls[c]];
    }
    free(map);
    return nc;
}

/* ---------------------------------------------------------- grid (App. A) */

/* Forward differences with the ghost row / column set to zero. */
void orc_grad_x(int m, int n, int k, double h, const double *phi, double *gx, double *gy)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j)
            for (int c = 0; c < k; ++c) {
                gx[I3(i, j, c, n, k)] = (i < m - 1) ? (phi[I3(i + 1, j, c, n, k)] - phi[I3(i, j, c, n, k)]) / h : 0.0;
                gy[I3(i, j, c, n, k)] = (j < n - 1) ? (phi[I3(i, j + 1, c, n, k)] - phi[I3(i, j, c, n, k)]) / h : 0.0;
            }
}

/* Backward differences with zero flux through the boundary: u_x on row -1
 * and on the ghost row m-1 is zero, u_y on column -1 and column n-1 too. */
void orc_div_x(int m, int n, int k, double h, const double *ux, const double *uy, double *out)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j)
            for (int c = 0; c < k; ++c) {
                double xr = (i < m - 1) ? ux[I3(i, j, c, n, k)] : 0.0;
                double xl = (i > 0) ? ux[I3(i - 1, j, c, n, k)] : 0.0;
                double yr = (j < n - 1) ? uy[I3(i, j, c, n, k)] : 0.0;
                double yl = (j > 0) ? uy[I3(i, j - 1, c, n, k)] : 0.0;
                out[I3(i, j, c, n, k)] = (xr - xl + yr - yl) / h;
            }
}

void orc_grad_G(int m, int n, int k, int l, const int *edges, const double *cost, const double *phi, double *gG)
{
    double *D = (double *)malloc(sizeof(double) * (size_t)(k * l > 0 ? k * l : 1));
    orc_incidence(k, l, edges, D);
    for (size_t p = 0; p < (size_t)m * (size_t)n; ++p) graph_grad(k, l, D, cost, phi + p * (size_t)k, gG + p * (size_t)l);
    free(D);
}

void orc_div_G(int m, int n, int k, int l, const int *edges, const double *cost, const double *w, double *out)
{
    double *D = (double *)malloc(sizeof(double) * (size_t)(k * l > 0 ? k * l : 1));
    orc_incidence(k, l, edges, D);
    for (size_t p = 0; p < (size_t)m * (size_t)n; ++p) graph_div(k, l, D, cost, w + p * (size_t)l, out + p * (size_t)k);
    free(D);
}

/* ------------------------------------------------------ shrinks (App. B) */

/* shrink_1 of a real scalar: (1 - t/|x|) x if |x| >= t, else 0. */
double orc_shrink1(double x, double t)
{
    double ax = fabs(x);
    return (ax >= t && ax > 0.0) ? (1.0 - t / ax) * x : 0.0;
}

/* shrink_2 of a d-vector, in place: (1 - t/||x||) x if ||x|| >= t, else 0. */
void orc_shrink2(int d, double *x, double t)
{
    double r = 0.0;
    for (int s = 0; s < d; ++s) r += x[s] * x[s];
    r = sqrt(r);
    double scale = (r >= t && r > 0.0) ? (1.0 - t / r) : 0.0;
    for (int s = 0; s < d; ++s) x[s] *= scale;
}

/* Shrink of the pixel flux block (u_x, u_y) in R^{k x 2} for the norm chosen
 * (Sec. 6.2 norms, shrinks applied component-wise as App. B allows). */
void orc_shrink_u(int unorm, int k, double *bx, double *by, double t)
{
    if (unorm == ORC_U_L12) {
        for (int c = 0; c < k; ++c) {
            double v[2] = {bx[c], by[c]};
            orc_shrink2(2, v, t);
            bx[c] = v[0];
            by[c] = v[1];
        }
    } else if (unorm == ORC_U_L1) {
        for (int c = 0; c < k; ++c) {
            bx[c] = orc_shrink1(bx[c], t);
            by[c] = orc_shrink1(by[c], t);
        }
    } else {
        double *v = (double *)malloc(sizeof(double) * 2 * (size_t)k);
        for (int c = 0; c < k; ++c) {
            v[c] = bx[c];
            v[k + c] = by[c];
        }
        orc_shrink2(2 * k, v, t);
        for (int c = 0; c < k; ++c) {
            bx[c] = v[c];
            by[c] = v[k + c];
        }
        free(v);
    }
}

void orc_shrink_w(int wnorm, int l, double *w, double t)
{
    if (wnorm == ORC_W_L1) {
        for (int e = 0; e < l; ++e) w[e] = orc_shrink1(w[e], t);
    } else {
        orc_shrink2(l, w, t);
    }
}

/* Pixel norms of Sec. 6.2 / App. A. */
double orc_norm_u(int unorm, int k, const double *bx, const double *by)
{
    double s = 0.0;
    if (unorm == ORC_U_L12) {
        for (int c = 0; c < k; ++c) s += sqrt(bx[c] * bx[c] + by[c] * by[c]);
    } else if (unorm == ORC_U_L1) {
        for (int c = 0; c < k; ++c) s += fabs(bx[c]) + fabs(by[c]);
    } else {
        for (int c = 0; c < k; ++c) s += bx[c] * bx[c] + by[c] * by[c];
        s = sqrt(s);
    }
    return s;
}

double orc_norm_w(int wnorm, int l, const double *w)
{
    double s = 0.0;
    if (wnorm == ORC_W_L1) {
        for (int e = 0; e < l; ++e) s += fabs(w[e]);
    } else {
        for (int e = 0; e < l; ++e) s += w[e] * w[e];
        s = sqrt(s);
    }
    return s;
}

/* ----------------------------------------------------------- problem set-up */

/* Default step sizes of Sec. 7.1 / 7.2 for the grid spacing h. */
void orc_default_steps(orc_problem *p)
{
    int side = p->m > p->n ? p->m : p->n;
    if (p->h <= 0.0) p->h = 1.0 / (double)(side - 1);
    if (p->l == 0) {
        if (p->mu <= 0.0) p->mu = p->h * p->h / (16.0 * p->tau);
        p->nu = 0.0;
    } else {
        if (p->mu <= 0.0) p->mu = p->h * p->h / (32.0 * p->tau);
        if (p->nu <= 0.0) p->nu = 1.0 / (4.0 * p->tau * orc_graph_lambda_max(p->k, p->l, p->edges, p->cost));
    }
}

/* f = lambda1 - lambda0, with the mean over each mass class removed.
 * Returns the largest relative imbalance |sum lambda0 - sum lambda1| /
 * max(sum |lambda0|, sum |lambda1|) over the classes. */
double orc_prepare_f(int m, int n, int k, int l, const int *edges, const double *lam0, const double *lam1, double *f)
{
    int *cls = (int *)malloc(sizeof(int) * (size_t)k);
    int nc = orc_mass_classes(k, l, edges, cls);
    double *s0 = (double *)calloc((size_t)nc, sizeof(double)), *s1 = (double *)calloc((size_t)nc, sizeof(double));
    double *a0 = (double *)calloc((size_t)nc, sizeof(double)), *a1 = (double *)calloc((size_t)nc, sizeof(double));
    double *cnt = (double *)calloc((size_t)nc, sizeof(double));
    size_t P = (size_t)m * (size_t)n;
    for (size_t p = 0; p < P; ++p)
        for (int c = 0; c < k; ++c) {
            size_t q = p * (size_t)k + (size_t)c;
            s0[cls[c]] += lam0[q];
            s1[cls[c]] += lam1[q];
            a0[cls[c]] += fabs(lam0[q]);
            a1[cls[c]] += fabs(lam1[q]);
            cnt[cls[c]] += 1.0;
        }
    double worst = 0.0;
    for (int g = 0; g < nc; ++g) {
        double den = a0[g] > a1[g] ? a0[g] : a1[g];
        double rel = den > 0 ? fabs(s0[g] - s1[g]) / den : 0.0;
        if (rel > worst) worst = rel;
    }
    for (size_t p = 0; p < P; ++p)
        for (int c = 0; c < k; ++c) {
            size_t q = p * (size_t)k + (size_t)c;
            f[q] = (lam1[q] - lam0[q]) - (s1[cls[c]] - s0[cls[c]]) / cnt[cls[c]];
        }
    free(cls);
    free(s0);
    free(s1);
    free(a0);
    free(a1);
    free(cnt);
    return worst;
}

/* ------------------------------------------------------------- PDHG step */

typedef struct {
    double *gx, *gy, *gG, *bx, *by, *bw, *dx, *dg;
} work_t;

static void work_alloc(const orc_problem *p, work_t *W)
{
    size_t Pk = (size_t)p->m * (size_t)p->n * (size_t)p->k;
    size_t Pl = (size_t)p->m * (size_t)p->n * (size_t)(p->l > 0 ? p->l : 1);
    W->gx = (double *)calloc(Pk, sizeof(double));
    W->gy = (double *)calloc(Pk, sizeof(double));
    W->bx = (double *)calloc(Pk, sizeof(double));
    W->by = (double *)calloc(Pk, sizeof(double));
    W->dx = (double *)calloc(Pk, sizeof(double));
    W->dg = (double *)calloc(Pk, sizeof(double));
    W->gG = (double *)calloc(Pl, sizeof(double));
    W->bw = (double *)calloc(Pl, sizeof(double));
}

static void work_free(work_t *W)
{
    free(W->gx);
    free(W->gy);
    free(W->gG);
    free(W->bx);
    free(W->by);
    free(W->bw);
    free(W->dx);
    free(W->dg);
}

/* One iteration of the first-order method for V-OMT (Sec. 7.2), S-OMT when
 * l = 0 (Sec. 7.1):
 *   u1  = shrink_u(u + mu grad phi, mu)
 *   w1  = shrink_w(w + nu grad_G phi, alpha nu)
 *   phi1 = phi + tau (div_x(2 u1 - u) + div_G(2 w1 - w) + f)            */
static void pdhg_step(const orc_problem *p, const double *f, const double *phi, const double *ux, const double *uy,
                      const double *w, double *phi1, double *ux1, double *uy1, double *w1, work_t *W)
{
    int m = p->m, n = p->n, k = p->k, l = p->l;
    size_t P = (size_t)m * (size_t)n;

    orc_grad_x(m, n, k, p->h, phi, W->gx, W->gy);
    for (size_t q = 0; q < P; ++q) {
        double *bx = ux1 + q * (size_t)k, *by = uy1 + q * (size_t)k;
        for (int c = 0; c < k; ++c) {
            bx[c] = ux[q * (size_t)k + c] + p->mu * W->gx[q * (size_t)k + c];
            by[c] = uy[q * (size_t)k + c] + p->mu * W->gy[q * (size_t)k + c];
        }
        orc_shrink_u(p->unorm, k, bx, by, p->mu);
        if (p->eps > 0.0)
            for (int c = 0; c < k; ++c) {
                bx[c] /= 1.0 + 2.0 * p->mu * p->eps;
                by[c] /= 1.0 + 2.0 * p->mu * p->eps;
            }
    }

    if (l > 0) {
        orc_grad_G(m, n, k, l, p->edges, p->cost, phi, W->gG);
        for (size_t q = 0; q < P; ++q) {
            double *b = w1 + q * (size_t)l;
            for (int e = 0; e < l; ++e) b[e] = w[q * (size_t)l + e] + p->nu * W->gG[q * (size_t)l + e];
            orc_shrink_w(p->wnorm, l, b, p->alpha * p->nu);
            if (p->eps > 0.0)
                for (int e = 0; e < l; ++e) b[e] /= 1.0 + 2.0 * p->nu * p->eps;
        }
    }

    for (size_t q = 0; q < P * (size_t)k; ++q) {
        W->bx[q] = 2.0 * ux1[q] - ux[q];
        W->by[q] = 2.0 * uy1[q] - uy[q];
    }
    orc_div_x(m, n, k, p->h, W->bx, W->by, W->dx);
    if (l > 0) {
        for (size_t q = 0; q < P * (size_t)l; ++q) W->bw[q] = 2.0 * w1[q] - w[q];
        orc_div_G(m, n, k, l, p->edges, p->cost, W->bw, W->dg);
    } else {
        for (size_t q = 0; q < P * (size_t)k; ++q) W->dg[q] = 0.0;
    }
    for (size_t q = 0; q < P * (size_t)k; ++q) phi1[q] = phi[q] + p->tau * (W->dx[q] + W->dg[q] + f[q]);
}

/* --------------------------------------------------------------- metrics */

/* Quantities reported at a check: out[0] = R^k (Sec. 6.1, with 1/nu on the
 * second block), out[1] = primal objective (with the regulariser), out[2] =
 * <phi1, f> (the dual objective when eps = 0),
 * out[3] = ||div_x u1 + div_G w1 + f||^2, out[4] = ||f||^2. */
void orc_metrics(const orc_problem *p, const double *f, const double *phi, const double *ux, const double *uy,
                 const double *w, const double *phi1, const double *ux1, const double *uy1, const double *w1,
                 double *out)
{
    int m = p->m, n = p->n, k = p->k, l = p->l;
    size_t P = (size_t)m * (size_t)n, Pk = P * (size_t)k, Pl = P * (size_t)l;
    double *dux = (double *)malloc(sizeof(double) * Pk), *duy = (double *)malloc(sizeof(double) * Pk);
    double *dw = (double *)malloc(sizeof(double) * (Pl > 0 ? Pl : 1));
    double *t1 = (double *)malloc(sizeof(double) * Pk), *t2 = (double *)malloc(sizeof(double) * Pk);
    double su = 0, sw = 0, sp = 0, cross = 0, prim = 0, dual = 0, mass = 0, ff = 0;

    for (size_t q = 0; q < Pk; ++q) {
        dux[q] = ux1[q] - ux[q];
        duy[q] = uy1[q] - uy[q];
        su += dux[q] * dux[q] + duy[q] * duy[q];
        double dp = phi1[q] - phi[q];
        sp += dp * dp;
    }
    for (size_t q = 0; q < Pl; ++q) {
        dw[q] = w1[q] - w[q];
        sw += dw[q] * dw[q];
    }
    /* <dphi, div_x du + div_G dw> */
    orc_div_x(m, n, k, p->h, dux, duy, t1);
    if (l > 0) orc_div_G(m, n, k, l, p->edges, p->cost, dw, t2);
    for (size_t q = 0; q < Pk; ++q) cross += (phi1[q] - phi[q]) * (t1[q] + (l > 0 ? t2[q] : 0.0));

    for (size_t q = 0; q < P; ++q) {
        prim += orc_norm_u(p->unorm, k, ux1 + q * (size_t)k, uy1 + q * (size_t)k);
        if (l > 0) prim += p->alpha * orc_norm_w(p->wnorm, l, w1 + q * (size_t)l);
    }
    if (p->eps > 0.0) {
        double sq = 0.0;
        for (size_t q = 0; q < Pk; ++q) sq += ux1[q] * ux1[q] + uy1[q] * uy1[q];
        for (size_t q = 0; q < Pl; ++q) sq += w1[q] * w1[q];
        prim += p->eps * sq;
    }
    orc_div_x(m, n, k, p->h, ux1, uy1, t1);
    if (l > 0) orc_div_G(m, n, k, l, p->edges, p->cost, w1, t2);
    for (size_t q = 0; q < Pk; ++q) {
        double r = t1[q] + (l > 0 ? t2[q] : 0.0) + f[q];
        mass += r * r;
        dual += phi1[q] * f[q];
        ff += f[q] * f[q];
    }
    out[0] = su / p->mu + (l > 0 ? sw / p->nu : 0.0) + sp / p->tau - 2.0 * cross;
    out[1] = prim;
    out[2] = dual;
    out[3] = mass;
    out[4] = ff;
    free(dux);
    free(duy);
    free(dw);
    free(t1);
    free(t2);
}

/* --------------------------------------------------------------- driver */

/* Runs the method from the state (phi, ux, uy, w), which it overwrites with
 * the last iterate.  Ghost components of u are forced to zero first.  Stops
 * after max_iters iterations, or at the first check (every check_every
 * iterations) whose sqrt(R/R0) <= tol when tol > 0.  A check is also taken
 * after the last iteration.  hist (nullable) receives sqrt(R/R0) at every
 * check, up to hist_cap entries.  Returns the number of checks taken. */
int orc_solve(const orc_problem *pin, const double *f, double *phi, double *ux, double *uy, double *w,
              int64_t max_iters, double tol, int check_every, orc_info *info, double *hist, int hist_cap)
{
    orc_problem p = *pin;
    int m = p.m, n = p.n, k = p.k, l = p.l;
    size_t P = (size_t)m * (size_t)n, Pk = P * (size_t)k, Pl = P * (size_t)(l > 0 ? l : 1);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j)
            for (int c = 0; c < k; ++c) {
                if (i == m - 1) ux[I3(i, j, c, n, k)] = 0.0;
                if (j == n - 1) uy[I3(i, j, c, n, k)] = 0.0;
            }
    double *phi1 = (double *)malloc(sizeof(double) * Pk), *ux1 = (double *)malloc(sizeof(double) * Pk);
    double *uy1 = (double *)malloc(sizeof(double) * Pk), *w1 = (double *)calloc(Pl, sizeof(double));
    work_t W;
    work_alloc(&p, &W);
    double ff = 0.0;
    for (size_t q = 0; q < Pk; ++q) ff += f[q] * f[q];
    double R0 = p.tau * ff;
    if (check_every <= 0) check_every = 64;

    memset(info, 0, sizeof(*info));
    int nchecks = 0;
    for (int64_t it = 1; it <= max_iters; ++it) {
        pdhg_step(&p, f, phi, ux, uy, w, phi1, ux1, uy1, w1, &W);
        int check = (it % check_every == 0) || (it == max_iters);
        if (check) {
            double met[5];
            orc_metrics(&p, f, phi, ux, uy, w, phi1, ux1, uy1, w1, met);
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
        memcpy(phi, phi1, sizeof(double) * Pk);
        memcpy(ux, ux1, sizeof(double) * Pk);
        memcpy(uy, uy1, sizeof(double) * Pk);
        if (l > 0) memcpy(w, w1, sizeof(double) * P * (size_t)l);
        if (check && tol > 0.0 && info->residual <= tol) {
            info->converged = 1;
            break;
        }
    }
    work_free(&W);
    free(phi1);
    free(ux1);
    free(uy1);
    free(w1);
    return nchecks;
}

/* One bare iteration (for first-iterate and operator tests). */
void orc_step(const orc_problem *p, const double *f, const double *phi, const double *ux, const double *uy,
              const double *w, double *phi1, double *ux1, double *uy1, double *w1)
{
    work_t W;
    work_alloc(p, &W);
    pdhg_step(p, f, phi, ux, uy, w, phi1, ux1, uy1, w1, &W);
    work_free(&W);
}
