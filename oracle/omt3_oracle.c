/*
 * Oracle for the vector OMT method on three-dimensional grids.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow FP64 single-threaded reference for
 * the HIP path's 3-D kernels; loaded only by the test-suite and the
 * benchmark's CPU-baseline leg.  Shares nothing with the HIP path.
 *
 * The paper states its method on 2-D grids and leaves 3-D imaging as future
 * work (Sec. 8.2).  The 3-D problem here is its axis-by-axis extension:
 *   - the staggered discretisation of App. A on an m x n x p grid: u has
 *     three components per channel, u_x on cell faces between i and i+1,
 *     u_y between j and j+1, u_z between z and z+1; the ghost components
 *     u_x(m-1, ., .), u_y(., n-1, .), u_z(., ., p-1) are zero and there is
 *     no flux through the boundary;
 *   - grad phi by forward differences, div_x by backward differences, both
 *     divided by h = 1/(max(m, n, p) - 1) unless given;
 *   - the norms of Sec. 6.2 with the spatial vector (u_x, u_y, u_z):
 *     ||u||_{1,2} sums over channels the Euclidean norm of that 3-vector;
 *     ||u||_1 sums the moduli of all 3k components; ||u||_2 is the
 *     Euclidean norm of all 3k;
 *   - the iteration of Sec. 7.2 unchanged, with the step rule carried over:
 *     the 3-D Neumann Laplacian has largest eigenvalue below 12/h^2 (8/h^2
 *     in 2-D), so mu = h^2/(48 tau) (h^2/(24 tau) without edges) keeps
 *     tau mu lambda_max(-Delta_x) at the 2-D rule's 1/4 (1/2), and
 *     nu = 1/(4 tau lambda_max(-Delta_G)) is unchanged;
 *   - R^k (Sec. 6.1 with 1/nu on the w block), the objectives and the
 *     constraint residual as in 2-D, quadratic regularisation (Sec. 9) as
 *     in 2-D.
 * Graph routines (Sec. 3.1) and the scalar / vector shrinks (App. B) are
 * the 2-D oracle's, in omt_oracle.c.
 *
 * Layout: [i][j][z][c], channel fastest: phi, f, u_x, u_y, u_z m*n*p*k;
 * w m*n*p*l.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* from omt_oracle.c */
void orc_incidence(int k, int l, const int *edges, double *D);
double orc_graph_lambda_max(int k, int l, const int *edges, const double *cost);
double orc_shrink1(double x, double t);
void orc_shrink2(int d, double *x, double t);
double orc_norm_w(int wnorm, int l, const double *w);
void orc_shrink_w(int wnorm, int l, double *w, double t);

typedef struct {
    int m, n, p, k, l;
    const int *edges;
    const double *cost;
    double alpha, tau, mu, nu, h;
    int unorm, wnorm;
    double eps;
} orc3_problem;

typedef struct {
    int64_t iters;
    double R, residual, primal, dual, rel_gap, mass_residual;
    int converged;
} orc3_info;

#define ID4(i, j, z, c, n, p, k) \
    (((((size_t)(i)) * (size_t)(n) + (size_t)(j)) * (size_t)(p) + (size_t)(z)) * (size_t)(k) + (size_t)(c))

/* Step sizes: the 2-D rule of Sec. 7.1 / 7.2 carried to 3-D (see above). */
void orc3_default_steps(orc3_problem *q)
{
    int side = q->m;
    if (q->n > side) side = q->n;
    if (q->p > side) side = q->p;
    if (q->h <= 0.0) q->h = 1.0 / (double)(side - 1);
    if (q->l == 0) {
        if (q->mu <= 0.0) q->mu = q->h * q->h / (24.0 * q->tau);
        q->nu = 0.0;
    } else {
        if (q->mu <= 0.0) q->mu = q->h * q->h / (48.0 * q->tau);
        if (q->nu <= 0.0) q->nu = 1.0 / (4.0 * q->tau * orc_graph_lambda_max(q->k, q->l, q->edges, q->cost));
    }
}

/* Forward differences, zero on the ghost face of each axis (App. A). */
void orc3_grad(int m, int n, int p, int k, double h, const double *phi, double *gx, double *gy, double *gz)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j)
            for (int z = 0; z < p; ++z)
                for (int c = 0; c < k; ++c) {
                    const size_t o = ID4(i, j, z, c, n, p, k);
                    gx[o] = i < m - 1 ? (phi[ID4(i + 1, j, z, c, n, p, k)] - phi[o]) / h : 0.0;
                    gy[o] = j < n - 1 ? (phi[ID4(i, j + 1, z, c, n, p, k)] - phi[o]) / h : 0.0;
                    gz[o] = z < p - 1 ? (phi[ID4(i, j, z + 1, c, n, p, k)] - phi[o]) / h : 0.0;
                }
}

/* Backward differences with zero flux through the boundary (App. A). */
void orc3_div(int m, int n, int p, int k, double h, const double *ux, const double *uy, const double *uz, double *out)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j)
            for (int z = 0; z < p; ++z)
                for (int c = 0; c < k; ++c) {
                    const size_t o = ID4(i, j, z, c, n, p, k);
                    const double xr = i < m - 1 ? ux[o] : 0.0, xl = i > 0 ? ux[ID4(i - 1, j, z, c, n, p, k)] : 0.0;
                    const double yr = j < n - 1 ? uy[o] : 0.0, yl = j > 0 ? uy[ID4(i, j - 1, z, c, n, p, k)] : 0.0;
                    const double zr = z < p - 1 ? uz[o] : 0.0, zl = z > 0 ? uz[ID4(i, j, z - 1, c, n, p, k)] : 0.0;
                    out[o] = (xr - xl + yr - yl + zr - zl) / h;
                }
}

/* grad_G and div_G at every pixel (Sec. 3.1): (grad_G x)_e = (D^T x)_e / c_e,
 * div_G y = -D diag(1/c) y. */
static void graph_grad_all(size_t P, int k, int l, const double *D, const double *cost, const double *x, double *y)
{
    for (size_t q = 0; q < P; ++q)
        for (int e = 0; e < l; ++e) {
            double s = 0.0;
            for (int c = 0; c < k; ++c) s += D[c * l + e] * x[q * (size_t)k + c];
            y[q * (size_t)l + e] = s / cost[e];
        }
}

static void graph_div_all(size_t P, int k, int l, const double *D, const double *cost, const double *y, double *x)
{
    for (size_t q = 0; q < P; ++q)
        for (int c = 0; c < k; ++c) {
            double s = 0.0;
            for (int e = 0; e < l; ++e) s += D[c * l + e] * (y[q * (size_t)l + e] / cost[e]);
            x[q * (size_t)k + c] = -s;
        }
}

/* Shrink of the flux block of one pixel: k channels, three directions. */
static void shrink_u3(int unorm, int k, double *bx, double *by, double *bz, double t)
{
    if (unorm == 0) { /* per channel, the spatial 3-vector */
        for (int c = 0; c < k; ++c) {
            double v[3] = {bx[c], by[c], bz[c]};
            orc_shrink2(3, v, t);
            bx[c] = v[0];
            by[c] = v[1];
            bz[c] = v[2];
        }
    } else if (unorm == 1) { /* every component */
        for (int c = 0; c < k; ++c) {
            bx[c] = orc_shrink1(bx[c], t);
            by[c] = orc_shrink1(by[c], t);
            bz[c] = orc_shrink1(bz[c], t);
        }
    } else { /* all 3k components at once */
        double *v = (double *)malloc(sizeof(double) * 3 * (size_t)k);
        for (int c = 0; c < k; ++c) {
            v[c] = bx[c];
            v[k + c] = by[c];
            v[2 * k + c] = bz[c];
        }
        orc_shrink2(3 * k, v, t);
        for (int c = 0; c < k; ++c) {
            bx[c] = v[c];
            by[c] = v[k + c];
            bz[c] = v[2 * k + c];
        }
        free(v);
    }
}

static double norm_u3(int unorm, int k, const double *bx, const double *by, const double *bz)
{
    double s = 0.0;
    if (unorm == 0) {
        for (int c = 0; c < k; ++c) s += sqrt(bx[c] * bx[c] + by[c] * by[c] + bz[c] * bz[c]);
    } else if (unorm == 1) {
        for (int c = 0; c < k; ++c) s += fabs(bx[c]) + fabs(by[c]) + fabs(bz[c]);
    } else {
        for (int c = 0; c < k; ++c) s += bx[c] * bx[c] + by[c] * by[c] + bz[c] * bz[c];
        s = sqrt(s);
    }
    return s;
}

/* One iteration of Sec. 7.2 on the 3-D grid:
 *   u1  = shrink_u(u + mu grad phi, mu)
 *   w1  = shrink_w(w + nu grad_G phi, alpha nu)
 *   phi1 = phi + tau (div_x(2 u1 - u) + div_G(2 w1 - w) + f)            */
void orc3_step(const orc3_problem *q, const double *f, const double *phi, const double *ux, const double *uy,
               const double *uz, const double *w, double *phi1, double *ux1, double *uy1, double *uz1, double *w1)
{
    const int m = q->m, n = q->n, p = q->p, k = q->k, l = q->l;
    const size_t P = (size_t)m * n * p, Pk = P * (size_t)k, Pl = P * (size_t)(l > 0 ? l : 1);
    double *gx = calloc(Pk, sizeof(double)), *gy = calloc(Pk, sizeof(double)), *gz = calloc(Pk, sizeof(double));
    double *bx = calloc(Pk, sizeof(double)), *by = calloc(Pk, sizeof(double)), *bz = calloc(Pk, sizeof(double));
    double *dx = calloc(Pk, sizeof(double)), *dg = calloc(Pk, sizeof(double));
    double *gG = calloc(Pl, sizeof(double)), *bw = calloc(Pl, sizeof(double));
    double *D = calloc((size_t)(k * l > 0 ? k * l : 1), sizeof(double));

    orc3_grad(m, n, p, k, q->h, phi, gx, gy, gz);
    for (size_t s = 0; s < P; ++s) {
        double *ax = ux1 + s * (size_t)k, *ay = uy1 + s * (size_t)k, *az = uz1 + s * (size_t)k;
        for (int c = 0; c < k; ++c) {
            const size_t o = s * (size_t)k + (size_t)c;
            ax[c] = ux[o] + q->mu * gx[o];
            ay[c] = uy[o] + q->mu * gy[o];
            az[c] = uz[o] + q->mu * gz[o];
        }
        shrink_u3(q->unorm, k, ax, ay, az, q->mu);
        if (q->eps > 0.0)
            for (int c = 0; c < k; ++c) {
                ax[c] /= 1.0 + 2.0 * q->mu * q->eps;
                ay[c] /= 1.0 + 2.0 * q->mu * q->eps;
                az[c] /= 1.0 + 2.0 * q->mu * q->eps;
            }
    }
    if (l > 0) {
        orc_incidence(k, l, q->edges, D);
        graph_grad_all(P, k, l, D, q->cost, phi, gG);
        for (size_t s = 0; s < P; ++s) {
            double *b = w1 + s * (size_t)l;
            for (int e = 0; e < l; ++e) b[e] = w[s * (size_t)l + e] + q->nu * gG[s * (size_t)l + e];
            orc_shrink_w(q->wnorm, l, b, q->alpha * q->nu);
            if (q->eps > 0.0)
                for (int e = 0; e < l; ++e) b[e] /= 1.0 + 2.0 * q->nu * q->eps;
        }
    }
    for (size_t s = 0; s < Pk; ++s) {
        bx[s] = 2.0 * ux1[s] - ux[s];
        by[s] = 2.0 * uy1[s] - uy[s];
        bz[s] = 2.0 * uz1[s] - uz[s];
    }
    orc3_div(m, n, p, k, q->h, bx, by, bz, dx);
    if (l > 0) {
        for (size_t s = 0; s < P * (size_t)l; ++s) bw[s] = 2.0 * w1[s] - w[s];
        graph_div_all(P, k, l, D, q->cost, bw, dg);
    }
    for (size_t s = 0; s < Pk; ++s) phi1[s] = phi[s] + q->tau * (dx[s] + dg[s] + f[s]);
    free(gx), free(gy), free(gz), free(bx), free(by), free(bz), free(dx), free(dg), free(gG), free(bw), free(D);
}

/* Check quantities of the step old -> new (Sec. 6.1; App. A objectives):
 * out = {R^k, primal, <phi1, f>, ||div_x u1 + div_G w1 + f||^2, ||f||^2}. */
void orc3_metrics(const orc3_problem *q, const double *f, const double *phi, const double *ux, const double *uy,
                  const double *uz, const double *w, const double *phi1, const double *ux1, const double *uy1,
                  const double *uz1, const double *w1, double *out)
{
    const int m = q->m, n = q->n, p = q->p, k = q->k, l = q->l;
    const size_t P = (size_t)m * n * p, Pk = P * (size_t)k, Pl = P * (size_t)l;
    double *ddx = calloc(Pk, sizeof(double)), *ddy = calloc(Pk, sizeof(double)), *ddz = calloc(Pk, sizeof(double));
    double *dw = calloc(Pl > 0 ? Pl : 1, sizeof(double)), *t1 = calloc(Pk, sizeof(double));
    double *t2 = calloc(Pk, sizeof(double)), *D = calloc((size_t)(k * l > 0 ? k * l : 1), sizeof(double));
    double su = 0, sw = 0, sp = 0, cross = 0, prim = 0, dual = 0, mass = 0, ff = 0;
    if (l > 0) orc_incidence(k, l, q->edges, D);
    for (size_t s = 0; s < Pk; ++s) {
        ddx[s] = ux1[s] - ux[s];
        ddy[s] = uy1[s] - uy[s];
        ddz[s] = uz1[s] - uz[s];
        su += ddx[s] * ddx[s] + ddy[s] * ddy[s] + ddz[s] * ddz[s];
        const double dp = phi1[s] - phi[s];
        sp += dp * dp;
    }
    for (size_t s = 0; s < Pl; ++s) {
        dw[s] = w1[s] - w[s];
        sw += dw[s] * dw[s];
    }
    orc3_div(m, n, p, k, q->h, ddx, ddy, ddz, t1);
    if (l > 0) graph_div_all(P, k, l, D, q->cost, dw, t2);
    for (size_t s = 0; s < Pk; ++s) cross += (phi1[s] - phi[s]) * (t1[s] + t2[s]);
    for (size_t s = 0; s < P; ++s) {
        prim += norm_u3(q->unorm, k, ux1 + s * (size_t)k, uy1 + s * (size_t)k, uz1 + s * (size_t)k);
        if (l > 0) prim += q->alpha * orc_norm_w(q->wnorm, l, w1 + s * (size_t)l);
    }
    if (q->eps > 0.0) {
        double sq = 0.0;
        for (size_t s = 0; s < Pk; ++s) sq += ux1[s] * ux1[s] + uy1[s] * uy1[s] + uz1[s] * uz1[s];
        for (size_t s = 0; s < Pl; ++s) sq += w1[s] * w1[s];
        prim += q->eps * sq;
    }
    orc3_div(m, n, p, k, q->h, ux1, uy1, uz1, t1);
    for (size_t s = 0; s < Pk; ++s) t2[s] = 0.0;
    if (l > 0) graph_div_all(P, k, l, D, q->cost, w1, t2);
    for (size_t s = 0; s < Pk; ++s) {
        const double r = t1[s] + t2[s] + f[s];
        mass += r * r;
        dual += phi1[s] * f[s];
        ff += f[s] * f[s];
    }
    out[0] = su / q->mu + (l > 0 ? sw / q->nu : 0.0) + sp / q->tau - 2.0 * cross;
    out[1] = prim;
    out[2] = dual;
    out[3] = mass;
    out[4] = ff;
    free(ddx), free(ddy), free(ddz), free(dw), free(t1), free(t2), free(D);
}

/* Runs the method from the given state (overwritten with the last iterate;
 * ghost components are zeroed first), checks every check_every iterations
 * and after the last, stops at the first check with sqrt(R/R0) <= tol when
 * tol > 0.  Returns the number of checks taken. */
int orc3_solve(const orc3_problem *q, const double *f, double *phi, double *ux, double *uy, double *uz, double *w,
               int64_t max_iters, double tol, int check_every, orc3_info *info)
{
    const int m = q->m, n = q->n, p = q->p, k = q->k, l = q->l;
    const size_t P = (size_t)m * n * p, Pk = P * (size_t)k, Pl = P * (size_t)(l > 0 ? l : 1);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j)
            for (int z = 0; z < p; ++z)
                for (int c = 0; c < k; ++c) {
                    if (i == m - 1) ux[ID4(i, j, z, c, n, p, k)] = 0.0;
                    if (j == n - 1) uy[ID4(i, j, z, c, n, p, k)] = 0.0;
                    if (z == p - 1) uz[ID4(i, j, z, c, n, p, k)] = 0.0;
                }
    double *phi1 = malloc(sizeof(double) * Pk), *ux1 = malloc(sizeof(double) * Pk);
    double *uy1 = malloc(sizeof(double) * Pk), *uz1 = malloc(sizeof(double) * Pk);
    double *w1 = calloc(Pl, sizeof(double));
    double ff = 0.0;
    for (size_t s = 0; s < Pk; ++s) ff += f[s] * f[s];
    const double R0 = q->tau * ff;
    if (check_every <= 0) check_every = 64;
    memset(info, 0, sizeof(*info));
    int nchecks = 0;
    for (int64_t it = 1; it <= max_iters; ++it) {
        orc3_step(q, f, phi, ux, uy, uz, w, phi1, ux1, uy1, uz1, w1);
        const int check = (it % check_every == 0) || (it == max_iters);
        if (check) {
            double met[5];
            orc3_metrics(q, f, phi, ux, uy, uz, w, phi1, ux1, uy1, uz1, w1, met);
            info->iters = it;
            info->R = met[0];
            info->residual = R0 > 0 ? sqrt(fmax(met[0], 0.0) / R0) : 0.0;
            info->primal = met[1];
            info->dual = met[2];
            info->rel_gap = met[1] > 0 ? (met[1] - met[2]) / met[1] : 0.0;
            info->mass_residual = ff > 0 ? sqrt(met[3] / ff) : 0.0;
            ++nchecks;
        }
        memcpy(phi, phi1, sizeof(double) * Pk);
        memcpy(ux, ux1, sizeof(double) * Pk);
        memcpy(uy, uy1, sizeof(double) * Pk);
        memcpy(uz, uz1, sizeof(double) * Pk);
        if (l > 0) memcpy(w, w1, sizeof(double) * P * (size_t)l);
        if (check && tol > 0.0 && info->residual <= tol) {
            info->converged = 1;
            break;
        }
    }
    free(phi1), free(ux1), free(uy1), free(uz1), free(w1);
    return nchecks;
}
