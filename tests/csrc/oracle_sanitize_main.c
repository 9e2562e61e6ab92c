/* Drives the oracle on a few small problems so that it can be run under
 * AddressSanitizer and UndefinedBehaviorSanitizer (host code only). */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int m, n, k, l;
    const int *edges;
    const double *cost;
    double alpha, tau, mu, nu, h;
    int unorm, wnorm;
    double eps;
} orc_problem;
typedef struct {
    int64_t iters;
    double R, residual, primal, dual, rel_gap, mass_residual;
    int converged;
} orc_info;

void orc_default_steps(orc_problem *p);
double orc_prepare_f(int m, int n, int k, int l, const int *edges, const double *lam0, const double *lam1, double *f);
int orc_solve(const orc_problem *p, const double *f, double *phi, double *ux, double *uy, double *w, int64_t max_iters,
              double tol, int check_every, orc_info *info, double *hist, int hist_cap);

static double frand(unsigned *s)
{
    *s = *s * 1103515245u + 12345u;
    return ((*s >> 8) & 0xffff) / 65536.0 + 0.01;
}

int main(void)
{
    const int tri[6] = {0, 1, 0, 2, 1, 2};
    const double cost[3] = {1.0, 0.5, 2.0};
    const int shapes[][4] = {{2, 2, 3, 3}, {5, 7, 3, 3}, {9, 4, 1, 0}, {6, 6, 2, 1}};
    unsigned seed = 7u;
    for (int s = 0; s < 4; ++s) {
        for (int unorm = 0; unorm < 3; ++unorm) {
            const int m = shapes[s][0], n = shapes[s][1], k = shapes[s][2], l = shapes[s][3];
            const size_t P = (size_t)m * n;
            double *a = malloc(sizeof(double) * P * k), *b = malloc(sizeof(double) * P * k);
            double *f = malloc(sizeof(double) * P * k), *phi = calloc(P * k, sizeof(double));
            double *ux = calloc(P * k, sizeof(double)), *uy = calloc(P * k, sizeof(double));
            double *w = calloc(P * (l > 0 ? l : 1), sizeof(double));
            double sa = 0, sb = 0;
            for (size_t q = 0; q < P * k; ++q) {
                a[q] = frand(&seed);
                b[q] = frand(&seed);
                sa += a[q];
                sb += b[q];
            }
            for (size_t q = 0; q < P * k; ++q) b[q] *= sa / sb;
            orc_problem p = {m, n, k, l, tri, cost, 0.7, 1.0, 0.0, 0.0, 0.0, unorm, unorm % 2, 0.1 * unorm};
            orc_default_steps(&p);
            orc_prepare_f(m, n, k, l, tri, a, b, f);
            orc_info info;
            double hist[64];
            orc_solve(&p, f, phi, ux, uy, w, 500, 0.0, 16, &info, hist, 64);
            printf("%dx%dx%d u%d: V %.9f residual %.3e\n", m, n, k, unorm, info.primal, info.residual);
            free(a);
            free(b);
            free(f);
            free(phi);
            free(ux);
            free(uy);
            free(w);
        }
    }
    return 0;
}
