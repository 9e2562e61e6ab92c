/*
 * Matrix optimal mass transport (M-OMT) on a 2-D grid: the first-order
 * primal-dual method of Ryu, Chen, Li and Osher, "Vector and Matrix Optimal
 * Mass Transport" (arXiv 1712.10279), Sec. 4 and Sec. 7.3, on one MI355X.
 *
 * Every pixel carries a k x k Hermitian matrix density Lambda(x) (a real
 * symmetric one in the real mode).  The method iterates
 *   U   <- shrink_u(U + mu grad_x Phi, mu)            U = (U_x, U_y), Hermitian
 *   W   <- shrink_w(W + nu grad_L Phi, alpha nu)      W = (W_1..W_l), skew-Hermitian
 *   Phi <- Phi + tau (div_x(2U' - U) + div_L(2W' - W) + Lambda1 - Lambda0)
 * with grad_L X = (L_s X - X L_s)_s and div_L Z = sum_s (-L_s Z_s + Z_s L_s)
 * (Sec. 4.1), the staggered grid and ghost cells of App. A applied entry by
 * entry, mu = h^2/(32 tau), nu = 1/(4 tau lambda_max(-Delta_L)) (Sec. 7.3),
 * and the residual, checks and stopping rule of omt_solve.
 *
 * The matrices are carried in orthonormal real coordinates of the Hermitian
 * and skew-Hermitian spaces (Hilbert-Schmidt inner product, Sec. 4), so that
 * each iteration is one pass of the fused vector kernels with a dense k^2 x
 * l k^2 operator: the same HBM-bound step, no per-pixel matrix algebra.
 *
 * All calls return an omt_status (include/omt.h); omt_last_error() gives the
 * detail.  Buffers follow omt_create: the workspace is the caller's device
 * memory of omt_matrix_workspace_bytes() bytes, 256-byte aligned, and must
 * outlive the handle; all work is enqueued on the caller's stream.
 */
#ifndef OMT_MATRIX_H
#define OMT_MATRIX_H

#include "omt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct omt_mctx *omt_matrix_handle;

/* Norms of Sec. 6.2 on H^2 (U) and S^l (W). */
typedef enum {
    OMT_M_FRO = 0, /* ||.||_2: Frobenius norm of the whole block                  */
    OMT_M_L1 = 1,  /* ||.||_1: sum of the moduli of all entries                   */
    OMT_M_NUC = 2  /* ||.||_{1,nuc}: sum of nuclear norms (not for complex 3 x 3)      */
} omt_mnorm;

typedef struct {
    int32_t m, n;       /* grid rows / columns, >= 2                               */
    int32_t k;          /* matrix order 2 or 3 (real or complex)                   */
    int32_t n_L;        /* l >= 1 matrices L_s (real k=2, k=3: <= 3; complex: <= 2) */
    const double *L;    /* host, l Hermitian k x k matrices, row-major, complex
                           entries as (re, im) pairs (l*k*k*2 doubles)              */
    int32_t real;       /* 1: L and the data are real symmetric (imaginary parts of
                           L must be 0; data are given as real entries)             */
    double alpha;       /* > 0, weight of the W term                               */
    double tau;         /* > 0, dual step                                          */
    double mu, nu;      /* 0: the rule of Sec. 7.3; else checked like omt_params   */
    double h;           /* 0: 1/(max(m,n)-1)                                       */
    omt_mnorm unorm, wnorm;
    omt_dtype dtype;    /* of the data, state and iterates                         */
    int32_t flags;      /* OMT_FLAG_COMPENSATED_PHI (FP32 only)                    */
    int32_t rows_per_wave; /* 0: library default                                   */
    int32_t tblock;     /* iterations per pass over HBM: 1 or 2 (2: FP32 with the
                           Frobenius or entry-wise norms, k x k coordinates <= 6, else
                           OMT_EUNSUPPORTED); 0: 2 where allowed on grids whose
                           single-iteration strips take 4 or more rows, else 1.  Every
                           value gives the same iterates bit for bit.             */
} omt_matrix_params;

/* Defaults: alpha 1, tau 1, Frobenius U, entry-wise W (the setting of the
 * diffusion-tensor example, Sec. 8.2), FP32, real mode off. */
omt_status omt_matrix_params_init(omt_matrix_params *p);

/* Host-only validation and the resolved h, mu, nu, lambda_max(-Delta_L)
 * (from the k^2 x k^2 matrix of -Delta_L, Sec. 7.3) and the coordinate
 * counts per pixel of Phi and of W (any output may be NULL).  Errors:
 * OMT_EINVAL for bad sizes, norms, steps or a non-Hermitian L; OMT_EGRAPH
 * when grad_L annihilates more than the multiples of I (the standing
 * assumption of Sec. 4.1); OMT_EUNSUPPORTED for shapes not compiled. */
omt_status omt_matrix_resolve(const omt_matrix_params *p, double *h, double *mu, double *nu, double *lambda_max,
                              int32_t *coords, int32_t *w_coords);
omt_status omt_matrix_workspace_bytes(const omt_matrix_params *p, size_t *bytes);

/* Lambda0, Lambda1: device, m*n*k*k entries per density in [i][j][a][b]
 * order of the params' dtype (complex: (re, im) pairs; real mode: real
 * entries); only the diagonal and upper triangle are read.  The total trace
 * must agree to 1e-6 relative (else OMT_EMASS); f = Lambda1 - Lambda0 has
 * (tr sum f / (m n k)) I removed.  Non-finite inputs give OMT_EINVAL. */
omt_status omt_matrix_create(const omt_matrix_params *p, const void *Lambda0, const void *Lambda1, void *workspace,
                             size_t ws_bytes, void *stream, omt_matrix_handle *out);

/* As omt_solve / omt_distance: M is ||U||_u + alpha ||W||_w of the iterate. */
omt_status omt_matrix_solve(omt_matrix_handle h, int64_t max_iters, double tol, int32_t check_every,
                            omt_info *info);
omt_status omt_matrix_distance(omt_matrix_handle h, double *M, omt_info *info);

/* dM/dLambda0 = Phi_e and dM/dLambda1 = -Phi_e with Phi_e = -Phi minus
 * (mean trace / k) I (dual problem, Sec. 4.2), in the layout of the data
 * (device, m*n*k*k entries; either may be NULL). */
omt_status omt_matrix_grad(omt_matrix_handle h, void *dM_dLambda0, void *dM_dLambda1);

/* Current iterate as matrices (device, any may be NULL): Phi and U_x, U_y
 * m*n*k*k entries each, W m*n*l*k*k entries ([i][j][s][a][b]). */
omt_status omt_matrix_get_state(omt_matrix_handle h, void *Phi, void *Ux, void *Uy, void *W);

/* As omt_time_steps for the coordinate problem, in the solve's launch shape
 * (T = tblock or its default iterations per launch; n must be a multiple of
 * T): mean microseconds per step launch over n / T timed launches. */
omt_status omt_matrix_time_steps(omt_matrix_handle h, int32_t rows_per_wave, int64_t n, double *us_per_launch);

omt_status omt_matrix_destroy(omt_matrix_handle h);

#ifdef __cplusplus
}
#endif

#endif /* OMT_MATRIX_H */
