/*
 * omt.h -- C ABI of the MI355X (gfx950) solver for vector-valued optimal
 * mass transport on a regular 2-D grid, after Ryu, Chen, Li and Osher,
 * "Vector and Matrix Optimal Mass Transport: Theory, Algorithm, and
 * Applications" (arXiv 1712.10279).
 *
 * The library solves the discrete vector-OMT problem of App. A,
 *
 *     V(rho0, rho1) = min ||u||_u + alpha ||w||_w
 *                     s.t. div_x u + div_G w = rho0 - rho1,
 *
 * (the continuous problem and its dual are stated in Sec. 3.2) with the
 * first-order primal-dual method of Sec. 7.2 (Sec. 7.1 when the channel graph
 * has no edges):
 *
 *     u   <- shrink_u(u + mu grad_x phi, mu)
 *     w   <- shrink_w(w + nu grad_G phi, alpha nu)
 *     phi <- phi + tau (div_x(2u' - u) + div_G(2w' - w) + rho1 - rho0).
 *
 * Conventions shared by every call:
 *   - Densities are cell masses (finite-volume integrals, App. A) in the
 *     paper's layout: m x n x k, channel index fastest, row i (the paper's x)
 *     slowest.  Grid spacing h = 1/(max(m,n)-1) unless given.
 *   - Only rho1 - rho0 enters the discrete problem, so signed inputs are
 *     accepted.  Per mass class (connected component of the channel graph)
 *     the two masses must agree to 1e-6 relative; the difference that is
 *     left is removed from rho1 - rho0 in FP64 before solving.
 *   - Device pointers are HIP device addresses on the current device; host
 *     pointers are ordinary process memory.  The caller owns every buffer.
 *   - All device work of a handle is enqueued on the stream given at create.
 *   - Every call returns an omt_status; no exception crosses the ABI.  A
 *     human-readable detail of the last failure on the calling thread is
 *     available from omt_last_error().
 *   - Exported potential: Phi = -phi with its mean over each mass class
 *     removed.  By the dual problem of Sec. 3.2, V = <phi, rho1 - rho0> at
 *     optimum, so dV/drho0 = Phi and dV/drho1 = -Phi.
 *   - Diagnostics (environment, read once per process): OMT_LOG=1 prints
 *     every failure to stderr, 2 also one line per solve (iterations, time,
 *     residual) and the batch's progress, 3 also one line per check;
 *     OMT_VERBOSE alone means 2.  Solves, check intervals and the other
 *     entry points are ROCTx ranges (rocprofv3 --marker-trace).
 *     OMT_POISON=1 fills the padding of every field (the columns past n of
 *     each row and the gaps between planes) with NaN at create, so that a
 *     kernel that read memory outside the grid would turn its results NaN.
 */
#ifndef OMT_H
#define OMT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OMT_OK = 0,
    OMT_EINVAL = 1,        /* bad argument: sizes, NULL, NaN/Inf data, tau/alpha <= 0, ... */
    OMT_EGRAPH = 2,        /* bad channel graph: a >= b, node out of range, duplicate edge, c <= 0 */
    OMT_EMASS = 3,         /* the two densities carry different mass in some mass class */
    OMT_ESTEP = 4,         /* given mu/nu violate tau mu 8/h^2 + tau nu lambda_max < 1 (Sec. 7.2) */
    OMT_ENOMEM = 5,        /* workspace smaller than omt_workspace_bytes() */
    OMT_EDEVICE = 6,       /* a HIP call failed */
    OMT_ENOTCONV = 7,      /* tol not reached within max_iters; outputs are valid */
    OMT_EDIVERGED = 8,     /* a check found a non-finite residual */
    OMT_EUNSUPPORTED = 9   /* valid request the library is not compiled for (e.g. k > 8) */
} omt_status;

/* Norms of Sec. 6.2. */
typedef enum {
    OMT_U_L12 = 0, /* sum over channels of the Euclidean norm of (u_x, u_y): the default */
    OMT_U_L1 = 1,  /* sum of absolute values of all 2k flux components            */
    OMT_U_L2 = 2   /* Euclidean norm of all 2k flux components of a pixel          */
} omt_unorm;

typedef enum {
    OMT_W_L1 = 0, /* sum of absolute values of the l transfers: the default */
    OMT_W_L2 = 1  /* Euclidean norm of the l transfers of a pixel            */
} omt_wnorm;

typedef enum { OMT_F32 = 0, OMT_F64 = 1 } omt_dtype;

/* Store the FP32 potential as an unevaluated sum hi + lo of two floats
 * updated with an error-free addition, so that increments far below the
 * FP32 spacing of phi are not lost. Ignored for OMT_F64. */
#define OMT_FLAG_COMPENSATED_PHI 1u

/* Largest channel count compiled into the library. */
#define OMT_MAX_CHANNELS 8

typedef struct {
    int32_t m, n;              /* grid rows and columns, each >= 2 */
    int32_t k;                 /* channels, 1 <= k <= OMT_MAX_CHANNELS */
    int32_t n_edges;           /* l >= 0 edges of the channel graph; 0 gives scalar OMT per channel */
    const int32_t *edges;      /* host, 2*l node indices (a_e, b_e) with 0 <= a_e < b_e < k (Sec. 3.1) */
    const double *edge_cost;   /* host, l costs c_e > 0 (edge weight 1/c_e^2), or NULL for all 1 */
    double alpha;              /* > 0, weight of the channel transfer (Sec. 3.2) */
    double tau;                /* > 0, dual step */
    double mu, nu;             /* 0: the rule of Sec. 7.2 (mu = h^2/(32 tau), h^2/(16 tau) if l = 0;
                                  nu = 1/(4 tau lambda_max(-Delta_G))); else checked as OMT_ESTEP says */
    double h;                  /* 0: 1/(max(m,n)-1) */
    int32_t unorm;             /* omt_unorm */
    int32_t wnorm;             /* omt_wnorm */
    int32_t dtype;             /* omt_dtype of inputs, outputs and iterates; reductions are FP64 */
    uint32_t flags;            /* OMT_FLAG_* */
    int32_t tblock;            /* iterations fused per pass over HBM (1, 2, 4, 8; FP64: 1, or 2 for
                                  k <= 3 without a dense graph); 0: the tuned value (omt_autotune,
                                  OMT_TUNE_CACHE), else 2 where compiled on grids whose
                                  single-iteration strips take 4 or more rows per wave (2 or more
                                  in FP64), else 1.
                                  Every value gives the same iterates bit for bit. */
    int32_t rows_per_wave;     /* rows one wavefront streams through; 0 = tuned default */
    double reg_eps;            /* >= 0: quadratic regularisation eps (|u|^2 + |w|^2), Euclidean squares of
                                  all components (Sec. 9); each shrink is then divided by 1 + 2 t eps with
                                  t = mu for u and nu for w.  0 gives the method of Sec. 7.2 exactly. */
    int32_t p;                 /* depth of a 3-D grid (slices along the third axis z); 0 or 1: the 2-D
                                  grid.  The paper states the method in 2-D and names 3-D as future work
                                  (Sec. 8.2); with p > 1 App. A's discretisation is applied along z too:
                                  u gains a third component per channel (u_z, zero on the last slice),
                                  h = 1/(max(m,n,p)-1), and the mu rule becomes h^2/(48 tau) (h^2/(24 tau)
                                  without edges), since the 3-D Laplacian's spectrum reaches 12/h^2 where
                                  the 2-D one reaches 8/h^2.  Densities are then m x n x p x k (channel
                                  fastest, z next), u m x n x p x k x 3, w m x n x p x l.  Compiled for
                                  k = 1 (no edges), k = 2 (one edge) and k = 3 (up to three edges), FP32 or
                                  FP64, one iteration per launch, without the compensated potential;
                                  OMT_EUNSUPPORTED otherwise.  rows_per_wave then counts the slices a
                                  wavefront marches through (0: chosen to fill the chip). */
} omt_params;

typedef struct {
    int64_t iters;          /* iterations done by the solve */
    double residual;        /* sqrt(R^k / R^0), R^k the fixed-point residual of Sec. 6.1 for the last
                               step (with 1/nu on the w block) and R^0 = tau ||rho1 - rho0||^2 */
    double primal;          /* ||u||_u + alpha ||w||_w (+ eps (|u|^2 + |w|^2)) at the last iterate */
    double dual;            /* <phi, rho1 - rho0> at the last iterate (the dual objective when eps = 0) */
    double rel_gap;         /* (primal - dual) / primal, the precision measure of Sec. 8.1 */
    double mass_residual;   /* ||div_x u + div_G w + rho1 - rho0|| / ||rho1 - rho0|| */
    double R;               /* R^k itself */
    int32_t converged;      /* 1 if residual <= tol at a check */
    int32_t checks;         /* checks taken */
} omt_info;

typedef struct omt_ctx *omt_handle;
typedef struct omt_bctx *omt_batch_handle;

/* Fill *p with defaults: alpha 1, tau 1, rule step sizes, ||u||_{1,2},
 * ||w||_1, FP32, no edges.  The caller still sets m, n, k and the graph. */
void omt_params_init(omt_params *p);

/* Host only (no device work).  Validate *p and report the resolved grid
 * spacing and step sizes and lambda_max(-Delta_G) (Sec. 7.2).  Any output
 * pointer may be NULL.  Size limit: the kernels address each field (the k
 * potential planes, the 2k flux planes, the transfer planes) with 32-bit
 * byte offsets, so max(2k, edges compiled) planes of m x ceil64(n) values
 * (4 or 8 bytes each, plus 4352 bytes of skew per plane) must stay below
 * 2 GiB (OMT_EUNSUPPORTED otherwise; at k = 8 in FP32 the largest square
 * grid is 5760 x 5760). */
omt_status omt_resolve_params(const omt_params *p, double *h, double *mu, double *nu, double *lambda_max);

/* Host only.  Bytes of device workspace omt_create needs for *p. */
omt_status omt_workspace_bytes(const omt_params *p, size_t *bytes);

/* Set up one problem.  rho0, rho1: device, m*n*k elements of p->dtype in the
 * paper's layout; they are read during the call and not kept.  workspace:
 * device, >= omt_workspace_bytes() bytes, 256-byte aligned, owned by the
 * caller and kept until omt_destroy.  stream: hipStream_t (NULL = default).
 * The call synchronises the stream once (mass check) and starts from
 * u = w = phi = 0 (Sec. 7.2 leaves the initial guess open). */
omt_status omt_create(const omt_params *p, const void *rho0, const void *rho1, void *workspace,
                      size_t ws_bytes, void *stream, omt_handle *out);

/* Run the method.  max_iters >= 0 iterations at most; tol > 0 stops at the
 * first check with residual <= tol, tol <= 0 runs exactly max_iters.  Checks
 * are taken every check_every iterations (<= 0: 64) and after the last one.
 * Iterations continue from the current state.  info may be NULL.  Returns
 * OMT_ENOTCONV when tol > 0 was not reached (outputs still valid). */
omt_status omt_solve(omt_handle h, int64_t max_iters, double tol, int32_t check_every, omt_info *info);

/* The transport cost V = ||u||_u + alpha ||w||_w of the current iterate
 * (FP64 reduction; the discrete primal objective of App. A).  Also fills
 * *info (nullable) with primal, dual, gap and mass residual of the iterate. */
omt_status omt_distance(omt_handle h, double *V, omt_info *info);

/* Gradients of V: d_rho0 = Phi, d_rho1 = -Phi (see the conventions above);
 * device, m*n*k elements of the handle's dtype, paper layout.  Either may be
 * NULL. */
omt_status omt_grad(omt_handle h, void *d_rho0, void *d_rho1);

/* Copy the state out / in (warm starts; the algorithm of Sec. 7.2 takes
 * initial guesses).  Device, handle dtype, paper layout: phi m*n*k, u
 * m*n*k*2 with the last index 0 for u_x and 1 for u_y, w m*n*l.  Any pointer
 * may be NULL (that part is left alone; on set it is zeroed).  Ghost
 * components (u_x on row m-1, u_y on column n-1, App. A) are zeroed on set. */
omt_status omt_get_state(omt_handle h, void *phi, void *u, void *w);
omt_status omt_set_state(omt_handle h, const void *phi, const void *u, const void *w);

/* Release the handle (host memory only; the workspace stays the caller's). */
omt_status omt_destroy(omt_handle h);

/* ------------------------------------------------------------- batched */

/* Many independent problems of possibly different sizes, channel counts and
 * graphs solved together: each launch advances all unfinished pairs by two
 * iterations (one HBM pass; the checked iteration and an odd one before it
 * by one), or by one if any problem sets tblock = 1, and the launches of a
 * check interval are replayed as one HIP graph.  params[b], rho0[b],
 * rho1[b] as for omt_create (device pointers);
 * one workspace of omt_batch_workspace_bytes().  Compiled problem types:
 * k = 1 without edges, k = 2 with one edge, k = 3 on the triangle or on the
 * path; anything else is OMT_EUNSUPPORTED.  Every problem of a batch shares
 * the dtype and OMT_FLAG_COMPENSATED_PHI (else OMT_EINVAL); each problem's
 * iterates are bit-identical to those of its own omt_solve. */
omt_status omt_batch_workspace_bytes(int32_t B, const omt_params *params, size_t *bytes);
omt_status omt_batch_create(int32_t B, const omt_params *params, const void *const *rho0,
                            const void *const *rho1, void *workspace, size_t ws_bytes, void *stream,
                            omt_batch_handle *out);
/* Each pair stops at its own first check with residual <= tol (checks every
 * check_every iterations, as omt_solve); infos: host array of B (nullable).
 * Every call starts all B problems from their current iterates.  As problems
 * stop, the strips of those still running are re-cut to as few rows as fill
 * the chip in one round (never more than each problem's default; rows fixed
 * by the caller or by omt_batch_autotune stay), which changes no iterate.
 * Environment:
 * OMT_BATCH_PERSISTENT selects the single persistent launch with grid
 * barriers instead of graph-replayed per-iteration launches; OMT_LOG >= 2
 * prints a line to stderr whenever more problems have stopped. */
omt_status omt_batch_solve(omt_batch_handle h, int64_t max_iters, double tol, int32_t check_every,
                           omt_info *infos);
omt_status omt_batch_distance(omt_batch_handle h, double *V /* host, B */);
omt_status omt_batch_grad(omt_batch_handle h, void *const *d_rho0, void *const *d_rho1);
omt_status omt_batch_get_state(omt_batch_handle h, int32_t b, void *phi, void *u, void *w);
/* Warm start of problem b of the batch (as omt_set_state; Sec. 7.2 takes
 * initial guesses); the next omt_batch_solve continues from it. */
omt_status omt_batch_set_state(omt_batch_handle h, int32_t b, const void *phi, const void *u, const void *w);
/* Choose the rows per strip of the batched step kernel for every shape class
 * of the batch (problems with the same grid and compiled type): each
 * candidate is timed over launches_per_trial launches (at least 4, HIP
 * events on the batch's private stream) of that class alone, in the launch
 * shape the batch's solves run (two iterations per launch when they do),
 * reading the current iterates without changing them.  Problems whose rows_per_wave the
 * caller fixed keep it.  The choice is kept in the handle (the next
 * omt_batch_solve uses it) and in the tuning cache under "batch <class>"
 * (OMT_TUNE_CACHE), where omt_batch_create finds it.  Rows never change the
 * iterates: every problem stays bit-identical to its own omt_solve.
 * rows: host array of B (nullable), the rows chosen per problem;
 * us_per_iter (nullable): one batched iteration of all B problems with the
 * chosen rows, in microseconds (a two-iteration launch counts as two).  launches_per_trial = 0 tunes nothing and
 * only reports the rows in use (us_per_iter 0).  Not for use while a solve
 * of this handle runs on another thread. */
omt_status omt_batch_autotune(omt_batch_handle h, int32_t launches_per_trial, int32_t *rows, double *us_per_iter);
omt_status omt_batch_destroy(omt_batch_handle h);

/* ----------------------------------------------------------- utilities */

/* Time the step kernel for each blocking depth T and rows-per-wave
 * candidate on the handle's problem (state is saved and restored), verify
 * that every candidate gives bit-identical iterates to T = 1, store the
 * fastest in the handle and in the tuning cache (the JSON file named by
 * OMT_TUNE_CACHE, if set).  best_t / best_rows / best_us (nullable) report
 * the choice and its time per iteration in microseconds. */
omt_status omt_autotune(omt_handle h, int32_t iters_per_trial, int32_t *best_t, int32_t *best_rows,
                        double *best_us);

/* Launch exactly n iterations of the step kernel with the given blocking
 * depth (T must divide n) and report the mean time per launch in
 * microseconds, measured with HIP events around one replay of the launches
 * captured as a HIP graph (the way the solve runs its check intervals), on
 * the handle's private stream after the work already on its stream.  For
 * measurement; the state advances by n iterations.  One more launch,
 * untimed, precedes them so that the queue is busy when the timed region
 * opens; it writes only the buffers the first timed launch overwrites. */
omt_status omt_time_steps(omt_handle h, int32_t T, int32_t rows_per_wave, int64_t n, double *us_per_launch);

/* ------------------------------------------------- without allocation */

/* Bytes of the device workspace inside the library used by omt_solve_static. */
#define OMT_STATIC_WORKSPACE_BYTES (64u << 20)

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc and its relatives): one whole solve of the
 * vector method -- the set-up of omt_create, the iterations of omt_solve,
 * then V as omt_distance and the gradients as omt_grad -- whose device
 * workspace is a fixed array inside the library of
 * OMT_STATIC_WORKSPACE_BYTES per GPU, held from the first call on a GPU
 * until the process ends.  The call allocates no device, pinned or heap
 * memory and captures no graph (so it is slower than a handle for short
 * check intervals).  Arguments as for omt_create / omt_solve; V (host),
 * d_rho0, d_rho1 (device, m*n*k of the dtype) and info are each nullable.
 * Iterates, V and gradients are bit-identical to omt_create + omt_solve +
 * omt_distance + omt_grad on the same problem.
 * Limits and sharing: a problem whose omt_workspace_bytes() exceed
 * OMT_STATIC_WORKSPACE_BYTES (for example FP32 with k = 3 above about
 * 790 x 790) is rejected with OMT_ENOMEM before any device work.  Every
 * call on one GPU uses that GPU's single array and starts by zeroing the
 * state it holds, so calls that overlap on one GPU (other threads or
 * streams) race and must be serialised by the caller.  The stream is
 * synchronised before the call returns.  Returns OMT_ENOTCONV as omt_solve
 * (outputs valid). */
omt_status omt_solve_static(const omt_params *p, const void *rho0, const void *rho1, int64_t max_iters, double tol,
                            int32_t check_every, double *V, void *d_rho0, void *d_rho1, omt_info *info,
                            void *stream);

const char *omt_strerror(omt_status s);
const char *omt_last_error(void);
int32_t omt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OMT_H */
