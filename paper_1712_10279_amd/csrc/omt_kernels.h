// Internal interface between the host driver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace omt {

constexpr int KMAX = 9;    // channels (8 for the vector method; 9 coordinates for complex 3 x 3 matrices)
constexpr int LMAX = 28;   // edges (complete graph on 8 nodes)
constexpr int WAVE = 64;
constexpr int STEP_WAVES_PER_WG = 4;
constexpr int NMET = 8;  // su, sw, sp, cross, primal, dual, mass, sum_phi
// rows of a check-iteration metrics tile (64 columns wide, one wave each)
constexpr int MET_ROWS = 8;

// Channel graphs the step kernel is compiled for.  The path (edges (c, c+1))
// and the complete graph (all a < b in lexicographic order) get their
// incidence structure at compile time; any other graph uses the dense
// matrix M = D diag(1/c) with the edge count rounded up to a bucket (the
// unused edges carry zero weight).
// G_MATRIX: the matrix method in orthonormal real coordinates of the
// Hermitian / skew-Hermitian matrices: a dense operator plus the grouped
// entry-wise norms (u norm 3, w norm 2) of that coordinate system.
// G_MATNUC: the same with the nuclear norms (u norm 4, w norm 3) compiled
// in as well (their per-pixel eigendecompositions cost registers, so the
// other matrix problems do not carry them).
enum GraphKind { G_NONE = 0, G_PATH = 1, G_COMPLETE = 2, G_DENSE = 3, G_MATRIX = 4, G_MATNUC = 5 };
constexpr bool is_matrix_kind(int gk) { return gk == G_MATRIX || gk == G_MATNUC; }

// Coordinates of the transfer variable compiled for a matrix problem with
// K coordinates of the potential and lc of the transfer: K = 3 (real 2 x 2,
// up to three L_s), 4 (complex 2 x 2, two L_s), 6 (real 3 x 3: two L_s, as
// in the diffusion-tensor example, or three) and 9 (complex 3 x 3, two
// L_s); 0 if not compiled.
inline int matrix_bucket(int K, int lc)
{
    if (K == 3) return lc <= 3 ? 3 : 0;
    if (K == 4) return lc <= 8 ? 8 : 0;
    if (K == 6) return lc <= 6 ? 6 : lc <= 9 ? 9 : 0;
    if (K == 9) return lc <= 18 ? 18 : 0;
    return 0;
}

inline int dense_bucket(int k, int l)
{
    if (l <= k - 1) return k - 1;  // trees
    return k * (k - 1) / 2;        // room for K_k
}

// Arguments of one fused PDHG launch (T iterations).  Arrays are SoA planes
// [plane][i][pitch]; u planes 0..k-1 hold u_x, k..2k-1 hold u_y.
template <typename R>
struct StepArgs {
    const R *phi_in;
    R *phi_out;
    const R *u_in;
    R *u_out;
    const R *w_in;
    R *w_out;
    const R *f;
    const float *plo_in;   // low parts of a compensated FP32 potential (or null)
    float *plo_out;
    int64_t plane;         // elements per plane
    int32_t m, n, pitch;
    int32_t l;             // edges in use (<= bucket)
    int32_t unorm, wnorm;
    int32_t rows;          // rows per wave
    int32_t ncolw, nroww;  // waves across / down the grid
    int32_t nwg;           // workgroups launched
    R mu, mu_h;            // mu, mu / h
    R nu, anu;             // nu, alpha nu
    R tau, inv_h;          // tau, 1 / h
    R ureg, wreg;          // 1 / (1 + 2 mu eps), 1 / (1 + 2 nu eps): regularised shrinks (1 without)
    double alpha;          // weight of the transfer term (objective)
    double eps;            // quadratic regularisation weight (objective)
    R ic[LMAX];            // 1 / c_e
    R gm[KMAX * LMAX];     // dense graphs: M = D diag(1/c), row c, column e at gm[c * LMAX + e]
    // grouped norms (G_MATRIX): weight of the group that starts at this
    // coordinate; 0 marks the second coordinate of a two-coordinate group
    R uwt[KMAX];
    R wwt[LMAX];
    // check launches: quad sums of the check terms, quantity q of row block
    // b (MET_ROWS rows) and quad g (4 columns) at qpart[q * qstride + b * nq + g]
    double *qpart;
    int64_t qstride;
    int32_t nq;
};

struct StepLaunch {
    int dtype;   // 0 f32, 1 f64
    int k, gk;   // channels, GraphKind
    int lb;      // edges compiled for
    int T;       // iterations per launch
    bool comp;   // compensated potential
    const void *args;
    hipStream_t stream;
    bool check = false;  // also take the check of the last iteration (args.qpart)
};

// Graph kinds whose step kernel can take the check in the same pass (the
// vector method; the matrix kinds run the separate metrics pass).
constexpr bool check_compiled(int gk) { return !is_matrix_kind(gk); }

// Defined once per channel count in step.hip (compiled per channel count).
hipError_t launch_step(const StepLaunch &L);
bool step_supported(int dtype, int k, int gk, int lb, int T, bool comp);
hipError_t step_blocks_per_cu(const StepLaunch &L, int *blocks);  // resident workgroups per CU
// Per-tile metrics of the step args' (in -> out) buffers into partials
// [ntiles][NMET]; tiles are 64 columns x 16 rows.
hipError_t launch_tile_metrics(const StepLaunch &L, int ncolw, int ntiles, double *partials);
// out[q] = sum of the ntiles rows of partials (one wave, fixed order).
hipError_t launch_reduce_tiles(const double *partials, int ntiles, double *out, hipStream_t s);
// Tile rows [nblk * ncolw][NMET] (tile = block * ncolw + column tile) from the
// quad sums a check launch stores (qpart[q * qstride + block * nq + quad]),
// adding each tile's 16 quads as the last four levels of wave_sum do.
hipError_t launch_quads_to_tiles(const double *qpart, int64_t qstride, int nq, int nblk, int ncolw, double *partials,
                                 hipStream_t s);

// ---------------------------------------------------------------- batched

// One problem of a batch.  v[par * 4 + wcur * 2 + check] are its step
// arguments for the iteration parity par (potential / flux buffers), the
// current w buffer and whether the iteration is a check (w out of place).
struct BatchPair {
    // step arguments of the batch's dtype (StepArgs<float> or <double>): 8
    // single-iteration variants (parity, w buffer, check), then 4 for two
    // iterations per launch (parity, w buffer)
    alignas(16) unsigned char v[12][sizeof(StepArgs<double>)];
    template <typename R>
    __host__ __device__ const StepArgs<R> &args(int var) const
    {
        return *reinterpret_cast<const StepArgs<R> *>(v[var]);
    }
    template <typename R>
    StepArgs<R> &args_mut(int var)
    {
        return *reinterpret_cast<StepArgs<R> *>(v[var]);
    }
    int type, l;
    int ncolw, tile0, ntiles;      // step strips: across, first in the list, count
    int ncolw2, tile0_2, ntiles2;  // strips of two-iteration launches likewise
    int mcolw, mtile0, mtiles;     // metric tiles likewise
    double mu, nu, tau, R0;
};

struct BatchPairState {
    int done, converged, cur, wcur;
    int64_t iters;
    int checks, pad;
    double met[NMET];
};

struct BatchArgs {
    const BatchPair *pairs;
    BatchPairState *state;
    const int *tile_pair, *tile_pair2, *mtile_pair;
    double *partials;
    unsigned *bar;  // barrier words, BAR_WORDS of them (see grid_sync in batch.hip)
    int B, total_tiles, total_tiles2, total_mtiles, check_every;
    int64_t max_iters;
    double tol;
};

constexpr int BAR_GROUPS = 8, BAR_GROUP0 = 32, BAR_STRIDE = 32;
constexpr int BAR_WORDS = BAR_GROUP0 + BAR_STRIDE * BAR_GROUPS;

int batch_type(int k, int gk, int lb);  // -1 if not compiled into the batched kernel
// dtype: 0 FP32 (comp: compensated potential), 1 FP64
hipError_t batch_blocks_per_cu(int dtype, bool comp, int *blocks);
hipError_t launch_batch(const BatchArgs &a, int dtype, bool comp, int nblocks, hipStream_t s);
// T iterations (1 or 2) of every unfinished problem; var = par * 4 + wcur * 2 +
// check for T = 1, 8 + par * 2 + wcur for T = 2
hipError_t launch_batch_step(const BatchArgs &a, int dtype, bool comp, int var, hipStream_t s, int T = 1);
// metrics tiles and per-problem decisions after a check iteration (iters =
// iterations since the previous check; last = the solve ends here; cur /
// wcur = buffers of the iterate after it, relative to the solve's start)
hipError_t launch_batch_check(const BatchArgs &a, int dtype, bool comp, int var, int iters, bool last, int cur,
                              int wcur, hipStream_t s);

// ---------------------------------------------------------------- auxiliary

struct SumsArgs {       // per-channel FP64 sums of two AoS densities
    const void *rho0, *rho1;
    int dtype;
    int64_t npix;
    int k;
    double *partials;   // [nblocks][4*k + 1]
    int nblocks;
};
hipError_t launch_sums(const SumsArgs &a, hipStream_t s);

struct MakeFArgs {
    const void *rho0, *rho1;
    int dtype;
    int m, n, k, pitch;
    int p;                // slices of a 3-D grid (1: 2-D); plane row z m + i
    int64_t plane;
    const double *shift;  // k values subtracted from rho1 - rho0 (device)
    void *f;
};
hipError_t launch_make_f(const MakeFArgs &a, hipStream_t s);

// Sum nblocks rows of width `width` in a fixed order into out[width].
hipError_t launch_reduce_rows(const double *partials, int nblocks, int width, double *out, hipStream_t s);

// Per-channel FP64 sums of the SoA potential (for the mean removal).
struct PlaneSumArgs {
    const void *phi;
    const float *plo;
    int dtype;
    int m, n, k, pitch;
    int64_t plane;
    double *partials;   // [nblocks][k]
    int nblocks;
};
hipError_t launch_plane_sums(const PlaneSumArgs &a, hipStream_t s);

// SoA <-> AoS copies.  mode: 0 potential out (dst = sign * (phi - mean[c])),
// 1 u out, 2 w out, 3 phi in, 4 u in (ghosts zeroed), 5 w in.
struct XferArgs {
    int p = 1;              // slices of a 3-D grid (1: 2-D); u then has 3 components
    const void *src;
    void *dst;
    const float *plo;       // compensated low part (potential out only)
    float *plo_out;         // zeroed on phi in
    int dtype;
    int m, n, k, pitch;
    int64_t plane;
    int mode;
    double sign;
    const double *mean;     // k values (device), potential out only
};
hipError_t launch_xfer(const XferArgs &a, hipStream_t s);

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
// NaN (all-ones words) into the padding of nplanes planes of plane_stride_bytes
// each: rows of row_elems elements of esz bytes, of which the first n are
// the grid's; everything past rows * row_elems in a plane is padding too
hipError_t launch_poison(void *p, int64_t nplanes, size_t plane_stride_bytes, int row_elems, int64_t rows, int n,
                         int esz, hipStream_t s);

// Matrices <-> orthonormal real coordinates of the matrix method.  Per pixel
// `count` k x k matrices (complex (re, im) pairs, or real entries when real
// is set) against `count` groups of ncoord coordinates; coordinate c of
// group g at pixel p sits at ((p * count + g) * ncoord + c) * cstride + coff.
// Hermitian coordinates: X_aa, then for a < b sqrt2 Re X_ab (and sqrt2
// Im X_ab); skew-Hermitian: Im X_aa (complex only), then the same pairs.
// Packing reads the upper triangle and the diagonal only.
struct MatrixXferArgs {
    const void *src;
    void *dst;
    int dtype;
    int64_t npix;
    int k, real, herm, pack;
    int count, cstride, coff;
};
hipError_t launch_matrix_xfer(const MatrixXferArgs &a, hipStream_t s);

}  // namespace omt
