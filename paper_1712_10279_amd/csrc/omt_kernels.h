// Internal interface between the host driver and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace omt {

constexpr int KMAX = 8;    // channels
constexpr int LMAX = 28;   // edges (complete graph on 8 nodes)
constexpr int WAVE = 64;
constexpr int STEP_WAVES_PER_WG = 4;

// Channel graphs the step kernel is compiled for.  The path (edges (c, c+1))
// and the complete graph (all a < b in lexicographic order) get their
// incidence structure at compile time; any other graph uses the dense
// matrix M = D diag(1/c) with the edge count rounded up to a bucket (the
// unused edges carry zero weight).
enum GraphKind { G_NONE = 0, G_PATH = 1, G_COMPLETE = 2, G_DENSE = 3 };

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
    R ic[LMAX];            // 1 / c_e
    R gm[KMAX * LMAX];     // dense graphs: M = D diag(1/c), row c, column e at gm[c * LMAX + e]
};

struct StepLaunch {
    int dtype;   // 0 f32, 1 f64
    int k, gk;   // channels, GraphKind
    int lb;      // edges compiled for
    int T;       // iterations per launch
    bool comp;   // compensated potential
    const void *args;
    hipStream_t stream;
};

// Defined once per channel count in step_k<K>.hip.
hipError_t launch_step(const StepLaunch &L);
bool step_supported(int dtype, int k, int gk, int lb, int T, bool comp);

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
    int64_t plane;
    const double *shift;  // k values subtracted from rho1 - rho0 (device)
    void *f;
};
hipError_t launch_make_f(const MakeFArgs &a, hipStream_t s);

// Metrics of the step (old -> new); old == new gives objectives of one iterate.
struct MetricArgs {
    const void *phi0, *phi1, *u0, *u1, *w0, *w1, *f;
    const float *plo0, *plo1;
    int dtype;
    int m, n, k, l, pitch;
    int64_t plane;
    int unorm, wnorm;
    double inv_h, alpha;
    double gm[KMAX * LMAX];
    double *partials;   // [nblocks][NMET]
    int nblocks;
};
constexpr int NMET = 8;  // su, sw, sp, cross, primal, dual, mass, sum_phi
hipError_t launch_metrics(const MetricArgs &a, hipStream_t s);

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

}  // namespace omt
