// Host driver and C ABI (include/omt.h) of the vector-OMT solver.
//
// Parameter validation, the step sizes of Sec. 7.2 (lambda_max(-Delta_G) by
// cyclic Jacobi on the k x k graph Laplacian of Sec. 3.1), the mass check,
// workspace layout, the iteration loop with its check cadence, and the
// stopping rule on the fixed-point residual R^k of Sec. 6.1.

#include <rocprofiler-sdk-roctx/roctx.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/omt.h"
#include "../../include/omt_matrix.h"
#include "grid3.h"
#include "omt_kernels.h"

#include <complex>

namespace omt {

hipError_t launch_step_k1(const StepLaunch &);
hipError_t launch_step_k2(const StepLaunch &);
hipError_t launch_step_k3(const StepLaunch &);
hipError_t launch_step_k4(const StepLaunch &);
hipError_t launch_step_k5(const StepLaunch &);
hipError_t launch_step_k6(const StepLaunch &);
hipError_t launch_step_k7(const StepLaunch &);
hipError_t launch_step_k8(const StepLaunch &);
hipError_t launch_step_k9(const StepLaunch &);
hipError_t launch_metrics_k1(const StepLaunch &, int, int, double *);
hipError_t launch_metrics_k2(const StepLaunch &, int, int, double *);
hipError_t launch_metrics_k3(const StepLaunch &, int, int, double *);
hipError_t launch_metrics_k4(const StepLaunch &, int, int, double *);
hipError_t launch_metrics_k5(const StepLaunch &, int, int, double *);
hipError_t launch_metrics_k6(const StepLaunch &, int, int, double *);
hipError_t launch_metrics_k7(const StepLaunch &, int, int, double *);
hipError_t launch_metrics_k8(const StepLaunch &, int, int, double *);
hipError_t launch_metrics_k9(const StepLaunch &, int, int, double *);
bool step_supported_k1(int, int, int, int, bool);
bool step_supported_k2(int, int, int, int, bool);
bool step_supported_k3(int, int, int, int, bool);
bool step_supported_k4(int, int, int, int, bool);
bool step_supported_k5(int, int, int, int, bool);
bool step_supported_k6(int, int, int, int, bool);
bool step_supported_k7(int, int, int, int, bool);
bool step_supported_k8(int, int, int, int, bool);
bool step_supported_k9(int, int, int, int, bool);

hipError_t launch_step(const StepLaunch &L)
{
    switch (L.k) {
        case 1: return launch_step_k1(L);
        case 2: return launch_step_k2(L);
        case 3: return launch_step_k3(L);
        case 4: return launch_step_k4(L);
        case 5: return launch_step_k5(L);
        case 6: return launch_step_k6(L);
        case 7: return launch_step_k7(L);
        case 8: return launch_step_k8(L);
        case 9: return launch_step_k9(L);
        default: return hipErrorInvalidValue;
    }
}

hipError_t step_blocks_per_cu_k1(const StepLaunch &, int *);
hipError_t step_blocks_per_cu_k2(const StepLaunch &, int *);
hipError_t step_blocks_per_cu_k3(const StepLaunch &, int *);
hipError_t step_blocks_per_cu_k4(const StepLaunch &, int *);
hipError_t step_blocks_per_cu_k5(const StepLaunch &, int *);
hipError_t step_blocks_per_cu_k6(const StepLaunch &, int *);
hipError_t step_blocks_per_cu_k7(const StepLaunch &, int *);
hipError_t step_blocks_per_cu_k8(const StepLaunch &, int *);
hipError_t step_blocks_per_cu_k9(const StepLaunch &, int *);

hipError_t step_blocks_per_cu(const StepLaunch &L, int *blocks)
{
    switch (L.k) {
        case 1: return step_blocks_per_cu_k1(L, blocks);
        case 2: return step_blocks_per_cu_k2(L, blocks);
        case 3: return step_blocks_per_cu_k3(L, blocks);
        case 4: return step_blocks_per_cu_k4(L, blocks);
        case 5: return step_blocks_per_cu_k5(L, blocks);
        case 6: return step_blocks_per_cu_k6(L, blocks);
        case 7: return step_blocks_per_cu_k7(L, blocks);
        case 8: return step_blocks_per_cu_k8(L, blocks);
        case 9: return step_blocks_per_cu_k9(L, blocks);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_tile_metrics(const StepLaunch &L, int ncolw, int ntiles, double *partials)
{
    switch (L.k) {
        case 1: return launch_metrics_k1(L, ncolw, ntiles, partials);
        case 2: return launch_metrics_k2(L, ncolw, ntiles, partials);
        case 3: return launch_metrics_k3(L, ncolw, ntiles, partials);
        case 4: return launch_metrics_k4(L, ncolw, ntiles, partials);
        case 5: return launch_metrics_k5(L, ncolw, ntiles, partials);
        case 6: return launch_metrics_k6(L, ncolw, ntiles, partials);
        case 7: return launch_metrics_k7(L, ncolw, ntiles, partials);
        case 8: return launch_metrics_k8(L, ncolw, ntiles, partials);
        case 9: return launch_metrics_k9(L, ncolw, ntiles, partials);
        default: return hipErrorInvalidValue;
    }
}

bool step_supported(int dtype, int k, int gk, int lb, int T, bool comp)
{
    switch (k) {
        case 1: return step_supported_k1(dtype, gk, lb, T, comp);
        case 2: return step_supported_k2(dtype, gk, lb, T, comp);
        case 3: return step_supported_k3(dtype, gk, lb, T, comp);
        case 4: return step_supported_k4(dtype, gk, lb, T, comp);
        case 5: return step_supported_k5(dtype, gk, lb, T, comp);
        case 6: return step_supported_k6(dtype, gk, lb, T, comp);
        case 7: return step_supported_k7(dtype, gk, lb, T, comp);
        case 8: return step_supported_k8(dtype, gk, lb, T, comp);
        case 9: return step_supported_k9(dtype, gk, lb, T, comp);
        default: return false;
    }
}

}  // namespace omt

using namespace omt;

// ------------------------------------------------------------------ errors

namespace {

// detail of the last failure on this thread (fixed storage: no call allocates
// to report an error)
thread_local char g_last_error[512];

// Verbosity from OMT_LOG (read once): 0 silent, 1 every failure, 2 also a
// line per solve, 3 also a line per check.  OMT_VERBOSE alone means 2.
int log_level()
{
    static const int level = [] {
        const char *v = std::getenv("OMT_LOG");
        if (v && *v) return std::max(0, std::atoi(v));
        return std::getenv("OMT_VERBOSE") ? 2 : 0;
    }();
    return level;
}

omt_status fail(omt_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    std::memcpy(g_last_error, buf, sizeof(buf));
    if (log_level() >= 1) std::fprintf(stderr, "omt: %s: %s\n", s == OMT_OK ? "note" : omt_strerror(s), buf);
    return s;
}

// A named range on the ROCTx marker stream (visible to rocprofv3
// --marker-trace; a no-op without a tool attached) for the scope's lifetime.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

#define HIP_TRY(expr)                                                                               \
    do {                                                                                            \
        hipError_t e_ = (expr);                                                                     \
        if (e_ != hipSuccess) return fail(OMT_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

// ------------------------------------------------------------------ graph

// Eigenvalues of a symmetric k x k matrix by the cyclic Jacobi method, in
// place: A (row-major, overwritten) and ev[k] are the caller's storage.
void jacobi_eigenvalues(double *A, int k, double *ev)
{
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int p = 0; p < k; ++p)
            for (int q = 0; q < k; ++q) {
                tot += A[p * k + q] * A[p * k + q];
                if (p != q) off += A[p * k + q] * A[p * k + q];
            }
        if (off <= 1e-30 * std::max(tot, 1e-300)) break;
        for (int p = 0; p + 1 < k; ++p)
            for (int q = p + 1; q < k; ++q) {
                const double apq = A[p * k + q];
                if (apq == 0.0) continue;
                const double th = (A[q * k + q] - A[p * k + p]) / (2.0 * apq);
                const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int r = 0; r < k; ++r) {
                    const double a = A[r * k + p], b = A[r * k + q];
                    A[r * k + p] = cs * a - sn * b;
                    A[r * k + q] = sn * a + cs * b;
                }
                for (int r = 0; r < k; ++r) {
                    const double a = A[p * k + r], b = A[q * k + r];
                    A[p * k + r] = cs * a - sn * b;
                    A[q * k + r] = sn * a + cs * b;
                }
            }
    }
    for (int p = 0; p < k; ++p) ev[p] = A[p * k + p];
}

struct Resolved {
    int m, n, k, l, gk, lb;
    int p = 1;  // slices of a 3-D grid (1: the 2-D grid)
    // fixed-size members: resolving a vector problem allocates nothing
    std::array<int32_t, 2 * LMAX> edges;
    std::array<double, LMAX> cost;
    double alpha, tau, mu, nu, h, lmax, eps;
    int unorm, wnorm, dtype;
    bool comp;
    int tblock, rows;
    std::array<int, KMAX> cls;  // mass class per channel (-1: no mass constraint, no mean removed)
    int ncls;
    // matrix method (G_MATRIX): dense operator, row c / column e at
    // gmat[c * LMAX + e], and the group weights of the grouped norms
    bool matrix = false;
    std::vector<double> gmat, uwt, wwt;
};

// Planes of a field lie one plane stride apart: m rows of the 64-aligned
// pitch, plus a skew of 4 KiB + 256 B.  Without it, planes of a power-of-two
// size (256^2, 512^2, 1024^2 FP32) put the same pixel of every plane on the
// same HBM channel and bank, and a strip's dozens of concurrent plane
// streams collide: a streaming probe of 36 read and 31 write planes of
// 1024^2 floats moved 5.0 TB/s unskewed and 6.0 TB/s with this skew.
#ifndef OMT_PLANE_SKEW_BYTES
#define OMT_PLANE_SKEW_BYTES (4096 + 256)
#endif
constexpr int64_t PLANE_SKEW_BYTES = OMT_PLANE_SKEW_BYTES;
static_assert(PLANE_SKEW_BYTES % 256 == 0, "planes stay 256-byte aligned");

int row_pitch(int n) { return (n + 63) / 64 * 64; }

int64_t plane_elems(int m, int n, int esz, int p = 1)
{
    return (int64_t)p * m * row_pitch(n) + PLANE_SKEW_BYTES / esz;
}

// flux components per channel: (u_x, u_y), and u_z on a 3-D grid
int ucomp(const Resolved &r) { return r.p > 1 ? 3 : 2; }

// The step kernels reach all planes of a field (phi, u, w or f) from one
// row through a buffer descriptor with 32-bit byte offsets: every field must
// stay below 2 GiB.
bool fields_fit(const Resolved &r)
{
    const int64_t planes = std::max(ucomp(r) * r.k, std::max(r.lb, 1));
    const int esz = r.dtype == OMT_F64 ? 8 : 4;
    return planes * plane_elems(r.m, r.n, esz, r.p) * esz < ((int64_t)1 << 31);
}

omt_status resolve(const omt_params *p, Resolved &r)
{
    if (!p) return fail(OMT_EINVAL, "params is NULL");
    if (p->m < 2 || p->n < 2) return fail(OMT_EINVAL, "grid must be at least 2 x 2 (got %d x %d)", p->m, p->n);
    if ((int64_t)p->m * p->n > (int64_t)1 << 31) return fail(OMT_EINVAL, "grid too large");
    if (p->k < 1) return fail(OMT_EINVAL, "k must be >= 1 (got %d)", p->k);
    if (p->k > OMT_MAX_CHANNELS) return fail(OMT_EUNSUPPORTED, "k = %d exceeds %d", p->k, OMT_MAX_CHANNELS);
    if (p->n_edges < 0) return fail(OMT_EGRAPH, "negative edge count");
    if (p->n_edges > 0 && !p->edges) return fail(OMT_EGRAPH, "edges is NULL");
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return fail(OMT_EINVAL, "alpha must be > 0");
    if (!(p->tau > 0.0) || !std::isfinite(p->tau)) return fail(OMT_EINVAL, "tau must be > 0");
    if (p->mu < 0.0 || p->nu < 0.0 || p->h < 0.0 || !std::isfinite(p->mu) || !std::isfinite(p->nu) ||
        !std::isfinite(p->h))
        return fail(OMT_EINVAL, "mu, nu, h must be finite and >= 0");
    if (p->unorm < 0 || p->unorm > 2) return fail(OMT_EINVAL, "unknown u norm %d", p->unorm);
    if (p->wnorm < 0 || p->wnorm > 1) return fail(OMT_EINVAL, "unknown w norm %d", p->wnorm);
    if (p->dtype != OMT_F32 && p->dtype != OMT_F64) return fail(OMT_EINVAL, "unknown dtype %d", p->dtype);
    if (p->tblock < 0 || p->rows_per_wave < 0) return fail(OMT_EINVAL, "tblock and rows_per_wave must be >= 0");
    if (!(p->reg_eps >= 0.0) || !std::isfinite(p->reg_eps)) return fail(OMT_EINVAL, "reg_eps must be finite and >= 0");
    if (p->p < 0) return fail(OMT_EINVAL, "depth p must be >= 0 (got %d)", p->p);
    if ((int64_t)p->m * p->n * std::max(p->p, 1) > (int64_t)1 << 31) return fail(OMT_EINVAL, "grid too large");

    r.m = p->m;
    r.n = p->n;
    r.k = p->k;
    r.l = p->n_edges;
    if (r.l > LMAX) return fail(OMT_EUNSUPPORTED, "%d edges exceed %d", r.l, LMAX);
    for (int q = 0; q < 2 * r.l; ++q) r.edges[q] = p->edges[q];
    for (int e = 0; e < r.l; ++e) r.cost[e] = 1.0;
    if (p->edge_cost)
        for (int e = 0; e < r.l; ++e) r.cost[e] = p->edge_cost[e];
    for (int e = 0; e < r.l; ++e) {
        const int a = r.edges[2 * e], b = r.edges[2 * e + 1];
        if (a < 0 || b >= r.k || a >= b)
            return fail(OMT_EGRAPH, "edge %d = (%d, %d): need 0 <= a < b < k = %d", e, a, b, r.k);
        if (!(r.cost[e] > 0.0) || !std::isfinite(r.cost[e]))
            return fail(OMT_EGRAPH, "edge %d has cost %g, need > 0", e, r.cost[e]);
        for (int f = 0; f < e; ++f)
            if (r.edges[2 * f] == a && r.edges[2 * f + 1] == b) return fail(OMT_EGRAPH, "duplicate edge (%d, %d)", a, b);
    }
    // graph kind: compiled incidence for the path and the complete graph in
    // canonical edge order, the dense matrix otherwise
    {
        bool path = r.l == r.k - 1, full = r.l == r.k * (r.k - 1) / 2;
        for (int e = 0; e < r.l && path; ++e) path = r.edges[2 * e] == e && r.edges[2 * e + 1] == e + 1;
        int e = 0;
        for (int a = 0; a < r.k && full; ++a)
            for (int b = a + 1; b < r.k && full; ++b, ++e) full = r.edges[2 * e] == a && r.edges[2 * e + 1] == b;
        if (r.l == 0) {
            r.gk = G_NONE;
            r.lb = 0;
        } else if (path) {
            r.gk = G_PATH;
            r.lb = r.l;
        } else if (full) {
            r.gk = G_COMPLETE;
            r.lb = r.l;
        } else {
            r.gk = G_DENSE;
            r.lb = dense_bucket(r.k, r.l);
        }
    }
    r.alpha = p->alpha;
    r.tau = p->tau;
    r.eps = p->reg_eps;
    r.unorm = p->unorm;
    r.wnorm = p->wnorm;
    r.dtype = p->dtype;
    r.comp = (p->flags & OMT_FLAG_COMPENSATED_PHI) && p->dtype == OMT_F32;
    r.tblock = p->tblock;
    r.rows = p->rows_per_wave;
    r.p = std::max(p->p, 1);
    r.h = p->h > 0.0 ? p->h : 1.0 / double(std::max(std::max(r.m, r.n), r.p) - 1);

    // lambda_max(-Delta_G), -Delta_G = D diag(1/c^2) D^T (Sec. 3.1)
    r.lmax = 0.0;
    if (r.l > 0) {
        double A[KMAX * KMAX] = {0.0}, ev[KMAX];
        for (int e = 0; e < r.l; ++e) {
            const int a = r.edges[2 * e], b = r.edges[2 * e + 1];
            const double wgt = 1.0 / (r.cost[e] * r.cost[e]);
            A[a * r.k + a] += wgt;
            A[b * r.k + b] += wgt;
            A[a * r.k + b] -= wgt;
            A[b * r.k + a] -= wgt;
        }
        jacobi_eigenvalues(A, r.k, ev);
        for (int c = 0; c < r.k; ++c) r.lmax = std::max(r.lmax, ev[c]);
    }
    // step sizes of Sec. 7.1 / 7.2 unless given; on a 3-D grid the bound
    // 8/h^2 of the 2-D Laplacian becomes 12/h^2 and the rule scales with it
    const double h2 = r.h * r.h;
    const double lx = r.p > 1 ? 12.0 : 8.0;
    r.mu = p->mu > 0.0 ? p->mu : (r.l == 0 ? h2 / (2.0 * lx * r.tau) : h2 / (4.0 * lx * r.tau));
    r.nu = r.l == 0 ? 0.0 : (p->nu > 0.0 ? p->nu : 1.0 / (4.0 * r.tau * r.lmax));
    if (p->mu > 0.0 || p->nu > 0.0) {
        const double cond = r.tau * r.mu * lx / h2 + r.tau * r.nu * r.lmax;
        if (!(cond < 1.0))
            return fail(OMT_ESTEP, "tau mu %g/h^2 + tau nu lambda_max = %g must be < 1 (Sec. 7.2)", lx, cond);
    }
    // mass classes: connected components of the channel graph
    for (int c = 0; c < r.k; ++c) r.cls[c] = c;
    for (bool ch = true; ch;) {
        ch = false;
        for (int e = 0; e < r.l; ++e) {
            int &a = r.cls[r.edges[2 * e]], &b = r.cls[r.edges[2 * e + 1]];
            const int lo = std::min(a, b);
            if (a != lo || b != lo) {
                a = b = lo;
                ch = true;
            }
        }
    }
    int map[KMAX];
    for (int c = 0; c < r.k; ++c) map[c] = -1;
    r.ncls = 0;
    for (int c = 0; c < r.k; ++c) {
        if (map[r.cls[c]] < 0) map[r.cls[c]] = r.ncls++;
        r.cls[c] = map[r.cls[c]];
    }
    if (!fields_fit(r))
        return fail(OMT_EUNSUPPORTED, "a field of %d x %d x %d x %d %s values exceeds 2 GiB", r.m, r.n, r.p,
                    std::max(ucomp(r) * r.k, r.lb), r.dtype == OMT_F64 ? "FP64" : "FP32");
    if (r.p > 1) {
        if (!step3_supported(r.dtype, r.k, r.gk, r.lb))
            return fail(OMT_EUNSUPPORTED, "3-D grids are compiled for k = 1, 2, 3 (k = %d, %d edges)", r.k, r.l);
        if (r.comp) return fail(OMT_EUNSUPPORTED, "3-D grids have no compensated potential");
        if (r.tblock > 1) return fail(OMT_EUNSUPPORTED, "3-D grids run one iteration per launch");
    }
    return OMT_OK;
}

// ------------------------------------------------------------------ layout

constexpr int METRIC_BLOCKS_MAX = 1024;
constexpr int SUM_BLOCKS_MAX = 512;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    int pitch;
    int64_t plane;  // elements
    size_t esz;
    size_t off_f, off_phi[2], off_u[2], off_w[2], off_plo[2], off_part, off_quad, off_res, off_vec, total;
    int64_t qstride;  // doubles per quantity of the quad sums of a check launch
    int nq, nqb;      // quads (4 columns) per row, row blocks (MET_ROWS rows)
};

Layout make_layout(const Resolved &r)
{
    Layout L;
    L.esz = r.dtype == OMT_F64 ? 8 : 4;
    L.pitch = row_pitch(r.n);
    L.plane = plane_elems(r.m, r.n, int(L.esz), r.p);
    const size_t pb = align256(size_t(L.plane) * L.esz);
    size_t o = 0;
    L.off_f = o;
    o += pb * r.k;
    for (int b = 0; b < 2; ++b) {
        L.off_phi[b] = o;
        o += pb * r.k;
    }
    for (int b = 0; b < 2; ++b) {
        L.off_u[b] = o;
        o += pb * ucomp(r) * r.k;
    }
    for (int b = 0; b < 2; ++b) {
        L.off_w[b] = o;
        o += pb * r.l;
    }
    const size_t pf = align256(size_t(L.plane) * 4);
    for (int b = 0; b < 2; ++b) {
        L.off_plo[b] = o;
        o += r.comp ? pf * r.k : 0;
    }
    L.off_part = o;
    const size_t met_tiles = size_t((r.n + WAVE - 1) / WAVE) * size_t((r.m + MET_ROWS - 1) / MET_ROWS) * size_t(r.p);
    size_t npart = std::max<size_t>(size_t(METRIC_BLOCKS_MAX) * KMAX, size_t(SUM_BLOCKS_MAX) * (4 * KMAX + 1));
    npart = std::max(npart, met_tiles * NMET);
    o += align256(sizeof(double) * npart);
    L.nq = (r.n + 3) / 4;
    L.nqb = (r.m + MET_ROWS - 1) / MET_ROWS;
    L.qstride = int64_t(L.nq) * L.nqb;
    L.off_quad = o;
    o += align256(sizeof(double) * NMET * size_t(L.qstride));
    L.off_res = o;
    o += align256(sizeof(double) * 64);
    L.off_vec = o;
    o += align256(sizeof(double) * 64);
    L.total = o;
    return L;
}

}  // namespace

// ------------------------------------------------------------------ handle

struct omt_ctx {
    Resolved r;
    Layout L;
    hipStream_t stream;
    int device;
    char *ws;
    void *f, *phi[2], *u[2], *w[2];
    float *plo[2];
    double *part, *quad, *res, *vec;
    double *host;  // pinned, 64 doubles
    int cur, wcur;
    double fnorm2;
    int metric_blocks;
    int64_t iters_done;
    omt_info last;
    bool have_last;
    int tuned_T, tuned_rows;   // from omt_autotune or the tuning cache (0: none)
    int user_rows;             // rows per wave the caller fixed (0: none); batched problems
    hipStream_t cap;           // private stream for capturing the check interval
    struct Graph {
        hipGraphExec_t exec;
        int K, T, rowsT, rows1, cur, wcur;  // what it was captured for
        int cur_after, wcur_after;          // buffer roles after one replay
    } graphs[2];
    int ngraphs;
};

namespace {

// Step arguments reading buffers (ci, wi) and writing buffers (co, wo).
template <typename R>
void fill_args(StepArgs<R> &a, const omt_ctx *h, int ci, int co, int wi, int wo, int rows, int ncolw, int nroww,
               int nwg)
{
    const Resolved &r = h->r;
    const int nc = ci, nx = co;
    a.phi_in = static_cast<const R *>(h->phi[nc]);
    a.phi_out = static_cast<R *>(h->phi[nx]);
    a.u_in = static_cast<const R *>(h->u[nc]);
    a.u_out = static_cast<R *>(h->u[nx]);
    a.w_in = static_cast<const R *>(h->w[wi]);
    a.w_out = static_cast<R *>(h->w[wo]);
    a.f = static_cast<const R *>(h->f);
    a.plo_in = r.comp ? h->plo[nc] : nullptr;
    a.plo_out = r.comp ? h->plo[nx] : nullptr;
    a.plane = h->L.plane;
    a.m = r.m;
    a.n = r.n;
    a.pitch = h->L.pitch;
    a.l = r.l;
    a.unorm = r.unorm;
    a.wnorm = r.wnorm;
    a.rows = rows;
    a.ncolw = ncolw;
    a.nroww = nroww;
    a.nwg = nwg;
    a.mu = R(r.mu);
    a.mu_h = R(r.mu / r.h);
    a.nu = R(r.nu);
    a.anu = R(r.alpha * r.nu);
    a.tau = R(r.tau);
    a.inv_h = R(1.0 / r.h);
    a.alpha = r.alpha;
    a.eps = r.eps;
    a.ureg = R(1.0 / (1.0 + 2.0 * r.mu * r.eps));
    a.wreg = R(1.0 / (1.0 + 2.0 * r.nu * r.eps));
    a.qpart = h->quad;
    a.qstride = h->L.qstride;
    a.nq = h->L.nq;
    for (int q = 0; q < KMAX * LMAX; ++q) a.gm[q] = R(0);
    for (int q = 0; q < LMAX; ++q) a.ic[q] = R(0);
    for (int q = 0; q < KMAX; ++q) a.uwt[q] = R(1);
    for (int q = 0; q < LMAX; ++q) a.wwt[q] = R(1);
    if (r.matrix) {
        for (int q = 0; q < KMAX * LMAX; ++q) a.gm[q] = R(r.gmat[q]);
        for (int c = 0; c < r.k; ++c) a.uwt[c] = R(r.uwt[c]);
        for (int e = 0; e < r.l; ++e) a.wwt[e] = R(r.wwt[e]);
        return;
    }
    for (int e = 0; e < r.l; ++e) {
        a.ic[e] = R(1.0 / r.cost[e]);
        a.gm[r.edges[2 * e] * LMAX + e] = R(1.0 / r.cost[e]);
        a.gm[r.edges[2 * e + 1] * LMAX + e] = R(-1.0 / r.cost[e]);
    }
}

// Step arguments of a 3-D launch reading buffers (ci, wi), writing (co, wo):
// zch slices per wave.
template <typename R>
void fill_args3(Step3Args<R> &a, const omt_ctx *h, int ci, int co, int wi, int wo, int zch)
{
    const Resolved &r = h->r;
    a.phi_in = static_cast<const R *>(h->phi[ci]);
    a.phi_out = static_cast<R *>(h->phi[co]);
    a.u_in = static_cast<const R *>(h->u[ci]);
    a.u_out = static_cast<R *>(h->u[co]);
    a.w_in = static_cast<const R *>(h->w[wi]);
    a.w_out = static_cast<R *>(h->w[wo]);
    a.f = static_cast<const R *>(h->f);
    a.plane = h->L.plane;
    a.m = r.m;
    a.n = r.n;
    a.p = r.p;
    a.pitch = h->L.pitch;
    a.l = r.l;
    a.unorm = r.unorm;
    a.wnorm = r.wnorm;
    a.ncolw = (r.n + G3_COLS - 1) / G3_COLS;
    a.nroww = (r.m + G3_ROWS - 1) / G3_ROWS;
    a.zch = std::max(1, std::min(zch, r.p));
    a.nzw = (r.p + a.zch - 1) / a.zch;
    const int64_t waves = int64_t(a.ncolw) * a.nroww * a.nzw;
    a.nwg = int((waves + STEP_WAVES_PER_WG - 1) / STEP_WAVES_PER_WG);
    a.mu = R(r.mu);
    a.mu_h = R(r.mu / r.h);
    a.nu = R(r.nu);
    a.anu = R(r.alpha * r.nu);
    a.tau = R(r.tau);
    a.inv_h = R(1.0 / r.h);
    a.ureg = R(1.0 / (1.0 + 2.0 * r.mu * r.eps));
    a.wreg = R(1.0 / (1.0 + 2.0 * r.nu * r.eps));
    for (int q = 0; q < KMAX * LMAX; ++q) a.gm[q] = R(0);
    for (int q = 0; q < LMAX; ++q) a.ic[q] = R(0);
    for (int e = 0; e < r.l; ++e) {
        a.ic[e] = R(1.0 / r.cost[e]);
        a.gm[r.edges[2 * e] * LMAX + e] = R(1.0 / r.cost[e]);
        a.gm[r.edges[2 * e + 1] * LMAX + e] = R(-1.0 / r.cost[e]);
    }
}

// Slices per wave on a 3-D grid: enough z chunks that about two waves per
// SIMD are resident (each chunk recomputes one extra slice, so no more).
int rule_zch(const omt_ctx *h)
{
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus < 1)
        cus = 256;
    const int64_t tiles = int64_t((h->r.n + G3_COLS - 1) / G3_COLS) * ((h->r.m + G3_ROWS - 1) / G3_ROWS);
    const int64_t want = int64_t(cus) * 4 * 2;
    const int64_t nz = std::max<int64_t>(1, std::min<int64_t>(h->r.p, (want + tiles - 1) / tiles));
    return int((h->r.p + nz - 1) / nz);
}

// Output columns of one wavefront: 64 aligned columns at one iteration per
// launch, 64 - 2T (plus halo lanes) when T iterations are pipelined.
int strip_cols(int T) { return T == 1 ? WAVE : WAVE - 2 * T; }

int rule_rows(const omt_ctx *h, int T);

int default_rows(const omt_ctx *h, int T)
{
    if (h->r.rows > 0) return h->r.rows;
    if (h->tuned_rows > 0 && h->tuned_T == T) return h->tuned_rows;
    if (h->r.p > 1) return rule_zch(h);
    return rule_rows(h, T);
}

int rule_rows(const omt_ctx *h, int T)
{
    // just enough rows per wave that every wave of the launch is resident at
    // once (one round over the chip), at most 32: a wave's rows are a chain of
    // dependent steps, so grids that fit the chip in one round take a single
    // row per wave (shortest chain) despite its extra halo row.  The round
    // counts at most two waves per SIMD even where three fit: two already
    // keep HBM busy, and the taller strips read fewer halo rows (1024^2 at
    // k = 8: 8 rows at two waves per SIMD 55.7 us, 6 rows at three 57.0 us)
    StepLaunch Lc;
    Lc.dtype = h->r.dtype;
    Lc.k = h->r.k;
    Lc.gk = h->r.gk;
    Lc.lb = h->r.lb;
    Lc.T = T;
    Lc.comp = h->r.comp;
    int bpc = 0, cus = 0;
    if (step_blocks_per_cu(Lc, &bpc) != hipSuccess || bpc < 1) bpc = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess || cus < 1)
        cus = 256;
    const int64_t slots = std::min<int64_t>(int64_t(bpc) * STEP_WAVES_PER_WG, 2 * 4) * cus;
    const int64_t ncolw = (h->r.n + strip_cols(T) - 1) / strip_cols(T);
    // the fewest rows whose strips, ceil(m / rows) per column block, all fit
    // in one round (T = 2 at 1024^2 k = 8: 9 rows would need 2,052 waves
    // for 2,048 slots, and the 4 left over take a whole second round)
    int64_t rows = std::max<int64_t>(1, (h->r.m * ncolw + slots - 1) / slots);
    while (rows < 32 && (h->r.m + rows - 1) / rows * ncolw > slots) ++rows;
    return int(std::min<int64_t>(rows, 32));
}

// One launch advancing T iterations.  w is updated in place when allowed.
// check: the launch also takes the check of its last iteration (its quad
// sums go to h->quad; rows must then be a multiple of MET_ROWS).
omt_status step_launch(omt_ctx *h, int T, int rows, bool w_inplace, hipStream_t stream = nullptr, bool check = false)
{
    if (!stream) stream = h->stream;
    const Resolved &r = h->r;
    if (r.p > 1) {
        // 3-D grids: one iteration per launch, rows = slices per wave; the
        // halo lanes and rows never read w, so w may be updated in place
        if (T != 1 || check)
            return fail(OMT_EUNSUPPORTED, "3-D grids run one iteration per launch (asked for T = %d)", T);
        const int wo = w_inplace ? h->wcur : 1 - h->wcur;
        hipError_t e;
        if (r.dtype == OMT_F64) {
            Step3Args<double> a;
            fill_args3(a, h, h->cur, 1 - h->cur, h->wcur, wo, rows);
            e = launch_step3(r.dtype, r.k, r.gk, r.lb, &a, stream);
        } else {
            Step3Args<float> a;
            fill_args3(a, h, h->cur, 1 - h->cur, h->wcur, wo, rows);
            e = launch_step3(r.dtype, r.k, r.gk, r.lb, &a, stream);
        }
        if (e != hipSuccess) return fail(OMT_EDEVICE, "3-D step launch: %s", hipGetErrorString(e));
        h->cur = 1 - h->cur;
        if (!w_inplace) h->wcur = 1 - h->wcur;
        h->iters_done += 1;
        return OMT_OK;
    }
    if (!step_supported(r.dtype, r.k, r.gk, r.lb, T, r.comp))
        return fail(OMT_EUNSUPPORTED, "no step kernel for dtype %d, k %d, graph kind %d (%d edges), T %d%s", r.dtype,
                    r.k, r.gk, r.lb, T, r.comp ? ", compensated" : "");
    if (T > 1) w_inplace = false;  // halo lanes of a pipelined step must see the old w
    const int ncolw = (r.n + strip_cols(T) - 1) / strip_cols(T);
    const int nroww = (r.m + rows - 1) / rows;
    const int nwg = ncolw * ((nroww + STEP_WAVES_PER_WG - 1) / STEP_WAVES_PER_WG);
    StepLaunch Lc;
    Lc.dtype = r.dtype;
    Lc.k = r.k;
    Lc.gk = r.gk;
    Lc.lb = r.lb;
    Lc.T = T;
    Lc.comp = r.comp;
    Lc.stream = stream;
    Lc.check = check;
    hipError_t e;
    const int wo = w_inplace ? h->wcur : 1 - h->wcur;
    if (r.dtype == OMT_F64) {
        StepArgs<double> a;
        fill_args(a, h, h->cur, 1 - h->cur, h->wcur, wo, rows, ncolw, nroww, nwg);
        Lc.args = &a;
        e = launch_step(Lc);
    } else {
        StepArgs<float> a;
        fill_args(a, h, h->cur, 1 - h->cur, h->wcur, wo, rows, ncolw, nroww, nwg);
        Lc.args = &a;
        e = launch_step(Lc);
    }
    if (e != hipSuccess) return fail(OMT_EDEVICE, "step launch: %s", hipGetErrorString(e));
    h->cur = 1 - h->cur;
    if (!w_inplace) h->wcur = 1 - h->wcur;
    h->iters_done += T;
    return OMT_OK;
}

// Metrics of (old -> new) state buffers; results into h->res[0..NMET).
omt_status run_metrics(omt_ctx *h, int old_c, int new_c, int old_w, int new_w, hipStream_t stream = nullptr)
{
    if (!stream) stream = h->stream;
    const Resolved &r = h->r;
    if (r.p > 1) {
        const int ncolw = (r.n + WAVE - 1) / WAVE;
        const int ntiles = ncolw * ((r.m + MET_ROWS - 1) / MET_ROWS) * r.p;
        Metrics3Launch Lm;
        Lm.dtype = r.dtype;
        Lm.k = r.k;
        Lm.gk = r.gk;
        Lm.lb = r.lb;
        Lm.alpha = r.alpha;
        Lm.eps = r.eps;
        Lm.ncolw = ncolw;
        Lm.ntiles = ntiles;
        Lm.partials = h->part;
        Lm.stream = stream;
        hipError_t e;
        if (r.dtype == OMT_F64) {
            Step3Args<double> a;
            fill_args3(a, h, old_c, new_c, old_w, new_w, 1);
            Lm.args = &a;
            e = launch_metrics3(Lm);
        } else {
            Step3Args<float> a;
            fill_args3(a, h, old_c, new_c, old_w, new_w, 1);
            Lm.args = &a;
            e = launch_metrics3(Lm);
        }
        if (e != hipSuccess) return fail(OMT_EDEVICE, "3-D metrics launch: %s", hipGetErrorString(e));
        HIP_TRY(launch_reduce_tiles(h->part, ntiles, h->res, stream));
        return OMT_OK;
    }
    const int ncolw = (r.n + WAVE - 1) / WAVE;
    const int ntiles = ncolw * ((r.m + MET_ROWS - 1) / MET_ROWS);
    StepLaunch Lc;
    Lc.dtype = r.dtype;
    Lc.k = r.k;
    Lc.gk = r.gk;
    Lc.lb = r.lb;
    Lc.T = 1;
    Lc.comp = r.comp;
    Lc.stream = stream;
    hipError_t e;
    if (r.dtype == OMT_F64) {
        StepArgs<double> a;
        fill_args(a, h, old_c, new_c, old_w, new_w, 16, ncolw, 0, 0);
        Lc.args = &a;
        e = launch_tile_metrics(Lc, ncolw, ntiles, h->part);
    } else {
        StepArgs<float> a;
        fill_args(a, h, old_c, new_c, old_w, new_w, 16, ncolw, 0, 0);
        Lc.args = &a;
        e = launch_tile_metrics(Lc, ncolw, ntiles, h->part);
    }
    if (e != hipSuccess) return fail(OMT_EDEVICE, "metrics launch: %s", hipGetErrorString(e));
    HIP_TRY(launch_reduce_tiles(h->part, ntiles, h->res, stream));
    return OMT_OK;
}

omt_status read_results(omt_ctx *h, int count, hipStream_t stream = nullptr)
{
    if (!stream) stream = h->stream;
    HIP_TRY(hipMemcpyAsync(h->host, h->res, sizeof(double) * count, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return OMT_OK;
}

void fill_info(omt_ctx *h, const double *met, omt_info *info)
{
    const Resolved &r = h->r;
    const double R = met[0] / r.mu + (r.l > 0 ? met[1] / r.nu : 0.0) + met[2] / r.tau - 2.0 * met[3];
    const double R0 = r.tau * h->fnorm2;
    info->R = R;
    info->residual = R0 > 0.0 ? std::sqrt(std::max(R, 0.0) / R0) : 0.0;
    if (!std::isfinite(R)) info->residual = R;
    info->primal = met[4];
    info->dual = met[5];
    info->rel_gap = met[4] > 0.0 ? (met[4] - met[5]) / met[4] : 0.0;
    info->mass_residual = h->fnorm2 > 0.0 ? std::sqrt(met[6] / h->fnorm2) : 0.0;
}

int tblock_of(const omt_ctx *h)
{
    if (h->r.p > 1) return 1;
    if (h->r.tblock > 0) return h->r.tblock;
    if (h->tuned_T > 0) return h->tuned_T;
    // untuned: two iterations per HBM pass where single-iteration strips
    // are tall (large grids), when compiled.  FP32, measured with the
    // autotuner's best shape against T = 1: 1.21x at 1024^2 k = 8, 1.36x at
    // 2048^2 k = 8, 1.31x at 1024^2 k = 3, 1.36x at 1024^2 k = 1; a tie at
    // 512^2 k = 8 (2 rows per wave) and none at 256^2 (1 row).  FP64 (k <= 3)
    // gains already at 2 rows: with the rule's rows 1.16x at 384^2 k = 3,
    // 1.28x at 384^2 k = 1, 1.05x at 512^2 k = 3, 1.18x at 512^2 k = 1, a tie
    // at 320^2 (1 row) and a loss at 256^2
    const int tall = h->r.dtype == OMT_F64 ? 2 : 4;
    if (rule_rows(h, 1) >= tall && step_supported(h->r.dtype, h->r.k, h->r.gk, h->r.lb, 2, h->r.comp)) return 2;
    return 1;
}

// ------------------------------------------------------------ tuning cache
//
// A JSON object, one entry per line: "key": {"T": t, "rows": r, "us": x},
// keyed by device architecture, channels, graph kind, edges, dtype,
// compensation and grid size.  Read at create, written by omt_autotune.

std::string tune_key(const omt_ctx *h)
{
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    char buf[256];
    snprintf(buf, sizeof(buf), "%s k%d g%d l%d %s c%d %dx%d", arch.c_str(), h->r.k, h->r.gk, h->r.l,
             h->r.dtype == OMT_F64 ? "f64" : "f32", h->r.comp ? 1 : 0, h->r.m, h->r.n);
    return buf;
}

struct TuneEntry {
    std::string key;
    int T, rows;
    double us;
};

std::vector<TuneEntry> tune_cache_read(const char *path)
{
    std::vector<TuneEntry> out;
    FILE *fp = path ? std::fopen(path, "r") : nullptr;
    if (!fp) return out;
    char line[512];
    while (std::fgets(line, sizeof(line), fp)) {
        char key[256];
        TuneEntry t;
        if (std::sscanf(line, " \"%255[^\"]\": {\"T\": %d, \"rows\": %d, \"us\": %lf", key, &t.T, &t.rows, &t.us) == 4) {
            t.key = key;
            out.push_back(t);
        }
    }
    std::fclose(fp);
    return out;
}

void tune_cache_load(omt_ctx *h)
{
    const char *path = std::getenv("OMT_TUNE_CACHE");
    if (!path) return;
    const std::string key = tune_key(h);
    for (const TuneEntry &t : tune_cache_read(path))
        if (t.key == key && step_supported(h->r.dtype, h->r.k, h->r.gk, h->r.lb, t.T, h->r.comp) && t.rows > 0) {
            h->tuned_T = t.T;
            h->tuned_rows = t.rows;
        }
}

void tune_cache_store_key(const std::string &key, int T, int rows, double us)
{
    const char *path = std::getenv("OMT_TUNE_CACHE");
    if (!path) return;
    std::vector<TuneEntry> all = tune_cache_read(path);
    bool found = false;
    for (TuneEntry &t : all)
        if (t.key == key) {
            t.T = T;
            t.rows = rows;
            t.us = us;
            found = true;
        }
    if (!found) all.push_back(TuneEntry{key, T, rows, us});
    const std::string tmp = std::string(path) + ".tmp";
    FILE *fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return;
    std::fprintf(fp, "{\n");
    for (size_t q = 0; q < all.size(); ++q)
        std::fprintf(fp, "\"%s\": {\"T\": %d, \"rows\": %d, \"us\": %.3f}%s\n", all[q].key.c_str(), all[q].T,
                     all[q].rows, all[q].us, q + 1 < all.size() ? "," : "");
    std::fprintf(fp, "}\n");
    std::fclose(fp);
    std::rename(tmp.c_str(), path);
}

void tune_cache_store(const omt_ctx *h, int T, int rows, double us) { tune_cache_store_key(tune_key(h), T, rows, us); }

// Rows per strip the batched solver's tuner stored for this problem's shape
// class, or 0.
int tune_cache_batch_rows(const omt_ctx *h)
{
    const char *path = std::getenv("OMT_TUNE_CACHE");
    if (!path) return 0;
    const std::string key = "batch " + tune_key(h);
    int rows = 0;
    for (const TuneEntry &t : tune_cache_read(path))
        if (t.key == key && t.T == 1 && t.rows > 0) rows = t.rows;
    return rows;
}

// Rows per wave of a check launch: a multiple of MET_ROWS near the step's,
// so that each aligned row block of the check sums lies in one wave.
int check_rows(int rows) { return std::max(MET_ROWS, (rows + MET_ROWS / 2) / MET_ROWS * MET_ROWS); }

// The single-iteration launch that also takes its check, then the check
// sums reduced in a fixed order into h->res: quads to tiles to totals.
omt_status check_launch(omt_ctx *h, int rows, hipStream_t stream)
{
    omt_status s = step_launch(h, 1, check_rows(rows), true, stream, true);
    if (s != OMT_OK) return s;
    const int ncolw = (h->r.n + WAVE - 1) / WAVE;
    HIP_TRY(launch_quads_to_tiles(h->quad, h->L.qstride, h->L.nq, h->L.nqb, ncolw, h->part, stream));
    HIP_TRY(launch_reduce_tiles(h->part, ncolw * h->L.nqb, h->res, stream));
    return OMT_OK;
}

// Enqueue one check interval of nblk iterations on stream: nblk - 1
// iterations T per launch while T fits, then single ones, then the checked
// iteration (R^k needs its old and new iterates).  Vector problems take the
// check inside that single-iteration launch (two-iteration launches with the
// check measured slower: its registers leave one wave per SIMD); matrix
// problems keep both iterates and run the separate metrics pass.
omt_status enqueue_interval(omt_ctx *h, int64_t nblk, int T, int rowsT, int rows1, hipStream_t stream)
{
    omt_status s;
    int64_t rest = nblk - 1;
    while (T > 1 && rest >= T) {
        if ((s = step_launch(h, T, rowsT, false, stream)) != OMT_OK) return s;
        rest -= T;
    }
    while (rest > 0) {
        if ((s = step_launch(h, 1, rows1, true, stream)) != OMT_OK) return s;
        --rest;
    }
    if (h->r.p == 1 && check_compiled(h->r.gk)) return check_launch(h, rows1, stream);
    const int oc = h->cur, ow = h->wcur;
    if ((s = step_launch(h, 1, rows1, false, stream)) != OMT_OK) return s;
    return run_metrics(h, oc, h->cur, ow, h->wcur, stream);
}

// A full check interval replayed as one HIP graph, captured on first use for
// the current buffer roles.  Every interval permutes the roles the same way
// (each launch swaps phi/u, each out-of-place launch swaps w), so at most two
// role sets alternate and two graphs cover a solve.
omt_status graph_interval(omt_ctx *h, int K, int T, int rowsT, int rows1)
{
    omt_ctx::Graph *g = nullptr;
    for (int q = 0; q < h->ngraphs; ++q) {
        omt_ctx::Graph &c = h->graphs[q];
        if (c.K == K && c.T == T && c.rowsT == rowsT && c.rows1 == rows1 && c.cur == h->cur && c.wcur == h->wcur)
            g = &c;
    }
    const int c0 = h->cur, w0 = h->wcur;
    const int64_t it0 = h->iters_done;
    if (!g) {
        if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        if (h->ngraphs == 2) {
            (void)hipGraphExecDestroy(h->graphs[0].exec);
            h->graphs[0] = h->graphs[1];
            h->ngraphs = 1;
        }
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
        omt_status s = enqueue_interval(h, K, T, rowsT, rows1, h->cap);
        hipError_t e = hipStreamEndCapture(h->cap, &graph);
        // capturing ran nothing: note where the launches leave the buffer
        // roles, then put the handle back
        const int c1 = h->cur, w1 = h->wcur;
        h->cur = c0;
        h->wcur = w0;
        h->iters_done = it0;
        if (s != OMT_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return s;
        }
        if (e != hipSuccess) return fail(OMT_EDEVICE, "capture: %s", hipGetErrorString(e));
        omt_ctx::Graph ng;
        ng.K = K;
        ng.T = T;
        ng.rowsT = rowsT;
        ng.rows1 = rows1;
        ng.cur = c0;
        ng.wcur = w0;
        ng.cur_after = c1;
        ng.wcur_after = w1;
        e = hipGraphInstantiateWithFlags(&ng.exec, graph, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(OMT_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
        h->graphs[h->ngraphs++] = ng;
        g = &h->graphs[h->ngraphs - 1];
    }
    HIP_TRY(hipGraphLaunch(g->exec, h->cap));
    // the replay moves the buffers exactly as the captured launches did
    h->cur = g->cur_after;
    h->wcur = g->wcur_after;
    h->iters_done = it0 + K;
    return read_results(h, NMET, h->cap);
}

omt_status create_resolved(const Resolved &r, const void *rho0, const void *rho1, void *workspace, size_t ws_bytes,
                           void *stream, omt_handle *out);
omt_status setup_ctx(omt_ctx *h, const Resolved &r, const void *rho0, const void *rho1, void *workspace,
                     size_t ws_bytes, void *stream);

// The iterations of omt_solve: intervals of check_every iterations, each
// ending with the check of Sec. 6.1; full intervals are replayed as HIP
// graphs when allow_graph is set (graphs allocate when first captured).
omt_status solve_ctx(omt_ctx *h, int64_t max_iters, double tol, int32_t check_every, omt_info *info,
                     bool allow_graph)
{
    if (max_iters < 0) return fail(OMT_EINVAL, "max_iters < 0");
    const int K = check_every > 0 ? check_every : 64;
    const int T = tblock_of(h);
    omt_info inf;
    std::memset(&inf, 0, sizeof(inf));
    omt_status s = OMT_OK;
    int64_t it = 0;
    const int rowsT = default_rows(h, T), rows1 = default_rows(h, 1);
    const bool use_graph = allow_graph && K >= 8;
    if (use_graph) HIP_TRY(hipStreamSynchronize(h->stream));
    const int verbosity = log_level();
    const auto t_start = std::chrono::steady_clock::now();
    while (it < max_iters) {
        TraceRange range("omt check interval");
        const int64_t nblk = std::min<int64_t>(K, max_iters - it);
        if (use_graph && nblk == K) {
            if ((s = graph_interval(h, K, T, rowsT, rows1)) != OMT_OK) return s;
        } else {
            if ((s = enqueue_interval(h, nblk, T, rowsT, rows1, h->stream)) != OMT_OK) return s;
            if ((s = read_results(h, NMET)) != OMT_OK) return s;
        }
        it += nblk;
        fill_info(h, h->host, &inf);
        inf.iters = it;
        inf.checks += 1;
        if (verbosity >= 3)
            std::fprintf(stderr, "omt: %lld iterations: residual %.3e, primal %.9g, dual %.9g, gap %.2e\n",
                         (long long)it, inf.residual, inf.primal, inf.dual, inf.rel_gap);
        if (!std::isfinite(inf.R) || !std::isfinite(inf.primal)) {
            h->last = inf;
            h->have_last = true;
            if (info) *info = inf;
            return fail(OMT_EDIVERGED, "non-finite residual after %lld iterations", (long long)it);
        }
        // same test as the batched kernel: R <= tol^2 R0
        if (tol > 0.0 && inf.R <= tol * tol * (h->r.tau * h->fnorm2)) {
            inf.converged = 1;
            break;
        }
    }
    h->last = inf;
    h->have_last = true;
    if (info) *info = inf;
    if (verbosity >= 2) {
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        std::fprintf(stderr, "omt: solve of %dx%dx%d k %d: %lld iterations in %.3f ms (T %d, %d rows), residual %.3e%s\n",
                     h->r.m, h->r.n, h->r.p, h->r.k, (long long)it, ms, T, rowsT, inf.residual,
                     inf.converged ? ", converged" : "");
    }
    if (tol > 0.0 && !inf.converged) return fail(OMT_ENOTCONV, "residual %.3g > tol %.3g after %lld iterations",
                                                  inf.residual, tol, (long long)it);
    return OMT_OK;
}

// ------------------------------------------------ static workspace
//
// omt_solve_static runs with its device workspace in `scratch`, a fixed
// array of the library's code object: the loader gives every GPU its own
// copy when the library first runs there, and it stays until the process
// ends.  Host code never uses the array's name as an address (in host code
// it stands for a host-side shadow): the device address of the current
// GPU's copy comes from hipGetSymbolAddress, once per device, and only that
// address is handed to kernels.
#ifndef OMT_STATIC_WORKSPACE_BYTES
#define OMT_STATIC_WORKSPACE_BYTES (64u << 20)
#endif
static_assert(OMT_STATIC_WORKSPACE_BYTES % 256 == 0, "static workspace keeps 256-byte alignment");

}  // namespace

static __device__ __align__(256) unsigned char scratch[OMT_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu;
void *g_static_ptr[STATIC_MAX_DEVICES];

// Device address of the current GPU's copy of `scratch`.
omt_status static_workspace(void **ptr)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= STATIC_MAX_DEVICES)
        return fail(OMT_EUNSUPPORTED, "device %d: the static workspace serves devices 0..%d", dev,
                    STATIC_MAX_DEVICES - 1);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(OMT_EDEVICE, "device %d: address of the static workspace: %s", dev, hipGetErrorString(e));
        g_static_ptr[dev] = p;
    }
    *ptr = g_static_ptr[dev];
    return OMT_OK;
}

}  // namespace

// ================================================================== C ABI

extern "C" {

void omt_params_init(omt_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->alpha = 1.0;
    p->tau = 1.0;
    p->unorm = OMT_U_L12;
    p->wnorm = OMT_W_L1;
    p->dtype = OMT_F32;
}

omt_status omt_resolve_params(const omt_params *p, double *h, double *mu, double *nu, double *lambda_max)
{
    Resolved r;
    omt_status s = resolve(p, r);
    if (s != OMT_OK) return s;
    if (h) *h = r.h;
    if (mu) *mu = r.mu;
    if (nu) *nu = r.nu;
    if (lambda_max) *lambda_max = r.lmax;
    return OMT_OK;
}

omt_status omt_workspace_bytes(const omt_params *p, size_t *bytes)
{
    if (!bytes) return fail(OMT_EINVAL, "bytes is NULL");
    Resolved r;
    omt_status s = resolve(p, r);
    if (s != OMT_OK) return s;
    *bytes = make_layout(r).total;
    return OMT_OK;
}

omt_status omt_create(const omt_params *p, const void *rho0, const void *rho1, void *workspace, size_t ws_bytes,
                      void *stream, omt_handle *out)
{
    TraceRange range("omt_create");
    if (!out) return fail(OMT_EINVAL, "out is NULL");
    *out = nullptr;
    Resolved r;
    omt_status s = resolve(p, r);
    if (s != OMT_OK) return s;
    return create_resolved(r, rho0, rho1, workspace, ws_bytes, stream, out);
}

}  // extern "C"

namespace {

// The set-up of omt_create for an already resolved problem (also used by the
// matrix method, whose data arrive packed into coordinates).
omt_status create_resolved(const Resolved &r, const void *rho0, const void *rho1, void *workspace, size_t ws_bytes,
                           void *stream, omt_handle *out)
{
    omt_ctx *h = new omt_ctx();
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&h->host), sizeof(double) * 64, hipHostMallocDefault);
    if (e != hipSuccess) {
        delete h;
        return fail(OMT_EDEVICE, "set-up: %s", hipGetErrorString(e));
    }
    omt_status s = setup_ctx(h, r, rho0, rho1, workspace, ws_bytes, stream);
    if (s != OMT_OK) {
        (void)hipHostFree(h->host);
        delete h;
        return s;
    }
    tune_cache_load(h);
    *out = h;
    return OMT_OK;
}

// Everything omt_create does on the device, into a context whose host
// buffer (64 doubles) the caller provides: mass check per class, f = rho1 -
// rho0 minus the class mean, zero state, ||f||^2.  Allocates nothing.
omt_status setup_ctx(omt_ctx *h, const Resolved &r, const void *rho0, const void *rho1, void *workspace,
                     size_t ws_bytes, void *stream)
{
    omt_status s = OMT_OK;
    if (!rho0 || !rho1) return fail(OMT_EINVAL, "rho0 / rho1 is NULL");
    if (!workspace) return fail(OMT_EINVAL, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(OMT_EINVAL, "workspace not 256-byte aligned");
    const Layout L = make_layout(r);
    if (ws_bytes < L.total) return fail(OMT_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, L.total);

    h->r = r;
    h->L = L;
    h->stream = static_cast<hipStream_t>(stream);
    h->ws = static_cast<char *>(workspace);
    h->f = h->ws + L.off_f;
    for (int b = 0; b < 2; ++b) {
        h->phi[b] = h->ws + L.off_phi[b];
        h->u[b] = h->ws + L.off_u[b];
        h->w[b] = h->ws + L.off_w[b];
        h->plo[b] = r.comp ? reinterpret_cast<float *>(h->ws + L.off_plo[b]) : nullptr;
    }
    h->part = reinterpret_cast<double *>(h->ws + L.off_part);
    h->quad = reinterpret_cast<double *>(h->ws + L.off_quad);
    h->res = reinterpret_cast<double *>(h->ws + L.off_res);
    h->vec = reinterpret_cast<double *>(h->ws + L.off_vec);
    h->cur = h->wcur = 0;
    h->iters_done = 0;
    h->have_last = false;
    const int64_t npix = (int64_t)r.m * r.n * r.p;
    h->metric_blocks = int(std::min<int64_t>(METRIC_BLOCKS_MAX, (npix + 255) / 256));
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) return fail(OMT_EDEVICE, "set-up: %s", hipGetErrorString(e));

    // FP64 per-channel masses and non-finite count of the inputs
    SumsArgs sa;
    sa.rho0 = rho0;
    sa.rho1 = rho1;
    sa.dtype = r.dtype;
    sa.npix = npix;
    sa.k = r.k;
    sa.partials = h->part;
    sa.nblocks = int(std::min<int64_t>(SUM_BLOCKS_MAX, (npix + 255) / 256));
    const int W = 4 * r.k + 1;
    e = launch_sums(sa, h->stream);
    if (e == hipSuccess) e = launch_reduce_rows(h->part, sa.nblocks, W, h->res, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(h->host, h->res, sizeof(double) * W, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(OMT_EDEVICE, "mass check: %s", hipGetErrorString(e));
    double sums[4 * KMAX + 1];
    std::memcpy(sums, h->host, sizeof(double) * W);
    if (sums[4 * r.k] > 0.0) return fail(OMT_EINVAL, "%.0f non-finite input values", sums[4 * r.k]);
    double s0[KMAX] = {0.0}, s1[KMAX] = {0.0}, a0[KMAX] = {0.0}, a1[KMAX] = {0.0}, cnt[KMAX] = {0.0};
    for (int c = 0; c < r.k; ++c) {
        const int g = r.cls[c];
        if (g < 0) continue;
        s0[g] += sums[4 * c];
        s1[g] += sums[4 * c + 1];
        a0[g] += sums[4 * c + 2];
        a1[g] += sums[4 * c + 3];
        cnt[g] += double(npix);
    }
    for (int g = 0; g < r.ncls; ++g) {
        const double den = std::max(a0[g], a1[g]);
        const double rel = den > 0.0 ? std::fabs(s0[g] - s1[g]) / den : 0.0;
        if (rel > 1e-6)
            return fail(OMT_EMASS, "mass class %d: sum rho0 = %.9g, sum rho1 = %.9g (relative %.3g > 1e-6)", g,
                        s0[g], s1[g], rel);
    }
    for (int c = 0; c < r.k; ++c) h->host[c] = r.cls[c] < 0 ? 0.0 : (s1[r.cls[c]] - s0[r.cls[c]]) / cnt[r.cls[c]];
    e = hipMemcpyAsync(h->vec, h->host, sizeof(double) * r.k, hipMemcpyHostToDevice, h->stream);
    // f = rho1 - rho0 - class mean, state = 0
    MakeFArgs fa;
    fa.rho0 = rho0;
    fa.rho1 = rho1;
    fa.dtype = r.dtype;
    fa.m = r.m;
    fa.p = r.p;
    fa.n = r.n;
    fa.k = r.k;
    fa.pitch = L.pitch;
    fa.plane = L.plane;
    fa.shift = h->vec;
    fa.f = h->f;
    if (e == hipSuccess) e = launch_zero(h->ws, L.off_part, h->stream);
    if (e == hipSuccess) e = launch_make_f(fa, h->stream);
    if (e == hipSuccess && std::getenv("OMT_POISON")) {
        // padding of f, phi, u, w (one plane stride apart), then of the
        // compensated low parts (FP32 planes)
        const size_t pb = align256(size_t(L.plane) * L.esz), pf = align256(size_t(L.plane) * 4);
        const int64_t rows = int64_t(r.m) * r.p;
        const int64_t nfield = int64_t(r.k) * 3 + int64_t(ucomp(r)) * r.k * 2 + int64_t(r.l) * 2;
        e = launch_poison(h->ws + L.off_f, nfield, pb, L.pitch, rows, r.n, int(L.esz), h->stream);
        if (e == hipSuccess && r.comp)
            e = launch_poison(h->ws + L.off_plo[0], int64_t(r.k) * 2, pf, L.pitch, rows, r.n, 4, h->stream);
    }
    if (e != hipSuccess) return fail(OMT_EDEVICE, "set-up: %s", hipGetErrorString(e));
    // ||f||^2 from the objectives of the zero state
    s = run_metrics(h, 0, 0, 0, 0);
    if (s == OMT_OK) s = read_results(h, NMET);
    if (s != OMT_OK) return s;
    h->fnorm2 = h->host[6];
    return OMT_OK;
}

}  // namespace

extern "C" {

omt_status omt_solve(omt_handle h, int64_t max_iters, double tol, int32_t check_every, omt_info *info)
{
    TraceRange range("omt_solve");
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    // full intervals are replayed as graphs unless OMT_NO_GRAPH is set
    return solve_ctx(h, max_iters, tol, check_every, info, !std::getenv("OMT_NO_GRAPH"));
}

omt_status omt_distance(omt_handle h, double *V, omt_info *info)
{
    TraceRange range("omt_distance");
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    omt_status s = run_metrics(h, h->cur, h->cur, h->wcur, h->wcur);
    if (s == OMT_OK) s = read_results(h, NMET);
    if (s != OMT_OK) return s;
    omt_info inf;
    std::memset(&inf, 0, sizeof(inf));
    fill_info(h, h->host, &inf);
    if (h->have_last) {
        inf.iters = h->last.iters;
        inf.residual = h->last.residual;
        inf.R = h->last.R;
        inf.converged = h->last.converged;
        inf.checks = h->last.checks;
    }
    if (V) *V = inf.primal;
    if (info) *info = inf;
    return OMT_OK;
}

omt_status omt_grad(omt_handle h, void *d_rho0, void *d_rho1)
{
    TraceRange range("omt_grad");
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    const Resolved &r = h->r;
    PlaneSumArgs pa;
    pa.phi = h->phi[h->cur];
    pa.plo = r.comp ? h->plo[h->cur] : nullptr;
    pa.dtype = r.dtype;
    pa.m = r.m * r.p;  // the plane's rows: every (slice, row) of a 3-D grid
    pa.n = r.n;
    pa.k = r.k;
    pa.pitch = h->L.pitch;
    pa.plane = h->L.plane;
    pa.partials = h->part;
    pa.nblocks = h->metric_blocks;
    HIP_TRY(launch_plane_sums(pa, h->stream));
    HIP_TRY(launch_reduce_rows(h->part, pa.nblocks, r.k, h->res, h->stream));
    omt_status s = read_results(h, r.k);
    if (s != OMT_OK) return s;
    double cs[KMAX] = {0.0}, cn[KMAX] = {0.0};
    for (int c = 0; c < r.k; ++c) {
        if (r.cls[c] < 0) continue;
        cs[r.cls[c]] += h->host[c];
        cn[r.cls[c]] += double(r.m) * r.n * r.p;
    }
    for (int c = 0; c < r.k; ++c) h->host[c] = r.cls[c] < 0 ? 0.0 : cs[r.cls[c]] / cn[r.cls[c]];
    HIP_TRY(hipMemcpyAsync(h->vec, h->host, sizeof(double) * r.k, hipMemcpyHostToDevice, h->stream));
    XferArgs xa;
    xa.src = h->phi[h->cur];
    xa.plo = pa.plo;
    xa.plo_out = nullptr;
    xa.dtype = r.dtype;
    xa.m = r.m;
    xa.p = r.p;
    xa.n = r.n;
    xa.k = r.k;
    xa.pitch = h->L.pitch;
    xa.plane = h->L.plane;
    xa.mode = 0;
    xa.mean = h->vec;
    if (d_rho0) {
        xa.dst = d_rho0;
        xa.sign = 1.0;
        HIP_TRY(launch_xfer(xa, h->stream));
    }
    if (d_rho1) {
        xa.dst = d_rho1;
        xa.sign = -1.0;
        HIP_TRY(launch_xfer(xa, h->stream));
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    return OMT_OK;
}

omt_status omt_get_state(omt_handle h, void *phi, void *u, void *w)
{
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    const Resolved &r = h->r;
    XferArgs xa;
    std::memset(&xa, 0, sizeof(xa));
    xa.dtype = r.dtype;
    xa.m = r.m;
    xa.p = r.p;
    xa.n = r.n;
    xa.pitch = h->L.pitch;
    xa.plane = h->L.plane;
    if (phi) {
        xa.src = h->phi[h->cur];
        xa.plo = r.comp ? h->plo[h->cur] : nullptr;
        xa.dst = phi;
        xa.k = r.k;
        xa.mode = 2;
        HIP_TRY(launch_xfer(xa, h->stream));
    }
    if (u) {
        xa.src = h->u[h->cur];
        xa.plo = nullptr;
        xa.dst = u;
        xa.k = r.k;
        xa.mode = 1;
        HIP_TRY(launch_xfer(xa, h->stream));
    }
    if (w && r.l > 0) {
        xa.src = h->w[h->wcur];
        xa.plo = nullptr;
        xa.dst = w;
        xa.k = r.l;
        xa.mode = 2;
        HIP_TRY(launch_xfer(xa, h->stream));
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    return OMT_OK;
}

omt_status omt_set_state(omt_handle h, const void *phi, const void *u, const void *w)
{
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    const Resolved &r = h->r;
    XferArgs xa;
    std::memset(&xa, 0, sizeof(xa));
    xa.dtype = r.dtype;
    xa.m = r.m;
    xa.p = r.p;
    xa.n = r.n;
    xa.pitch = h->L.pitch;
    xa.plane = h->L.plane;
    xa.src = phi;
    xa.dst = h->phi[h->cur];
    xa.plo_out = r.comp ? h->plo[h->cur] : nullptr;
    xa.k = r.k;
    xa.mode = 3;
    HIP_TRY(launch_xfer(xa, h->stream));
    xa.src = u;
    xa.dst = h->u[h->cur];
    xa.plo_out = nullptr;
    xa.mode = 4;
    HIP_TRY(launch_xfer(xa, h->stream));
    if (r.l > 0) {
        xa.src = w;
        xa.dst = h->w[h->wcur];
        xa.k = r.l;
        xa.mode = 3;
        HIP_TRY(launch_xfer(xa, h->stream));
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->have_last = false;
    return OMT_OK;
}

omt_status omt_destroy(omt_handle h)
{
    if (!h) return OMT_OK;
    for (int q = 0; q < h->ngraphs; ++q) (void)hipGraphExecDestroy(h->graphs[q].exec);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->host) (void)hipHostFree(h->host);
    delete h;
    return OMT_OK;
}

omt_status omt_time_steps(omt_handle h, int32_t T, int32_t rows_per_wave, int64_t n, double *us_per_launch)
{
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    if (T < 1 || n < T || n % T != 0) return fail(OMT_EINVAL, "need T >= 1 dividing n (T %d, n %lld)", T, (long long)n);
    if (rows_per_wave < 0) return fail(OMT_EINVAL, "rows_per_wave < 0");
    const int rows = rows_per_wave > 0 ? rows_per_wave : default_rows(h, T);
    // The timed launches are captured into a HIP graph and replayed once on
    // the handle's private stream, as the solve replays its check
    // intervals, so that the time is that of the kernels back to back and not
    // of the host's launch rate.  An untimed launch goes first, so that the
    // queue is busy when the timed region opens: it reads the current iterate
    // and writes the other buffers (w out of place) without making them
    // current, so the timed launches start from the caller's state.
    if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const int c0 = h->cur, w0 = h->wcur;
    const int64_t it0 = h->iters_done;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    omt_status s = OMT_OK;
    for (int64_t q = 0; q < n / T && s == OMT_OK; ++q) s = step_launch(h, T, rows, T == 1, h->cap);
    hipError_t e = hipStreamEndCapture(h->cap, &graph);
    const int c1 = h->cur, w1 = h->wcur;
    const int64_t it1 = h->iters_done;
    h->cur = c0;
    h->wcur = w0;
    h->iters_done = it0;
    if (s == OMT_OK && e == hipSuccess) e = hipGraphInstantiateWithFlags(&exec, graph, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (s != OMT_OK || e != hipSuccess) {
        if (exec) (void)hipGraphExecDestroy(exec);
        return s != OMT_OK ? s : fail(OMT_EDEVICE, "timed launches: %s", hipGetErrorString(e));
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        s = step_launch(h, T, rows, false, h->cap);
        h->cur = c0;
        h->wcur = w0;
        h->iters_done = it0;
    }
    if (e == hipSuccess && s == OMT_OK) e = hipEventRecord(e0, h->cap);
    if (e == hipSuccess && s == OMT_OK) e = hipGraphLaunch(exec, h->cap);
    if (e == hipSuccess && s == OMT_OK) e = hipEventRecord(e1, h->cap);
    if (e == hipSuccess && s == OMT_OK) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess && s == OMT_OK) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipGraphExecDestroy(exec);
    if (s != OMT_OK) return s;
    if (e != hipSuccess) return fail(OMT_EDEVICE, "timed launches: %s", hipGetErrorString(e));
    h->cur = c1;
    h->wcur = w1;
    h->iters_done = it1;
    h->have_last = false;
    if (us_per_launch) *us_per_launch = 1000.0 * double(ms) / double(n / T);
    return OMT_OK;
}

omt_status omt_solve_static(const omt_params *p, const void *rho0, const void *rho1, int64_t max_iters, double tol,
                            int32_t check_every, double *V, void *d_rho0, void *d_rho1, omt_info *info, void *stream)
{
    TraceRange range("omt_solve_static");
    Resolved r;
    omt_status s = resolve(p, r);
    if (s != OMT_OK) return s;
    if (max_iters < 0) return fail(OMT_EINVAL, "max_iters < 0");
    const size_t need = make_layout(r).total;
    if (need > size_t(OMT_STATIC_WORKSPACE_BYTES))
        return fail(OMT_ENOMEM, "the problem needs %zu bytes of device workspace; the static workspace holds %zu",
                    need, size_t(OMT_STATIC_WORKSPACE_BYTES));
    void *ws = nullptr;
    if ((s = static_workspace(&ws)) != OMT_OK) return s;
    // a context on the stack with a pageable host buffer: no graph, stream,
    // pinned or device memory belongs to it, so nothing is released after
    omt_ctx h{};
    double host[64];
    h.host = host;
    if ((s = setup_ctx(&h, r, rho0, rho1, ws, need, stream)) != OMT_OK) return s;
    const omt_status sv = solve_ctx(&h, max_iters, tol, check_every, info, false);
    if (sv != OMT_OK && sv != OMT_ENOTCONV) return sv;
    if (V && (s = omt_distance(&h, V, nullptr)) != OMT_OK) return s;
    if ((d_rho0 || d_rho1) && (s = omt_grad(&h, d_rho0, d_rho1)) != OMT_OK) return s;
    if (!V && !d_rho0 && !d_rho1) HIP_TRY(hipStreamSynchronize(h.stream));
    return sv;
}

omt_status omt_autotune(omt_handle h, int32_t iters_per_trial, int32_t *best_t, int32_t *best_rows, double *best_us)
{
    TraceRange range("omt_autotune");
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    const Resolved &r = h->r;
    const size_t pb = align256(size_t(h->L.plane) * h->L.esz), pf = align256(size_t(h->L.plane) * 4);
    const size_t n_phi = pb * r.k, n_u = pb * ucomp(r) * r.k, n_w = pb * r.l, n_lo = r.comp ? pf * r.k : 0;
    const size_t total = n_phi + n_u + n_w + n_lo;
    char *snap = nullptr;
    HIP_TRY(hipMalloc(&snap, total));  // temporary copy of the state (freed below)
    std::vector<char> ref(total), got(total);
    const int c0 = h->cur, w0 = h->wcur;
    const int64_t it0 = h->iters_done;
    auto save = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(snap, h->phi[c0], n_phi, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(snap + n_phi, h->u[c0], n_u, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess && n_w)
            e = hipMemcpyAsync(snap + n_phi + n_u, h->w[w0], n_w, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess && n_lo)
            e = hipMemcpyAsync(snap + n_phi + n_u + n_w, h->plo[c0], n_lo, hipMemcpyDeviceToDevice, h->stream);
        return e;
    };
    auto restore = [&]() -> hipError_t {
        h->cur = c0;
        h->wcur = w0;
        h->iters_done = it0;
        hipError_t e = hipMemcpyAsync(h->phi[c0], snap, n_phi, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(h->u[c0], snap + n_phi, n_u, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess && n_w)
            e = hipMemcpyAsync(h->w[w0], snap + n_phi + n_u, n_w, hipMemcpyDeviceToDevice, h->stream);
        if (e == hipSuccess && n_lo)
            e = hipMemcpyAsync(h->plo[c0], snap + n_phi + n_u + n_w, n_lo, hipMemcpyDeviceToDevice, h->stream);
        return e;
    };
    auto fetch = [&](std::vector<char> &dst) -> hipError_t {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e == hipSuccess) e = hipMemcpy(dst.data(), h->phi[h->cur], n_phi, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(dst.data() + n_phi, h->u[h->cur], n_u, hipMemcpyDeviceToHost);
        if (e == hipSuccess && n_w) e = hipMemcpy(dst.data() + n_phi + n_u, h->w[h->wcur], n_w, hipMemcpyDeviceToHost);
        if (e == hipSuccess && n_lo)
            e = hipMemcpy(dst.data() + n_phi + n_u + n_w, h->plo[h->cur], n_lo, hipMemcpyDeviceToHost);
        return e;
    };
    omt_status st = OMT_OK;
    hipError_t e = save();
    const int n = std::max(8, (iters_per_trial + 7) / 8 * 8);
    int bT = 1, bR = 0;
    double bUs = 1e300, b1Us = 1e300;
    int b1R = 0;
    const int Ts[] = {1, 2, 4, 8};
    for (int T : Ts) {
        if (e != hipSuccess || st != OMT_OK) break;
        if (r.p > 1 ? T != 1 : !step_supported(r.dtype, r.k, r.gk, r.lb, T, r.comp)) continue;
        // a fixed ladder plus the one-round rule's rows and their neighbours
        // (on a 3-D grid: slices per wave and the rule's choice)
        std::vector<int> Rs = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
        const int rr = r.p > 1 ? rule_zch(h) : rule_rows(h, T);
        for (int d = -2; d <= 2; ++d)
            if (rr + d >= 1 && std::find(Rs.begin(), Rs.end(), rr + d) == Rs.end()) Rs.push_back(rr + d);
        for (int rows : Rs) {
            if (rows > (r.p > 1 ? r.p : r.m) && rows != 2) continue;
            if ((e = restore()) != hipSuccess) break;
            double us = 0.0;
            if ((st = omt_time_steps(h, T, rows, T, &us)) != OMT_OK) break;  // warm-up launch
            if ((e = restore()) != hipSuccess) break;
            if ((st = omt_time_steps(h, T, rows, n, &us)) != OMT_OK) break;
            const double per_iter = us / T;
            if (per_iter < bUs) {
                bUs = per_iter;
                bT = T;
                bR = rows;
            }
            if (T == 1 && per_iter < b1Us) {
                b1Us = per_iter;
                b1R = rows;
            }
        }
    }
    // the winner must reproduce single-iteration launches bit for bit
    bool same = true;
    if (e == hipSuccess && st == OMT_OK && bT > 1) {
        if ((e = restore()) == hipSuccess) st = omt_time_steps(h, 1, b1R, n, nullptr);
        if (e == hipSuccess && st == OMT_OK) e = fetch(ref);
        if (e == hipSuccess && st == OMT_OK) e = restore();
        if (e == hipSuccess && st == OMT_OK) st = omt_time_steps(h, bT, bR, n, nullptr);
        if (e == hipSuccess && st == OMT_OK) e = fetch(got);
        same = e == hipSuccess && st == OMT_OK && std::memcmp(ref.data(), got.data(), total) == 0;
        if (!same) {
            bT = 1;
            bR = b1R;
            bUs = b1Us;
        }
    }
    if (e == hipSuccess) e = restore();
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(snap);
    if (st != OMT_OK) return st;
    if (e != hipSuccess) return fail(OMT_EDEVICE, "autotune: %s", hipGetErrorString(e));
    h->tuned_T = bT;
    h->tuned_rows = bR;
    h->have_last = false;
    if (best_t) *best_t = bT;
    if (best_rows) *best_rows = bR;
    if (best_us) *best_us = bUs;
    tune_cache_store(h, bT, bR, bUs);
    if (!same) return fail(OMT_OK, "a blocked launch differed from single launches; tuned to T = 1");
    return OMT_OK;
}

}  // extern "C"

// ================================================================ batched

struct omt_bctx {
    int B;
    std::vector<omt_ctx *> ctx;
    hipStream_t stream;  // caller's stream
    hipStream_t cap;     // private stream the solve graph is captured and replayed on
    char *ws;
    BatchPair *d_pairs;
    BatchPairState *d_state;
    int *d_tile_pair, *d_tile_pair2, *d_mtile_pair;
    double *d_partials;
    unsigned *d_bar;
    int total_tiles, total_mtiles;  // strips / metric tiles in the current lists
    int full_tiles, full_mtiles;    // ... with every problem in them
    int cap_tiles;                  // room of the strip list (one row per strip)
    int total_tiles2;               // strips of two-iteration launches in the current list
    int T;                          // iterations per launch of the launches per iteration (1 or 2)
    int resident;                   // workgroups of the persistent kernel the chip holds at once
    int cus;                        // compute units of the device
    bool tuned;                     // rows per strip from omt_batch_autotune: kept as they are
    bool comp;
    int dtype;
    int nblocks;
    std::vector<BatchPair> pairs;
    std::vector<BatchPairState> st;
    struct Graph {
        hipGraphExec_t exec;
        int K, par0, w0;
        double tol;  // baked into the decision launches
    } graphs[2];
    int ngraphs;
    unsigned *host_stopped;  // pinned
};

namespace {

// Rows per strip in the batched kernel: a strip's rows are a chain of
// dependent steps, so small grids take short strips (their iterations are
// latency-bound) and large grids 8 rows (fewer halo rows per strip).
// Measured on the 96-pair batch: one row for the 64-pixel grids and two to
// four for the middle sizes was 2% slower overall (more halo traffic while
// every problem is active) than this rule.
int batch_rows_default(int m) { return std::max(2, std::min(8, (m + 31) / 32)); }

struct BatchLayout {
    std::vector<size_t> off, bytes;
    std::vector<int> mtiles;
    size_t off_pairs, off_state, off_tp, off_tp2, off_mtp, off_part, off_bar, total;
    int cap_tiles, cap_tiles2, total_mtiles;  // strip lists sized for one row per strip
};

omt_status batch_layout(int32_t B, const omt_params *params, BatchLayout &L, bool *comp, int *dtype)
{
    if (B < 1) return fail(OMT_EINVAL, "batch size %d < 1", B);
    if (!params) return fail(OMT_EINVAL, "params is NULL");
    size_t o = 0;
    L.cap_tiles = L.cap_tiles2 = L.total_mtiles = 0;
    for (int p = 0; p < B; ++p) {
        Resolved r;
        omt_status s = resolve(&params[p], r);
        if (s != OMT_OK) return fail(s, "problem %d: %s", p, g_last_error);
        if (p == 0) *dtype = r.dtype;
        if (r.dtype != *dtype) return fail(OMT_EINVAL, "problem %d: all problems of a batch must share the dtype", p);
        if (batch_type(r.k, r.gk, r.lb) < 0)
            return fail(OMT_EUNSUPPORTED, "problem %d: k = %d with this graph is not compiled into the batched kernel",
                        p, r.k);
        if (p == 0) *comp = r.comp;
        if (r.comp != *comp) return fail(OMT_EINVAL, "problem %d: all problems must share the compensated flag", p);
        const size_t b = make_layout(r).total;
        L.off.push_back(o);
        L.bytes.push_back(b);
        o += align256(b);
        const int ncolw = (r.n + WAVE - 1) / WAVE;
        L.mtiles.push_back(ncolw * ((r.m + MET_ROWS - 1) / MET_ROWS));
        L.cap_tiles += ncolw * r.m;
        L.cap_tiles2 += (r.n + strip_cols(2) - 1) / strip_cols(2) * r.m;
        L.total_mtiles += L.mtiles.back();
    }
    L.off_pairs = o;
    o += align256(sizeof(BatchPair) * B);
    L.off_state = o;
    o += align256(sizeof(BatchPairState) * B);
    L.off_tp = o;
    o += align256(sizeof(int) * size_t(L.cap_tiles));
    L.off_tp2 = o;
    o += align256(sizeof(int) * size_t(L.cap_tiles2));
    L.off_mtp = o;
    o += align256(sizeof(int) * L.total_mtiles);
    L.off_part = o;
    o += align256(sizeof(double) * NMET * size_t(L.total_mtiles));
    L.off_bar = o;
    o += align256(sizeof(unsigned) * BAR_WORDS);
    L.total = o;
    return OMT_OK;
}

void destroy_batch(omt_bctx *h)
{
    for (int q = 0; q < h->ngraphs; ++q) (void)hipGraphExecDestroy(h->graphs[q].exec);
    if (h->host_stopped) (void)hipHostFree(h->host_stopped);
    for (omt_ctx *c : h->ctx) omt_destroy(c);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    delete h;
}


// Persistent schedule: the whole solve in one launch with grid barriers,
// captured in a graph together with the clearing of its state.
omt_status batch_solve_persistent(omt_bctx *h, const BatchArgs &ba)
{
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_zero(h->d_state, sizeof(BatchPairState) * h->B, h->cap);
    if (e == hipSuccess) e = launch_zero(h->d_bar, sizeof(unsigned) * BAR_WORDS, h->cap);
    if (e == hipSuccess) e = launch_batch(ba, h->dtype, h->comp, h->nblocks, h->cap);
    hipError_t e2 = hipStreamEndCapture(h->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(OMT_EDEVICE, "capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiateWithFlags(&exec, graph, 0);
    if (e == hipSuccess) e = hipGraphLaunch(exec, h->cap);
    if (e == hipSuccess) e = hipStreamSynchronize(h->cap);
    if (exec) (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(OMT_EDEVICE, "batched solve: %s", hipGetErrorString(e));
    return OMT_OK;
}

// Enqueue one check interval of nblk iterations: nblk launches that advance
// every unfinished problem, then the metrics and the decisions.
hipError_t batch_enqueue_interval(omt_bctx *h, const BatchArgs &ba, int64_t nblk, int &par, int &wpar, bool last,
                                  hipStream_t s)
{
    // par / wpar: phi-u and w buffers of the iterate (relative to the solve's
    // start) before the interval, and after it on return.  Two iterations
    // per launch move phi, u and w out of place; single-iteration launches
    // update w in place except the checked last one, which keeps the old w
    // for the check.
    hipError_t e = hipSuccess;
    const int64_t n2 = h->T == 2 ? (nblk - 1) / 2 : 0;
    for (int64_t q = 0; q < n2 && e == hipSuccess; ++q) {
        e = launch_batch_step(ba, h->dtype, h->comp, 8 + par * 2 + wpar, s, 2);
        par ^= 1;
        wpar ^= 1;
    }
    for (int64_t q = 2 * n2; q < nblk - 1 && e == hipSuccess; ++q) {
        e = launch_batch_step(ba, h->dtype, h->comp, par * 4 + wpar * 2, s, 1);
        par ^= 1;
    }
    const int var = par * 4 + wpar * 2 + 1;
    if (e == hipSuccess) e = launch_batch_step(ba, h->dtype, h->comp, var, s, 1);
    par ^= 1;
    wpar ^= 1;
    if (e == hipSuccess) e = launch_batch_check(ba, h->dtype, h->comp, var, int(nblk), last, par, wpar, s);
    return e;
}

// Graph schedule: every full check interval is replayed as one captured
// graph; after each interval only the count of stopped problems is read.
// Strip and metric-tile lists of the problems marked active, in problem
// order; each problem's first strip / tile index is stored in its
// descriptor.  Uploaded on the capture stream; the descriptors are uploaded
// by the caller.
hipError_t batch_set_lists(omt_bctx *h, const std::vector<char> &active)
{
    std::vector<int> tp, tp2, mtp;
    for (int p = 0; p < h->B; ++p) {
        BatchPair &bp = h->pairs[p];
        if (!active[p]) continue;
        bp.tile0 = int(tp.size());
        bp.tile0_2 = int(tp2.size());
        bp.mtile0 = int(mtp.size());
        for (int q = 0; q < bp.ntiles; ++q) tp.push_back(p);
        if (h->T == 2)
            for (int q = 0; q < bp.ntiles2; ++q) tp2.push_back(p);
        for (int q = 0; q < bp.mtiles; ++q) mtp.push_back(p);
    }
    h->total_tiles = int(tp.size());
    h->total_tiles2 = int(tp2.size());
    h->total_mtiles = int(mtp.size());
    hipError_t e = hipSuccess;
    if (!tp.empty())
        e = hipMemcpyAsync(h->d_tile_pair, tp.data(), sizeof(int) * tp.size(), hipMemcpyHostToDevice, h->cap);
    if (e == hipSuccess && !tp2.empty())
        e = hipMemcpyAsync(h->d_tile_pair2, tp2.data(), sizeof(int) * tp2.size(), hipMemcpyHostToDevice, h->cap);
    if (e == hipSuccess && !mtp.empty())
        e = hipMemcpyAsync(h->d_mtile_pair, mtp.data(), sizeof(int) * mtp.size(), hipMemcpyHostToDevice, h->cap);
    // the host vectors go out of scope: finish the copies first
    if (e == hipSuccess) e = hipStreamSynchronize(h->cap);
    return e;
}

// Workgroups of the persistent schedule: every one resident at once, and no
// more than the strips keep busy (about two strips per wave): fewer
// workgroups make the grid barriers cheaper for small batches.
void batch_size_grid(omt_bctx *h)
{
    const int want = (h->full_tiles + 2 * STEP_WAVES_PER_WG - 1) / (2 * STEP_WAVES_PER_WG);
    h->nblocks = std::max(1, std::min(h->resident, want));
}

// Step arguments of problem p for every (parity, w buffer, check) variant,
// relative to the problem's buffers at the start of the solve.
void batch_fill_args(omt_bctx *h, int p)
{
    omt_ctx *c = h->ctx[p];
    BatchPair &bp = h->pairs[p];
    const int ncolw = bp.ncolw, rows = c->r.rows, nroww = (c->r.m + rows - 1) / rows;
    for (int var = 0; var < 8; ++var) {
        const int par = var / 4, wv = (var / 2) % 2, chk = var % 2;
        const int ci = (c->cur + par) & 1, wi = (c->wcur + wv) & 1;
        if (h->dtype == OMT_F64)
            fill_args(bp.args_mut<double>(var), c, ci, 1 - ci, wi, chk ? 1 - wi : wi, rows, ncolw, nroww, 0);
        else
            fill_args(bp.args_mut<float>(var), c, ci, 1 - ci, wi, chk ? 1 - wi : wi, rows, ncolw, nroww, 0);
    }
    // two iterations per launch: phi, u and w all out of place
    for (int var = 8; var < 12 && h->T == 2; ++var) {
        const int par = (var - 8) / 2, wv = (var - 8) % 2;
        const int ci = (c->cur + par) & 1, wi = (c->wcur + wv) & 1;
        if (h->dtype == OMT_F64)
            fill_args(bp.args_mut<double>(var), c, ci, 1 - ci, wi, 1 - wi, rows, bp.ncolw2, nroww, 0);
        else
            fill_args(bp.args_mut<float>(var), c, ci, 1 - ci, wi, 1 - wi, rows, bp.ncolw2, nroww, 0);
    }
}

// Rows per strip of the problems in the lists: the fewest rows (at most each
// problem's default) with which all their strips are resident in one round
// at two waves per SIMD, as for a single problem.  A full batch keeps the
// default rule; once only a few large problems are left they get more,
// shorter strips, which the chip would otherwise leave idle.  Rows never
// change the iterates.  Problems with rows fixed by the caller, and batches
// tuned by omt_batch_autotune, keep theirs.
void batch_retile(omt_bctx *h, const std::vector<char> &active)
{
    if (h->tuned) return;
    const int64_t slots = int64_t(h->cus) * 4 * 2;
    auto strips = [&](int R) {
        int64_t t = 0;
        for (int p = 0; p < h->B; ++p) {
            if (!active[p]) continue;
            const omt_ctx *c = h->ctx[p];
            const int rp = c->user_rows > 0 ? c->user_rows : std::min(R, batch_rows_default(c->r.m));
            t += int64_t(h->T == 2 ? h->pairs[p].ncolw2 : h->pairs[p].ncolw) * ((c->r.m + rp - 1) / rp);
        }
        return t;
    };
    int R = 1;
    while (R < 8 && strips(R) > slots) ++R;
    for (int p = 0; p < h->B; ++p) {
        omt_ctx *c = h->ctx[p];
        if (!active[p] || c->user_rows > 0) continue;
        const int rp = std::min(R, batch_rows_default(c->r.m));
        if (rp == c->r.rows) continue;
        c->r.rows = rp;
        h->pairs[p].ntiles = h->pairs[p].ncolw * ((c->r.m + rp - 1) / rp);
        h->pairs[p].ntiles2 = h->pairs[p].ncolw2 * ((c->r.m + rp - 1) / rp);
        batch_fill_args(h, p);
    }
}

void batch_drop_graphs(omt_bctx *h)
{
    for (int q = 0; q < h->ngraphs; ++q) (void)hipGraphExecDestroy(h->graphs[q].exec);
    h->ngraphs = 0;
}

omt_status batch_solve_graphs(omt_bctx *h, BatchArgs ba, int64_t max_iters, int K)
{
    HIP_TRY(launch_zero(h->d_state, sizeof(BatchPairState) * h->B, h->cap));
    HIP_TRY(launch_zero(h->d_bar, sizeof(unsigned) * BAR_WORDS, h->cap));
    int64_t done = 0;
    unsigned stopped = 0;
    const bool verbose = log_level() >= 2;
    auto last_note = std::chrono::steady_clock::now();
    int par = 0, wpar = 0;  // buffers of the iterate, relative to the solve's start
    while (done < max_iters && stopped < unsigned(h->B)) {
        const int64_t nblk = std::min<int64_t>(K, max_iters - done);
        const bool last = done + nblk == max_iters;
        const int par0 = par, w0 = wpar;
        if (nblk == K && !last) {
            omt_bctx::Graph *g = nullptr;
            for (int q = 0; q < h->ngraphs; ++q)
                if (h->graphs[q].K == K && h->graphs[q].par0 == par0 && h->graphs[q].w0 == w0 &&
                    h->graphs[q].tol == ba.tol)
                    g = &h->graphs[q];
            if (!g) {
                if (h->ngraphs == 2) {
                    (void)hipGraphExecDestroy(h->graphs[0].exec);
                    h->graphs[0] = h->graphs[1];
                    h->ngraphs = 1;
                }
                hipGraph_t graph = nullptr;
                HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
                int pc = par0, wc = w0;
                hipError_t e = batch_enqueue_interval(h, ba, K, pc, wc, false, h->cap);
                hipError_t e2 = hipStreamEndCapture(h->cap, &graph);
                if (e != hipSuccess || e2 != hipSuccess) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return fail(OMT_EDEVICE, "capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
                }
                omt_bctx::Graph ng;
                ng.K = K;
                ng.par0 = par0;
                ng.w0 = w0;
                ng.tol = ba.tol;
                e = hipGraphInstantiateWithFlags(&ng.exec, graph, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess) return fail(OMT_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
                h->graphs[h->ngraphs++] = ng;
                g = &h->graphs[h->ngraphs - 1];
            }
            HIP_TRY(hipGraphLaunch(g->exec, h->cap));
        } else {
            int pc = par0, wc = w0;
            HIP_TRY(batch_enqueue_interval(h, ba, nblk, pc, wc, last, h->cap));
        }
        // buffers after the interval: each launch moves phi and u, the
        // two-iteration launches and the checked launch also move w
        const int64_t n2 = h->T == 2 ? (nblk - 1) / 2 : 0, n1 = nblk - 1 - 2 * n2;
        par ^= int((n2 + n1 + 1) & 1);
        wpar ^= int((n2 + 1) & 1);
        done += nblk;
        HIP_TRY(hipMemcpyAsync(h->host_stopped, h->d_bar + 3, sizeof(unsigned), hipMemcpyDeviceToHost, h->cap));
        HIP_TRY(hipStreamSynchronize(h->cap));
        if (verbose) {
            // a line when problems stop, and at least every 20 s otherwise
            const auto now = std::chrono::steady_clock::now();
            if (*h->host_stopped != stopped || now - last_note > std::chrono::seconds(20)) {
                std::fprintf(stderr, "omt batch: %u of %d problems stopped after %lld iterations\n",
                             *h->host_stopped, h->B, (long long)done);
                last_note = now;
            }
        }
        const bool more = *h->host_stopped != stopped;
        stopped = *h->host_stopped;
        if (more && stopped < unsigned(h->B) && done < max_iters) {
            // drop the stopped problems from the lists once their strips are
            // a quarter of the launch: later launches then cover only the
            // problems still running (new graphs are captured for them)
            HIP_TRY(hipMemcpyAsync(h->st.data(), h->d_state, sizeof(BatchPairState) * h->B, hipMemcpyDeviceToHost,
                                   h->cap));
            HIP_TRY(hipStreamSynchronize(h->cap));
            std::vector<char> active(h->B, 0);
            int live = 0;
            for (int p = 0; p < h->B; ++p) {
                active[p] = h->st[p].done ? 0 : 1;
                if (active[p]) live += h->pairs[p].ntiles;
            }
            if (4 * live <= 3 * h->total_tiles) {
                batch_retile(h, active);
                HIP_TRY(batch_set_lists(h, active));
                HIP_TRY(hipMemcpyAsync(h->d_pairs, h->pairs.data(), sizeof(BatchPair) * h->B, hipMemcpyHostToDevice,
                                       h->cap));
                HIP_TRY(hipStreamSynchronize(h->cap));
                batch_drop_graphs(h);
                ba.total_tiles = h->total_tiles;
                ba.total_tiles2 = h->total_tiles2;
                ba.total_mtiles = h->total_mtiles;
            }
        }
    }
    return OMT_OK;
}

}  // namespace

extern "C" {

omt_status omt_batch_workspace_bytes(int32_t B, const omt_params *params, size_t *bytes)
{
    if (!bytes) return fail(OMT_EINVAL, "bytes is NULL");
    BatchLayout L;
    bool comp = false;
    int dtype = 0;
    omt_status s = batch_layout(B, params, L, &comp, &dtype);
    if (s != OMT_OK) return s;
    *bytes = L.total;
    return OMT_OK;
}

omt_status omt_batch_create(int32_t B, const omt_params *params, const void *const *rho0, const void *const *rho1,
                            void *workspace, size_t ws_bytes, void *stream, omt_batch_handle *out)
{
    if (!out) return fail(OMT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!rho0 || !rho1) return fail(OMT_EINVAL, "rho0 / rho1 is NULL");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(OMT_EINVAL, "workspace missing or not 256-byte aligned");
    BatchLayout L;
    bool comp = false;
    int dtype = 0;
    omt_status s = batch_layout(B, params, L, &comp, &dtype);
    if (s != OMT_OK) return s;
    if (ws_bytes < L.total) return fail(OMT_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, L.total);

    omt_bctx *h = new omt_bctx();
    h->B = B;
    h->stream = static_cast<hipStream_t>(stream);
    h->ws = static_cast<char *>(workspace);
    h->comp = comp;
    h->dtype = dtype;
    h->cap_tiles = L.cap_tiles;
    h->total_mtiles = h->full_mtiles = L.total_mtiles;
    h->d_pairs = reinterpret_cast<BatchPair *>(h->ws + L.off_pairs);
    h->d_state = reinterpret_cast<BatchPairState *>(h->ws + L.off_state);
    h->d_tile_pair = reinterpret_cast<int *>(h->ws + L.off_tp);
    h->d_tile_pair2 = reinterpret_cast<int *>(h->ws + L.off_tp2);
    h->d_mtile_pair = reinterpret_cast<int *>(h->ws + L.off_mtp);
    h->d_partials = reinterpret_cast<double *>(h->ws + L.off_part);
    h->d_bar = reinterpret_cast<unsigned *>(h->ws + L.off_bar);
    for (int p = 0; p < B; ++p) {
        omt_ctx *c = nullptr;
        s = omt_create(&params[p], rho0[p], rho1[p], h->ws + L.off[p], L.bytes[p], stream, &c);
        if (s != OMT_OK) {
            char why[sizeof(g_last_error)];
            std::memcpy(why, g_last_error, sizeof(why));
            destroy_batch(h);
            return fail(s, "problem %d: %s", p, why);
        }
        h->ctx.push_back(c);
    }
    // rows per strip: the caller's, else the batched tuner's cached choice
    // for the problem's shape class, else the default rule
    bool cached = false;
    for (int p = 0; p < B; ++p) {
        omt_ctx *c = h->ctx[p];
        c->user_rows = c->r.rows;
        if (c->r.rows <= 0) {
            c->r.rows = tune_cache_batch_rows(c);
            cached = cached || c->r.rows > 0;
        }
        if (c->r.rows <= 0) c->r.rows = batch_rows_default(c->r.m);
    }
    // two iterations per launch (outside the checked ones) when every problem
    // has them compiled and none asks for one per launch (tblock 1)
    bool t2 = true;
    for (int p = 0; p < B; ++p) {
        const Resolved &r = h->ctx[p]->r;
        if (r.tblock == 1 || !step_supported(r.dtype, r.k, r.gk, r.lb, 2, r.comp)) t2 = false;
    }
    h->T = t2 ? 2 : 1;
    // problem descriptors and the strip / tile lists
    std::vector<int> tp, tp2, mtp;
    h->pairs.resize(B);
    int t0 = 0, t02 = 0, m0 = 0;
    for (int p = 0; p < B; ++p) {
        omt_ctx *c = h->ctx[p];
        BatchPair &bp = h->pairs[p];
        std::memset(&bp, 0, sizeof(bp));
        const int ncolw = (c->r.n + WAVE - 1) / WAVE;
        bp.type = batch_type(c->r.k, c->r.gk, c->r.lb);
        bp.l = c->r.l;
        bp.ncolw = ncolw;
        bp.tile0 = t0;
        bp.ntiles = ncolw * ((c->r.m + c->r.rows - 1) / c->r.rows);
        bp.ncolw2 = (c->r.n + strip_cols(2) - 1) / strip_cols(2);
        bp.tile0_2 = t02;
        bp.ntiles2 = bp.ncolw2 * ((c->r.m + c->r.rows - 1) / c->r.rows);
        bp.mcolw = ncolw;
        bp.mtile0 = m0;
        bp.mtiles = L.mtiles[p];
        bp.mu = c->r.mu;
        bp.nu = c->r.nu;
        bp.tau = c->r.tau;
        bp.R0 = c->r.tau * c->fnorm2;
        for (int q = 0; q < bp.ntiles; ++q) tp.push_back(p);
        if (h->T == 2)
            for (int q = 0; q < bp.ntiles2; ++q) tp2.push_back(p);
        for (int q = 0; q < L.mtiles[p]; ++q) mtp.push_back(p);
        t0 += bp.ntiles;
        t02 += h->T == 2 ? bp.ntiles2 : 0;
        m0 += L.mtiles[p];
    }
    h->total_tiles = h->full_tiles = t0;
    h->total_tiles2 = t02;
    h->st.resize(B);
    hipError_t e = hipMemcpyAsync(h->d_tile_pair, tp.data(), sizeof(int) * tp.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && !tp2.empty())
        e = hipMemcpyAsync(h->d_tile_pair2, tp2.data(), sizeof(int) * tp2.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->d_mtile_pair, mtp.data(), sizeof(int) * mtp.size(), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&h->host_stopped), sizeof(unsigned), 0);
    int bpc = 0, cus = 0, dev = 0;
    if (e == hipSuccess) e = batch_blocks_per_cu(dtype, comp, &bpc);
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) {
        destroy_batch(h);
        return fail(OMT_EDEVICE, "batch set-up: %s", hipGetErrorString(e));
    }
    if (bpc < 1) {
        destroy_batch(h);
        return fail(OMT_EDEVICE, "batched kernel does not fit on a compute unit");
    }
    h->resident = bpc * cus;
    h->cus = cus;
    h->tuned = cached;  // rows from the tuning cache are kept like tuned ones
    batch_size_grid(h);
    *out = h;
    return OMT_OK;
}

omt_status omt_batch_solve(omt_batch_handle h, int64_t max_iters, double tol, int32_t check_every, omt_info *infos)
{
    TraceRange range("omt_batch_solve");
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    if (max_iters < 0) return fail(OMT_EINVAL, "max_iters < 0");
    const int K = check_every > 0 ? check_every : 64;
    if (max_iters == 0) {
        for (int p = 0; p < h->B && infos; ++p) std::memset(&infos[p], 0, sizeof(omt_info));
        return OMT_OK;
    }
    // rows for the whole batch (a previous solve may have left the rows of
    // its last problems), then the step arguments for every (parity, w
    // buffer, check) combination from each problem's current buffers
    const int full_before = h->full_tiles;
    const bool persistent = std::getenv("OMT_BATCH_PERSISTENT") != nullptr;
    if (!persistent) batch_retile(h, std::vector<char>(h->B, 1));
    for (int p = 0; p < h->B; ++p) batch_fill_args(h, p);
    int full = 0;
    for (int p = 0; p < h->B; ++p) full += h->pairs[p].ntiles;
    h->full_tiles = full;
    batch_size_grid(h);
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (h->total_tiles != h->full_tiles || h->total_mtiles != h->full_mtiles || full != full_before) {
        // a previous solve dropped stopped problems, or rows changed: every
        // problem runs again
        HIP_TRY(batch_set_lists(h, std::vector<char>(h->B, 1)));
        batch_drop_graphs(h);
    }
    HIP_TRY(hipMemcpyAsync(h->d_pairs, h->pairs.data(), sizeof(BatchPair) * h->B, hipMemcpyHostToDevice, h->cap));
    BatchArgs ba;
    ba.pairs = h->d_pairs;
    ba.state = h->d_state;
    ba.tile_pair = h->d_tile_pair;
    ba.tile_pair2 = h->d_tile_pair2;
    ba.mtile_pair = h->d_mtile_pair;
    ba.partials = h->d_partials;
    ba.bar = h->d_bar;
    ba.B = h->B;
    ba.total_tiles = h->total_tiles;
    ba.total_tiles2 = h->total_tiles2;
    ba.total_mtiles = h->total_mtiles;
    ba.check_every = K;
    ba.max_iters = max_iters;
    ba.tol = tol;
    if (persistent) {
        omt_status ps = batch_solve_persistent(h, ba);
        if (ps != OMT_OK) return ps;
    } else {
        omt_status gs = batch_solve_graphs(h, ba, max_iters, K);
        if (gs != OMT_OK) return gs;
    }
    unsigned bar[4];
    HIP_TRY(hipMemcpy(bar, h->d_bar, sizeof(bar), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(h->st.data(), h->d_state, sizeof(BatchPairState) * h->B, hipMemcpyDeviceToHost));
    if (bar[2] != 0u) return fail(OMT_EDEVICE, "batched solve: a grid barrier timed out (workgroups not co-resident)");
    bool all = true, bad = false;
    for (int p = 0; p < h->B; ++p) {
        omt_ctx *c = h->ctx[p];
        const BatchPairState &st = h->st[p];
        omt_info inf;
        std::memset(&inf, 0, sizeof(inf));
        fill_info(c, st.met, &inf);
        inf.iters = st.iters;
        inf.checks = st.checks;
        inf.converged = st.converged;
        c->cur = (c->cur + (st.cur == 1 ? 1 : 0) + 0) & 1;
        c->wcur = (c->wcur + (st.wcur == 1 ? 1 : 0)) & 1;
        c->iters_done += st.iters;
        c->last = inf;
        c->have_last = true;
        if (infos) infos[p] = inf;
        if (!inf.converged) all = false;
        if (!std::isfinite(inf.R)) bad = true;
    }
    if (bad) return fail(OMT_EDIVERGED, "a problem of the batch has a non-finite residual");
    if (tol > 0.0 && !all) return fail(OMT_ENOTCONV, "some problems did not reach tol %.3g", tol);
    return OMT_OK;
}

omt_status omt_batch_distance(omt_batch_handle h, double *V)
{
    if (!h || !V) return fail(OMT_EINVAL, "handle or V is NULL");
    for (int p = 0; p < h->B; ++p) {
        omt_status s = omt_distance(h->ctx[p], &V[p], nullptr);
        if (s != OMT_OK) return s;
    }
    return OMT_OK;
}

omt_status omt_batch_grad(omt_batch_handle h, void *const *d0, void *const *d1)
{
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    for (int p = 0; p < h->B; ++p) {
        omt_status s = omt_grad(h->ctx[p], d0 ? d0[p] : nullptr, d1 ? d1[p] : nullptr);
        if (s != OMT_OK) return s;
    }
    return OMT_OK;
}

omt_status omt_batch_get_state(omt_batch_handle h, int32_t b, void *phi, void *u, void *w)
{
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    if (b < 0 || b >= h->B) return fail(OMT_EINVAL, "problem index %d out of range", b);
    return omt_get_state(h->ctx[b], phi, u, w);
}

omt_status omt_batch_set_state(omt_batch_handle h, int32_t b, const void *phi, const void *u, const void *w)
{
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    if (b < 0 || b >= h->B) return fail(OMT_EINVAL, "problem index %d out of range", b);
    // the next omt_batch_solve builds its step arguments from the problem's
    // current buffers, which this fills
    return omt_set_state(h->ctx[b], phi, u, w);
}

omt_status omt_batch_autotune(omt_batch_handle h, int32_t launches_per_trial, int32_t *rows, double *us_per_iter)
{
    TraceRange range("omt_batch_autotune");
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    if (launches_per_trial < 0) return fail(OMT_EINVAL, "launches_per_trial < 0");
    if (launches_per_trial == 0) {
        // report the rows in use, tune nothing
        for (int p = 0; p < h->B && rows; ++p) rows[p] = h->ctx[p]->r.rows;
        if (us_per_iter) *us_per_iter = 0.0;
        return OMT_OK;
    }
    const int n = std::max(4, int(launches_per_trial));
    // problems of one shape class (grid, compiled type) share their rows;
    // problems whose rows the caller fixed keep them
    std::vector<std::vector<int>> classes;
    {
        std::vector<std::string> keys;
        for (int p = 0; p < h->B; ++p) {
            const omt_ctx *c = h->ctx[p];
            if (c->user_rows > 0) continue;
            char key[64];
            std::snprintf(key, sizeof(key), "%d %d %d", c->r.m, c->r.n, h->pairs[p].type);
            const auto it = std::find(keys.begin(), keys.end(), std::string(key));
            if (it == keys.end()) {
                keys.emplace_back(key);
                classes.push_back({p});
            } else {
                classes[size_t(it - keys.begin())].push_back(p);
            }
        }
    }
    BatchArgs ba;
    ba.pairs = h->d_pairs;
    ba.state = h->d_state;
    ba.tile_pair = h->d_tile_pair;
    ba.tile_pair2 = h->d_tile_pair2;
    ba.mtile_pair = h->d_mtile_pair;
    ba.partials = h->d_partials;
    ba.bar = h->d_bar;
    ba.B = h->B;
    ba.total_mtiles = h->total_mtiles;
    ba.check_every = 64;
    ba.max_iters = 1;
    ba.tol = 0.0;
    // the timed launches are the ones the batch's solves run (two
    // iterations per launch when the batch does): variant 1 of the step
    // arguments, or variant 8 for two iterations (read the current phi, u,
    // w; write all three to the other buffers), so the current iterates are
    // never changed
    const int tv = h->T == 2 ? 8 : 1;
    auto set_rows = [&](int p, int R) {
        omt_ctx *c = h->ctx[p];
        BatchPair &bp = h->pairs[p];
        c->r.rows = R;
        bp.ntiles = bp.ncolw * ((c->r.m + R - 1) / R);
        bp.ntiles2 = bp.ncolw2 * ((c->r.m + R - 1) / R);
        const int nroww = (c->r.m + R - 1) / R, ci = c->cur, wi = c->wcur;
        const int ncw = tv == 8 ? bp.ncolw2 : bp.ncolw;
        if (h->dtype == OMT_F64)
            fill_args(bp.args_mut<double>(tv), c, ci, 1 - ci, wi, 1 - wi, R, ncw, nroww, 0);
        else
            fill_args(bp.args_mut<float>(tv), c, ci, 1 - ci, wi, 1 - wi, R, ncw, nroww, 0);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto timed = [&](const std::vector<char> &active, double *us) -> hipError_t {
        hipError_t e = batch_set_lists(h, active);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->d_pairs, h->pairs.data(), sizeof(BatchPair) * h->B, hipMemcpyHostToDevice, h->cap);
        ba.total_tiles = h->total_tiles;
        ba.total_tiles2 = h->total_tiles2;
        if (e == hipSuccess) e = launch_batch_step(ba, h->dtype, h->comp, tv, h->cap, h->T);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, h->cap);
        for (int q = 0; q < n && e == hipSuccess; ++q) e = launch_batch_step(ba, h->dtype, h->comp, tv, h->cap, h->T);
        if (e == hipSuccess) e = hipEventRecord(e1, h->cap);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        *us = 1000.0 * double(ms) / (double(n) * h->T);  // per iteration
        return e;
    };
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    // every problem counts as unfinished while it is timed
    if (e == hipSuccess) e = launch_zero(h->d_state, sizeof(BatchPairState) * h->B, h->cap);
    const int cand[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
    for (size_t q = 0; q < classes.size() && e == hipSuccess; ++q) {
        const std::vector<int> &cls = classes[q];
        const int m = h->ctx[cls[0]]->r.m;
        std::vector<char> active(h->B, 0);
        for (int p : cls) active[p] = 1;
        int bestR = h->ctx[cls[0]]->r.rows;
        double best = 1e300;
        for (int R : cand) {
            if (R > m && R != 1) continue;
            for (int p : cls) set_rows(p, R);
            double us = 0.0;
            if ((e = timed(active, &us)) != hipSuccess) break;
            if (us < best) {
                best = us;
                bestR = R;
            }
        }
        for (int p : cls) set_rows(p, bestR);
        tune_cache_store_key("batch " + tune_key(h->ctx[cls[0]]), 1, bestR, best);
    }
    // every problem in the lists again, with its tuned rows
    double all_us = 0.0;
    if (e == hipSuccess) e = timed(std::vector<char>(h->B, 1), &all_us);
    if (e == hipSuccess) e = hipStreamSynchronize(h->cap);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(OMT_EDEVICE, "batch autotune: %s", hipGetErrorString(e));
    h->full_tiles = h->total_tiles;
    h->tuned = true;
    batch_size_grid(h);
    batch_drop_graphs(h);
    for (int p = 0; p < h->B; ++p) {
        h->ctx[p]->have_last = false;
        if (rows) rows[p] = h->ctx[p]->r.rows;
    }
    if (us_per_iter) *us_per_iter = all_us;
    return OMT_OK;
}

omt_status omt_batch_destroy(omt_batch_handle h)
{
    if (h) destroy_batch(h);
    return OMT_OK;
}

const char *omt_strerror(omt_status s)
{
    switch (s) {
        case OMT_OK: return "ok";
        case OMT_EINVAL: return "invalid argument";
        case OMT_EGRAPH: return "invalid channel graph";
        case OMT_EMASS: return "densities carry different mass";
        case OMT_ESTEP: return "step sizes violate the convergence condition";
        case OMT_ENOMEM: return "workspace too small";
        case OMT_EDEVICE: return "HIP error";
        case OMT_ENOTCONV: return "tolerance not reached";
        case OMT_EDIVERGED: return "iteration diverged";
        case OMT_EUNSUPPORTED: return "not compiled into this library";
        default: return "unknown status";
    }
}

const char *omt_last_error(void) { return g_last_error; }

int32_t omt_version(void) { return 1; }

}  // extern "C"

// ================================================================== matrix OMT

struct omt_mctx {
    omt_ctx *c;          // the problem in coordinates
    int k, K, Ks, l;     // matrix order, coordinates of Phi and of one W_s, matrices L_s
    bool real;
    int dtype;
    int64_t npix;
    hipStream_t stream;
    char *stage;         // npix * max(2K, l Ks) values: packed data, unpacked outputs
};

namespace {

using cplx = std::complex<double>;

// Orthonormal basis (Hilbert-Schmidt inner product) of the Hermitian (herm)
// or skew-Hermitian k x k matrices, in the coordinate order of the kernels:
// diagonal first (skew: i E_aa, complex only), then for a < b the real pair
// (E_ab +- E_ba)/sqrt2 and, complex only, the imaginary one i(E_ab -+ E_ba)/sqrt2.
std::vector<std::vector<cplx>> matrix_basis(int k, bool real, bool herm)
{
    std::vector<std::vector<cplx>> B;
    const double r = std::sqrt(0.5);
    if (herm || !real)
        for (int a = 0; a < k; ++a) {
            std::vector<cplx> E(k * k, 0.0);
            E[a * k + a] = herm ? cplx(1.0, 0.0) : cplx(0.0, 1.0);
            B.push_back(E);
        }
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b) {
            std::vector<cplx> E(k * k, 0.0);
            E[a * k + b] = r;
            E[b * k + a] = herm ? r : -r;
            B.push_back(E);
            if (!real) {
                std::vector<cplx> F(k * k, 0.0);
                F[a * k + b] = cplx(0.0, r);
                F[b * k + a] = herm ? cplx(0.0, -r) : cplx(0.0, r);
                B.push_back(F);
            }
        }
    return B;
}

double hs_dot(const std::vector<cplx> &X, const std::vector<cplx> &Y)
{
    double s = 0.0;
    for (size_t q = 0; q < X.size(); ++q) s += (X[q] * std::conj(Y[q])).real();
    return s;
}

struct MatrixSpec {
    int k, K, Ks, l;
    bool real;
};

omt_status resolve_matrix(const omt_matrix_params *p, Resolved &r, MatrixSpec &ms)
{
    if (!p) return fail(OMT_EINVAL, "params is NULL");
    if (p->m < 2 || p->n < 2) return fail(OMT_EINVAL, "grid must be at least 2 x 2 (got %d x %d)", p->m, p->n);
    if ((int64_t)p->m * p->n > (int64_t)1 << 31) return fail(OMT_EINVAL, "grid too large");
    if (p->k < 2) return fail(OMT_EINVAL, "matrix order k must be >= 2 (got %d)", p->k);
    if (p->n_L < 1 || !p->L) return fail(OMT_EINVAL, "need at least one matrix L_s");
    if (p->real != 0 && p->real != 1) return fail(OMT_EINVAL, "real must be 0 or 1");
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) return fail(OMT_EINVAL, "alpha must be > 0");
    if (!(p->tau > 0.0) || !std::isfinite(p->tau)) return fail(OMT_EINVAL, "tau must be > 0");
    if (p->mu < 0.0 || p->nu < 0.0 || p->h < 0.0 || !std::isfinite(p->mu) || !std::isfinite(p->nu) ||
        !std::isfinite(p->h))
        return fail(OMT_EINVAL, "mu, nu, h must be finite and >= 0");
    if (p->unorm < 0 || p->unorm > 2 || p->wnorm < 0 || p->wnorm > 2) return fail(OMT_EINVAL, "unknown norm");

    if (p->dtype != OMT_F32 && p->dtype != OMT_F64) return fail(OMT_EINVAL, "unknown dtype %d", p->dtype);
    if (p->rows_per_wave < 0) return fail(OMT_EINVAL, "rows_per_wave must be >= 0");
    if (p->tblock < 0 || p->tblock > 2) return fail(OMT_EINVAL, "tblock must be 0, 1 or 2 (got %d)", p->tblock);
    const int k = p->k, l = p->n_L;
    const bool real = p->real != 0;
    ms.k = k;
    ms.l = l;
    ms.real = real;
    ms.K = real ? k * (k + 1) / 2 : k * k;
    ms.Ks = real ? k * (k - 1) / 2 : k * k;
    const int lc = l * ms.Ks;
    if (ms.K > KMAX || matrix_bucket(ms.K, lc) == 0)
        return fail(OMT_EUNSUPPORTED, "%s k = %d with %d matrices L_s is not compiled", real ? "real" : "complex", k, l);
    if ((p->unorm == OMT_M_NUC || p->wnorm == OMT_M_NUC) && ms.K == 9)
        return fail(OMT_EUNSUPPORTED, "nuclear norms of complex 3 x 3 matrices are not compiled");
    // L: Hermitian (real symmetric in the real mode)
    std::vector<std::vector<cplx>> L(l, std::vector<cplx>(k * k));
    double big = 0.0;
    for (int s = 0; s < l; ++s)
        for (int q = 0; q < k * k; ++q) {
            L[s][q] = cplx(p->L[2 * (s * k * k + q)], p->L[2 * (s * k * k + q) + 1]);
            if (!std::isfinite(L[s][q].real()) || !std::isfinite(L[s][q].imag()))
                return fail(OMT_EINVAL, "L_%d has a non-finite entry", s);
            big = std::max(big, std::abs(L[s][q]));
        }
    if (!(big > 0.0)) return fail(OMT_EGRAPH, "every L_s is zero");
    for (int s = 0; s < l; ++s)
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) {
                if (std::abs(L[s][a * k + b] - std::conj(L[s][b * k + a])) > 1e-12 * big)
                    return fail(OMT_EINVAL, "L_%d is not Hermitian", s);
                if (real && L[s][a * k + b].imag() != 0.0)
                    return fail(OMT_EINVAL, "L_%d is not real (real mode)", s);
            }
    // the operator grad_L in coordinates: G[(s, q)][c] = <S_q, L_s H_c - H_c L_s>
    auto coord_op = [&](bool rl, int &nK, int &nKs) {
        const auto HB = matrix_basis(k, rl, true), SB = matrix_basis(k, rl, false);
        nK = int(HB.size());
        nKs = int(SB.size());
        std::vector<double> G(size_t(l) * nKs * nK, 0.0);
        for (int c = 0; c < nK; ++c)
            for (int s = 0; s < l; ++s) {
                std::vector<cplx> Z(k * k, 0.0);
                for (int a = 0; a < k; ++a)
                    for (int b = 0; b < k; ++b) {
                        cplx v = 0.0;
                        for (int q = 0; q < k; ++q)
                            v += L[s][a * k + q] * HB[c][q * k + b] - HB[c][a * k + q] * L[s][q * k + b];
                        Z[a * k + b] = v;
                    }
                for (int q = 0; q < nKs; ++q) G[size_t(s * nKs + q) * nK + c] = hs_dot(SB[q], Z);
            }
        return G;
    };
    int gK = 0, gKs = 0;
    const std::vector<double> G = coord_op(real, gK, gKs);
    // -Delta_L = G^T G on all Hermitian matrices (the k^2 x k^2 matrix of
    // Sec. 7.3, also in the real mode): its spectrum gives nu, and its kernel
    // must be the multiples of I (the standing assumption of Sec. 4.1)
    int fK = 0, fKs = 0;
    const std::vector<double> Gf = coord_op(false, fK, fKs);
    const int fl = l * fKs;
    std::vector<double> A(size_t(fK) * fK, 0.0);
    for (int a = 0; a < fK; ++a)
        for (int b = 0; b < fK; ++b) {
            double v = 0.0;
            for (int e = 0; e < fl; ++e) v += Gf[size_t(e) * fK + a] * Gf[size_t(e) * fK + b];
            A[a * fK + b] = v;
        }
    std::vector<double> ev(fK);
    jacobi_eigenvalues(A.data(), fK, ev.data());
    double lmax = 0.0;
    for (double v : ev) lmax = std::max(lmax, v);
    int nker = 0;
    for (double v : ev)
        if (v <= 1e-10 * lmax) ++nker;
    if (nker != 1)
        return fail(OMT_EGRAPH, "grad_L annihilates a %d-dimensional space; the method needs exactly the multiples of I",
                    nker);

    r = Resolved();
    r.m = p->m;
    r.n = p->n;
    r.k = ms.K;
    r.l = lc;
    r.gk = (p->unorm == OMT_M_NUC || p->wnorm == OMT_M_NUC) ? G_MATNUC : G_MATRIX;
    r.lb = matrix_bucket(ms.K, lc);
    r.alpha = p->alpha;
    r.tau = p->tau;
    r.eps = 0.0;
    // u norm 2 / 3 / 4 and w norm 1 / 2 / 3: Frobenius, grouped entry-wise, nuclear
    r.unorm = p->unorm == OMT_M_FRO ? 2 : p->unorm == OMT_M_L1 ? 3 : 4;
    r.wnorm = p->wnorm == OMT_M_FRO ? 1 : p->wnorm == OMT_M_L1 ? 2 : 3;
    r.dtype = p->dtype;
    r.comp = (p->flags & OMT_FLAG_COMPENSATED_PHI) && p->dtype == OMT_F32;
    r.tblock = p->tblock;
    r.rows = p->rows_per_wave;
    r.h = p->h > 0.0 ? p->h : 1.0 / double(std::max(r.m, r.n) - 1);
    r.lmax = lmax;
    const double h2 = r.h * r.h;
    r.mu = p->mu > 0.0 ? p->mu : h2 / (32.0 * r.tau);
    r.nu = p->nu > 0.0 ? p->nu : 1.0 / (4.0 * r.tau * lmax);
    if (p->mu > 0.0 || p->nu > 0.0) {
        const double cond = r.tau * r.mu * 8.0 / h2 + r.tau * r.nu * lmax;
        if (!(cond < 1.0))
            return fail(OMT_ESTEP, "tau mu 8/h^2 + tau nu lambda_max = %g must be < 1 (Sec. 7.3)", cond);
    }
    r.matrix = true;
    r.gmat.assign(KMAX * LMAX, 0.0);
    for (int c = 0; c < ms.K; ++c)
        for (int e = 0; e < lc; ++e) r.gmat[c * LMAX + e] = G[size_t(e) * ms.K + c];
    // grouped entry-wise norm: diagonal coordinates weigh 1; an off-diagonal
    // pair (X_ab, X_ba) weighs 2 |X_ab| = sqrt2 |coordinates|
    const int nd = k;
    r.uwt.assign(ms.K, 0.0);
    for (int c = 0; c < ms.K; ++c) r.uwt[c] = c < nd ? 1.0 : (real || (c - nd) % 2 == 0 ? std::sqrt(2.0) : 0.0);
    r.wwt.assign(lc, 0.0);
    const int snd = real ? 0 : k;
    for (int s = 0; s < l; ++s)
        for (int q = 0; q < ms.Ks; ++q)
            r.wwt[s * ms.Ks + q] = q < snd ? 1.0 : (real || (q - snd) % 2 == 0 ? std::sqrt(2.0) : 0.0);
    // mass: only the trace is conserved; the diagonal coordinates form the
    // one class whose mean is removed
    for (int c = 0; c < ms.K; ++c) r.cls[c] = -1;
    for (int c = 0; c < nd; ++c) r.cls[c] = 0;
    r.ncls = 1;
    if (!fields_fit(r))
        return fail(OMT_EUNSUPPORTED, "a field of %d x %d x %d %s coordinates exceeds 2 GiB", r.m, r.n,
                    std::max(2 * r.k, r.lb), r.dtype == OMT_F64 ? "FP64" : "FP32");
    if (r.tblock > 1 && !step_supported(r.dtype, r.k, r.gk, r.lb, r.tblock, r.comp))
        return fail(OMT_EUNSUPPORTED, "no %d-iteration step for %s %d coordinates with these norms", r.tblock,
                    r.dtype == OMT_F64 ? "FP64" : "FP32", r.k);
    return OMT_OK;
}

size_t matrix_stage_bytes(const Resolved &r, const MatrixSpec &ms)
{
    const size_t per = size_t(std::max(2 * ms.K, ms.l * ms.Ks));
    return align256(size_t(r.m) * r.n * per * (r.dtype == OMT_F64 ? 8 : 4));
}

hipError_t matrix_xfer(const omt_mctx *h, const void *src, void *dst, bool herm, bool pack, int count, int cstride,
                       int coff)
{
    MatrixXferArgs a;
    a.src = src;
    a.dst = dst;
    a.dtype = h->dtype;
    a.npix = h->npix;
    a.k = h->k;
    a.real = h->real ? 1 : 0;
    a.herm = herm ? 1 : 0;
    a.pack = pack ? 1 : 0;
    a.count = count;
    a.cstride = cstride;
    a.coff = coff;
    return launch_matrix_xfer(a, h->stream);
}

}  // namespace

extern "C" {

omt_status omt_matrix_params_init(omt_matrix_params *p)
{
    if (!p) return fail(OMT_EINVAL, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->alpha = 1.0;
    p->tau = 1.0;
    p->unorm = OMT_M_FRO;
    p->wnorm = OMT_M_L1;
    p->dtype = OMT_F32;
    return OMT_OK;
}

omt_status omt_matrix_resolve(const omt_matrix_params *p, double *h, double *mu, double *nu, double *lambda_max,
                              int32_t *coords, int32_t *w_coords)
{
    Resolved r;
    MatrixSpec ms;
    omt_status s = resolve_matrix(p, r, ms);
    if (s != OMT_OK) return s;
    if (h) *h = r.h;
    if (mu) *mu = r.mu;
    if (nu) *nu = r.nu;
    if (lambda_max) *lambda_max = r.lmax;
    if (coords) *coords = ms.K;
    if (w_coords) *w_coords = ms.l * ms.Ks;
    return OMT_OK;
}

omt_status omt_matrix_workspace_bytes(const omt_matrix_params *p, size_t *bytes)
{
    if (!bytes) return fail(OMT_EINVAL, "bytes is NULL");
    Resolved r;
    MatrixSpec ms;
    omt_status s = resolve_matrix(p, r, ms);
    if (s != OMT_OK) return s;
    *bytes = align256(make_layout(r).total) + matrix_stage_bytes(r, ms);
    return OMT_OK;
}

omt_status omt_matrix_create(const omt_matrix_params *p, const void *Lambda0, const void *Lambda1, void *workspace,
                             size_t ws_bytes, void *stream, omt_matrix_handle *out)
{
    if (!out) return fail(OMT_EINVAL, "out is NULL");
    *out = nullptr;
    Resolved r;
    MatrixSpec ms;
    omt_status s = resolve_matrix(p, r, ms);
    if (s != OMT_OK) return s;
    if (!Lambda0 || !Lambda1) return fail(OMT_EINVAL, "Lambda0 / Lambda1 is NULL");
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(OMT_EINVAL, "workspace missing or not 256-byte aligned");
    const size_t core = align256(make_layout(r).total), need = core + matrix_stage_bytes(r, ms);
    if (ws_bytes < need) return fail(OMT_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, need);
    omt_mctx *h = new omt_mctx();
    h->c = nullptr;
    h->k = ms.k;
    h->K = ms.K;
    h->Ks = ms.Ks;
    h->l = ms.l;
    h->real = ms.real;
    h->dtype = r.dtype;
    h->npix = int64_t(r.m) * r.n;
    h->stream = static_cast<hipStream_t>(stream);
    h->stage = static_cast<char *>(workspace) + core;
    // pack both densities into coordinates (two halves of the staging area),
    // then set up the coordinate problem from them
    const size_t half = size_t(h->npix) * ms.K * (r.dtype == OMT_F64 ? 8 : 4);
    hipError_t e = matrix_xfer(h, Lambda0, h->stage, true, true, 1, 1, 0);
    if (e == hipSuccess) e = matrix_xfer(h, Lambda1, h->stage + half, true, true, 1, 1, 0);
    if (e != hipSuccess) {
        delete h;
        return fail(OMT_EDEVICE, "packing: %s", hipGetErrorString(e));
    }
    s = create_resolved(r, h->stage, h->stage + half, workspace, core, stream, &h->c);
    if (s != OMT_OK) {
        delete h;
        return s;
    }
    *out = h;
    return OMT_OK;
}

omt_status omt_matrix_solve(omt_matrix_handle h, int64_t max_iters, double tol, int32_t check_every, omt_info *info)
{
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    return omt_solve(h->c, max_iters, tol, check_every, info);
}

omt_status omt_matrix_distance(omt_matrix_handle h, double *M, omt_info *info)
{
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    return omt_distance(h->c, M, info);
}

omt_status omt_matrix_grad(omt_matrix_handle h, void *d0, void *d1)
{
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    const size_t half = size_t(h->npix) * h->K * (h->dtype == OMT_F64 ? 8 : 4);
    omt_status s = omt_grad(h->c, d0 ? h->stage : nullptr, d1 ? h->stage + half : nullptr);
    if (s != OMT_OK) return s;
    if (d0) HIP_TRY(matrix_xfer(h, h->stage, d0, true, false, 1, 1, 0));
    if (d1) HIP_TRY(matrix_xfer(h, h->stage + half, d1, true, false, 1, 1, 0));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return OMT_OK;
}

omt_status omt_matrix_get_state(omt_matrix_handle h, void *Phi, void *Ux, void *Uy, void *W)
{
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    if (Phi) {
        omt_status s = omt_get_state(h->c, h->stage, nullptr, nullptr);
        if (s != OMT_OK) return s;
        HIP_TRY(matrix_xfer(h, h->stage, Phi, true, false, 1, 1, 0));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    if (Ux || Uy) {
        // u arrives as m x n x K x 2 (x and y interleaved)
        omt_status s = omt_get_state(h->c, nullptr, h->stage, nullptr);
        if (s != OMT_OK) return s;
        if (Ux) HIP_TRY(matrix_xfer(h, h->stage, Ux, true, false, 1, 2, 0));
        if (Uy) HIP_TRY(matrix_xfer(h, h->stage, Uy, true, false, 1, 2, 1));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    if (W) {
        omt_status s = omt_get_state(h->c, nullptr, nullptr, h->stage);
        if (s != OMT_OK) return s;
        HIP_TRY(matrix_xfer(h, h->stage, W, false, false, h->l, 1, 0));
        HIP_TRY(hipStreamSynchronize(h->stream));
    }
    return OMT_OK;
}

omt_status omt_matrix_time_steps(omt_matrix_handle h, int32_t rows_per_wave, int64_t n, double *us_per_launch)
{
    if (!h) return fail(OMT_EINVAL, "handle is NULL");
    return omt_time_steps(h->c, tblock_of(h->c), rows_per_wave, n, us_per_launch);
}

omt_status omt_matrix_destroy(omt_matrix_handle h)
{
    if (h) {
        if (h->c) omt_destroy(h->c);
        delete h;
    }
    return OMT_OK;
}

}  // extern "C"
