// Fused PDHG iteration of the vector-OMT method (Sec. 7.2) for gfx950.
//
// One wavefront owns a strip of columns (lanes are columns, so every load
// and store is a coalesced row segment) and a chunk of rows, and streams down
// the rows.  Each lane keeps its own column's state in registers; the
// neighbours a step needs come from the adjacent lane (right potential for
// grad_y, left flux for div_y) or from the previous row held in registers
// (flux for div_x).
//
// One iteration per launch (T = 1): the strip is 64 aligned columns.  The two
// values from outside it -- the potential one column to the right and the
// extrapolated flux u_y one column to the left -- are rebuilt from loads in
// which lane c carries channel c, and the left flux is recomputed with the
// same u-update code as every other pixel.
//
// T > 1 iterations per launch: stage t works on iteration t+1, one row
// behind stage t-1, so one pass over HBM advances the strip by T iterations.
// The strip is 64 - 2T columns plus T recomputed halo lanes on each side, and
// T halo rows above and T-1 below; only the interior is stored.
//
// Per pixel and iteration (App. A discretisation, ghosts u_x(m-1,.) = 0 and
// u_y(., n-1) = 0, Sec. 7.2 updates):
//   u~  = u + mu grad_x phi                    -> shrink_u(., mu)
//   w~  = w + nu grad_G phi                    -> shrink_w(., alpha nu)
//   phi' = phi + tau (div_x(2u'-u) + div_G(2w'-w) + f),   f = rho1 - rho0.
//
// Compiled once per channel count (OMT_K) to keep build units small.

#include "metrics_device.h"

#ifndef OMT_K
#error "compile with -DOMT_K=<channels>"
#endif

namespace omt {
namespace {

using namespace dev;

// CHK: the launch also takes the check of its last iteration (Sec. 6.1),
// writing quad sums of the check terms to a.qpart.
template <typename R, int K, int GK, int L, int T, bool COMP, bool CHK>
__global__ __launch_bounds__(WAVE *STEP_WAVES_PER_WG) void pdhg_step_kernel(const StepArgs<R> a)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int g = xcd_remap(blockIdx.x, a.nwg);
    const int wc = g % a.ncolw;
    const int wr = (g / a.ncolw) * STEP_WAVES_PER_WG + (threadIdx.x / WAVE);
    if (wr >= a.nroww) return;  // whole wave leaves; no barriers follow
    process_strip<R, K, GK, L, T, COMP, CHK>(a, wc, wr, lane);
}

template <typename R, int K, int GK, int L, bool COMP>
__global__ __launch_bounds__(WAVE *STEP_WAVES_PER_WG) void tile_metrics_kernel(const StepArgs<R> a, int ncolw,
                                                                                int ntiles, double *partials)
{
    const int lane = threadIdx.x & (WAVE - 1);
    // the tile index made provably wave-uniform, so the row bounds derived
    // from it branch on the scalar unit
    const int t = blockIdx.x * STEP_WAVES_PER_WG + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    if (t >= ntiles) return;
    double v[NMET];
    tile_metrics<R, K, GK, L, COMP>(a, t % ncolw, t / ncolw, lane, v);
#pragma unroll
    for (int q = 0; q < NMET; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) partials[(int64_t)t * NMET + q] = s;
    }
}

template <typename R, int GK, int L, int T, bool COMP>
hipError_t launch_one(const StepLaunch &Lc)
{
    const StepArgs<R> &a = *static_cast<const StepArgs<R> *>(Lc.args);
    // the check is compiled into single-iteration launches of the vector method
    if constexpr (check_compiled(GK) && T == 1) {
        if (Lc.check) {
            hipLaunchKernelGGL((pdhg_step_kernel<R, OMT_K, GK, L, T, COMP, true>), dim3(a.nwg),
                               dim3(WAVE * STEP_WAVES_PER_WG), 0, Lc.stream, a);
            return hipGetLastError();
        }
    } else {
        if (Lc.check) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((pdhg_step_kernel<R, OMT_K, GK, L, T, COMP, false>), dim3(a.nwg), dim3(WAVE * STEP_WAVES_PER_WG),
                       0, Lc.stream, a);
    return hipGetLastError();
}

template <typename R, int GK, int L, int T, bool COMP>
hipError_t occ_one(int *blocks)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, pdhg_step_kernel<R, OMT_K, GK, L, T, COMP, false>,
                                                         WAVE * STEP_WAVES_PER_WG, 0);
}

// the matrix kind with Frobenius or entry-wise norms also runs two
// iterations per pass in FP32 (not the 9-coordinate complex 3 x 3 kind)
constexpr bool MAT_T2 = OMT_K <= 6;

// FP64 also runs two iterations per launch for up to three channels on the
// vector kinds (154 VGPRs at k = 3, the occupancy of one iteration per launch)
constexpr bool F64_T2 = OMT_K <= 3;

template <int GK, int L>
hipError_t occ_T(const StepLaunch &Lc, int *blocks)
{
    if (Lc.dtype == 1) {
        if constexpr (F64_T2 && GK != G_DENSE && !is_matrix_kind(GK)) {
            if (Lc.T == 2) return occ_one<double, GK, L, 2, false>(blocks);
        }
        return occ_one<double, GK, L, 1, false>(blocks);
    }
    if (Lc.T == 1) return Lc.comp ? occ_one<float, GK, L, 1, true>(blocks) : occ_one<float, GK, L, 1, false>(blocks);
    if constexpr (GK == G_MATRIX && MAT_T2) {
        if (Lc.T == 2) return Lc.comp ? occ_one<float, GK, L, 2, true>(blocks) : occ_one<float, GK, L, 2, false>(blocks);
    }
    if constexpr (GK != G_DENSE && !is_matrix_kind(GK)) {
        switch (Lc.T) {
            case 2: return Lc.comp ? occ_one<float, GK, L, 2, true>(blocks) : occ_one<float, GK, L, 2, false>(blocks);
#if OMT_K <= 5
            case 4: return Lc.comp ? occ_one<float, GK, L, 4, true>(blocks) : occ_one<float, GK, L, 4, false>(blocks);
#endif
#if OMT_K <= 3
            case 8: return Lc.comp ? occ_one<float, GK, L, 8, true>(blocks) : occ_one<float, GK, L, 8, false>(blocks);
#endif
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

template <typename R, int GK, int L, bool COMP>
hipError_t launch_met(const StepLaunch &Lc, int ncolw, int ntiles, double *partials)
{
    const StepArgs<R> &a = *static_cast<const StepArgs<R> *>(Lc.args);
    const int nb = (ntiles + STEP_WAVES_PER_WG - 1) / STEP_WAVES_PER_WG;
    hipLaunchKernelGGL((tile_metrics_kernel<R, OMT_K, GK, L, COMP>), dim3(nb), dim3(WAVE * STEP_WAVES_PER_WG), 0,
                       Lc.stream, a, ncolw, ntiles, partials);
    return hipGetLastError();
}

template <int GK, int L>
hipError_t dispatch_met(const StepLaunch &Lc, int ncolw, int ntiles, double *partials)
{
    if (Lc.dtype == 1) return launch_met<double, GK, L, false>(Lc, ncolw, ntiles, partials);
    return Lc.comp ? launch_met<float, GK, L, true>(Lc, ncolw, ntiles, partials)
                   : launch_met<float, GK, L, false>(Lc, ncolw, ntiles, partials);
}

// Blocking depths compiled for this channel count (register budget); dense
// graphs run one iteration per launch, FP64 one or two (F64_T2).
constexpr bool t_ok(int T) { return T == 1 || T == 2 || (T == 4 && OMT_K <= 5) || (T == 8 && OMT_K <= 3); }

template <int GK, int L>
hipError_t dispatch_T(const StepLaunch &Lc)
{
    if (Lc.dtype == 1) {
        if (Lc.T == 1 && !Lc.comp) return launch_one<double, GK, L, 1, false>(Lc);
        if constexpr (F64_T2 && GK != G_DENSE && !is_matrix_kind(GK)) {
            if (Lc.T == 2 && !Lc.comp) return launch_one<double, GK, L, 2, false>(Lc);
        }
        return hipErrorInvalidValue;
    }
    if (Lc.T == 1) return Lc.comp ? launch_one<float, GK, L, 1, true>(Lc) : launch_one<float, GK, L, 1, false>(Lc);
    if constexpr (GK == G_MATRIX && MAT_T2) {
        if (Lc.T == 2) return Lc.comp ? launch_one<float, GK, L, 2, true>(Lc) : launch_one<float, GK, L, 2, false>(Lc);
    }
    if constexpr (GK != G_DENSE && !is_matrix_kind(GK)) {
        switch (Lc.T) {
            case 2: return Lc.comp ? launch_one<float, GK, L, 2, true>(Lc) : launch_one<float, GK, L, 2, false>(Lc);
#if OMT_K <= 5
            case 4: return Lc.comp ? launch_one<float, GK, L, 4, true>(Lc) : launch_one<float, GK, L, 4, false>(Lc);
#endif
#if OMT_K <= 3
            case 8: return Lc.comp ? launch_one<float, GK, L, 8, true>(Lc) : launch_one<float, GK, L, 8, false>(Lc);
#endif
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

constexpr int L_TREE = OMT_K - 1;
constexpr int L_FULL = OMT_K * (OMT_K - 1) / 2;
// matrix problems compiled for this coordinate count (0: none)
constexpr int L_MAT = OMT_K == 3 ? 3 : OMT_K == 4 ? 8 : OMT_K == 6 ? 9 : OMT_K == 9 ? 18 : 0;
constexpr int L_MAT2 = OMT_K == 6 ? 6 : 0;  // a second bucket (two L_s for real 3 x 3)

}  // namespace

#define OMT_CAT2(a, b) a##b
#define OMT_CAT(a, b) OMT_CAT2(a, b)

hipError_t OMT_CAT(launch_step_k, OMT_K)(const StepLaunch &Lc)
{
#if OMT_K <= 8  // the vector method has at most 8 channels
    if (Lc.gk == G_NONE && Lc.lb == 0) return dispatch_T<G_NONE, 0>(Lc);
#if OMT_K >= 2
    if (Lc.gk == G_PATH && Lc.lb == L_TREE) return dispatch_T<G_PATH, L_TREE>(Lc);
#endif
#if OMT_K >= 3
    if (Lc.gk == G_COMPLETE && Lc.lb == L_FULL) return dispatch_T<G_COMPLETE, L_FULL>(Lc);
    if (Lc.gk == G_DENSE && Lc.lb == L_TREE) return dispatch_T<G_DENSE, L_TREE>(Lc);
    if (Lc.gk == G_DENSE && Lc.lb == L_FULL) return dispatch_T<G_DENSE, L_FULL>(Lc);
#endif
#endif
#if OMT_K == 3 || OMT_K == 4 || OMT_K == 6 || OMT_K == 9
    if (Lc.gk == G_MATRIX && Lc.lb == L_MAT) return dispatch_T<G_MATRIX, L_MAT>(Lc);
#endif
#if OMT_K == 3 || OMT_K == 4 || OMT_K == 6
    if (Lc.gk == G_MATNUC && Lc.lb == L_MAT) return dispatch_T<G_MATNUC, L_MAT>(Lc);
#endif
#if OMT_K == 6
    if (Lc.gk == G_MATRIX && Lc.lb == L_MAT2) return dispatch_T<G_MATRIX, L_MAT2>(Lc);
    if (Lc.gk == G_MATNUC && Lc.lb == L_MAT2) return dispatch_T<G_MATNUC, L_MAT2>(Lc);
#endif
    return hipErrorInvalidValue;
}

hipError_t OMT_CAT(launch_metrics_k, OMT_K)(const StepLaunch &Lc, int ncolw, int ntiles, double *partials)
{
#if OMT_K <= 8  // the vector method has at most 8 channels
    if (Lc.gk == G_NONE && Lc.lb == 0) return dispatch_met<G_NONE, 0>(Lc, ncolw, ntiles, partials);
#if OMT_K >= 2
    if (Lc.gk == G_PATH && Lc.lb == L_TREE) return dispatch_met<G_PATH, L_TREE>(Lc, ncolw, ntiles, partials);
#endif
#if OMT_K >= 3
    if (Lc.gk == G_COMPLETE && Lc.lb == L_FULL) return dispatch_met<G_COMPLETE, L_FULL>(Lc, ncolw, ntiles, partials);
    if (Lc.gk == G_DENSE && Lc.lb == L_TREE) return dispatch_met<G_DENSE, L_TREE>(Lc, ncolw, ntiles, partials);
    if (Lc.gk == G_DENSE && Lc.lb == L_FULL) return dispatch_met<G_DENSE, L_FULL>(Lc, ncolw, ntiles, partials);
#endif
#endif
#if OMT_K == 3 || OMT_K == 4 || OMT_K == 6 || OMT_K == 9
    if (Lc.gk == G_MATRIX && Lc.lb == L_MAT) return dispatch_met<G_MATRIX, L_MAT>(Lc, ncolw, ntiles, partials);
#endif
#if OMT_K == 3 || OMT_K == 4 || OMT_K == 6
    if (Lc.gk == G_MATNUC && Lc.lb == L_MAT) return dispatch_met<G_MATNUC, L_MAT>(Lc, ncolw, ntiles, partials);
#endif
#if OMT_K == 6
    if (Lc.gk == G_MATRIX && Lc.lb == L_MAT2) return dispatch_met<G_MATRIX, L_MAT2>(Lc, ncolw, ntiles, partials);
    if (Lc.gk == G_MATNUC && Lc.lb == L_MAT2) return dispatch_met<G_MATNUC, L_MAT2>(Lc, ncolw, ntiles, partials);
#endif
    return hipErrorInvalidValue;
}

hipError_t OMT_CAT(step_blocks_per_cu_k, OMT_K)(const StepLaunch &Lc, int *blocks)
{
#if OMT_K <= 8  // the vector method has at most 8 channels
    if (Lc.gk == G_NONE && Lc.lb == 0) return occ_T<G_NONE, 0>(Lc, blocks);
#if OMT_K >= 2
    if (Lc.gk == G_PATH && Lc.lb == L_TREE) return occ_T<G_PATH, L_TREE>(Lc, blocks);
#endif
#if OMT_K >= 3
    if (Lc.gk == G_COMPLETE && Lc.lb == L_FULL) return occ_T<G_COMPLETE, L_FULL>(Lc, blocks);
    if (Lc.gk == G_DENSE && Lc.lb == L_TREE) return occ_T<G_DENSE, L_TREE>(Lc, blocks);
    if (Lc.gk == G_DENSE && Lc.lb == L_FULL) return occ_T<G_DENSE, L_FULL>(Lc, blocks);
#endif
#endif
#if OMT_K == 3 || OMT_K == 4 || OMT_K == 6 || OMT_K == 9
    if (Lc.gk == G_MATRIX && Lc.lb == L_MAT) return occ_T<G_MATRIX, L_MAT>(Lc, blocks);
#endif
#if OMT_K == 3 || OMT_K == 4 || OMT_K == 6
    if (Lc.gk == G_MATNUC && Lc.lb == L_MAT) return occ_T<G_MATNUC, L_MAT>(Lc, blocks);
#endif
#if OMT_K == 6
    if (Lc.gk == G_MATRIX && Lc.lb == L_MAT2) return occ_T<G_MATRIX, L_MAT2>(Lc, blocks);
    if (Lc.gk == G_MATNUC && Lc.lb == L_MAT2) return occ_T<G_MATNUC, L_MAT2>(Lc, blocks);
#endif
    return hipErrorInvalidValue;
}

bool OMT_CAT(step_supported_k, OMT_K)(int dtype, int gk, int lb, int T, bool comp)
{
    bool ok = (OMT_K <= 8 && gk == G_NONE && lb == 0);
    ok = ok || (OMT_K >= 2 && OMT_K <= 8 && gk == G_PATH && lb == L_TREE);
    ok = ok || (OMT_K >= 3 && OMT_K <= 8 && gk == G_COMPLETE && lb == L_FULL);
    ok = ok || (OMT_K >= 3 && OMT_K <= 8 && gk == G_DENSE && (lb == L_TREE || lb == L_FULL));
    ok = ok || (L_MAT > 0 && gk == G_MATRIX && (lb == L_MAT || (L_MAT2 > 0 && lb == L_MAT2)));
    ok = ok || (L_MAT > 0 && OMT_K != 9 && gk == G_MATNUC && (lb == L_MAT || (L_MAT2 > 0 && lb == L_MAT2)));
    if (!ok) return false;
    if (dtype == 1) return !comp && (T == 1 || (F64_T2 && T == 2 && gk != G_DENSE && !is_matrix_kind(gk)));
    if (gk == G_MATRIX) return T == 1 || (MAT_T2 && T == 2);
    if (gk == G_DENSE || is_matrix_kind(gk)) return T == 1;
    return t_ok(T);
}

}  // namespace omt
