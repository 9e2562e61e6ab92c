// Batched PDHG solver: many independent problems (different grid sizes,
// channel counts and graphs) iterated together.  Two schedules share the
// per-strip and per-tile code: launches per iteration replayed as a graph
// (the default, at the end of this file) and one persistent launch (below).
//
// Persistent launch:
// The grid is sized to the number of workgroups the chip holds at once, so
// every workgroup is resident, and it stays for the whole solve.  Each
// iteration the waves walk the list of strips (64 columns x rows) of all
// unfinished problems, run the same per-strip code as the per-launch step
// kernel, and meet at a grid barrier.  At a check iteration they compute the
// metrics tiles, meet, let one wave per problem reduce its tiles and decide
// whether the problem has converged (it then drops out of the strip list),
// and meet again.  The barrier's wait is bounded: if it ever expires every
// wave sees the abort flag and leaves, and the host reports the error.
//
// Supported problem types (compiled in): k = 1 without edges, k = 2 with one
// edge, k = 3 on the complete graph (triangle) or on the path; FP32 (with or
// without the compensated potential) or FP64, one dtype per batch; one
// iteration per pass in the persistent launch, one or two in the launches
// per iteration.

#include "metrics_device.h"

namespace omt {
namespace {

using namespace dev;

constexpr unsigned SPIN_LIMIT = 1u << 25;  // ~ seconds of s_sleep before a barrier gives up

__device__ __forceinline__ unsigned ld_acq(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier over nblocks resident workgroups, in two levels so that
// no counter sees more than a few dozen arrivals: workgroups meet in 8
// groups (blockIdx mod 8, which is also how workgroups are dealt to the
// XCDs), the last of each group meets the others at the top.  Words of bar:
// [0] top arrivals, [1] generation, [2] abort flag, [3] problems stopped,
// [BAR_GROUP0 + BAR_STRIDE g] arrivals of group g (own cache line).
// Returns true if the barrier was abandoned (abort flag set).
__device__ bool grid_sync(unsigned *bar, unsigned nblocks)
{
    __shared__ int s_abort;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned G = nblocks < BAR_GROUPS ? nblocks : BAR_GROUPS;
        const unsigned g = blockIdx.x % G;
        const unsigned gsize = nblocks / G + (g < nblocks % G ? 1u : 0u);
        const unsigned gen = ld_acq(&bar[1]);
        unsigned *grp = &bar[BAR_GROUP0 + BAR_STRIDE * g];
        bool released = false;
        if (__hip_atomic_fetch_add(grp, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u == gsize) {
            __hip_atomic_store(grp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u == G) {
                __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&bar[1], gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                released = true;
            }
        }
        if (!released) {
            unsigned spins = 0;
            while (ld_acq(&bar[1]) == gen) {
                if (ld_acq(&bar[2]) != 0u) break;
                if (++spins > SPIN_LIMIT) {
                    __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        s_abort = int(ld_acq(&bar[2]));
    }
    __syncthreads();
    __threadfence();
    return s_abort != 0;
}

// The step arguments are copied out of the table once, before any store, so
// that the compiler need not reload them after every store it cannot prove
// disjoint from the table.
template <typename R, bool COMP, int T = 1>
__device__ __forceinline__ void strip_by_type(int type, const StepArgs<R> &src, int wc, int wr, int lane)
{
    const StepArgs<R> a = src;
    switch (type) {
        case 0: process_strip<R, 1, G_NONE, 0, T, COMP>(a, wc, wr, lane); break;
        case 1: process_strip<R, 2, G_PATH, 1, T, COMP>(a, wc, wr, lane); break;
        case 2: process_strip<R, 3, G_COMPLETE, 3, T, COMP>(a, wc, wr, lane); break;
        case 3: process_strip<R, 3, G_PATH, 2, T, COMP>(a, wc, wr, lane); break;
        default: break;
    }
}

template <typename R, bool COMP>
__device__ __forceinline__ void metrics_by_type(int type, const StepArgs<R> &src, int wc, int wr, int lane,
                                                double (&v)[NMET])
{
    const StepArgs<R> a = src;
    switch (type) {
        case 0: tile_metrics<R, 1, G_NONE, 0, COMP>(a, wc, wr, lane, v); break;
        case 1: tile_metrics<R, 2, G_PATH, 1, COMP>(a, wc, wr, lane, v); break;
        case 2: tile_metrics<R, 3, G_COMPLETE, 3, COMP>(a, wc, wr, lane, v); break;
        case 3: tile_metrics<R, 3, G_PATH, 2, COMP>(a, wc, wr, lane, v); break;
        default:
            for (int q = 0; q < NMET; ++q) v[q] = 0.0;
            break;
    }
}

template <typename R, bool COMP>
__global__ __launch_bounds__(WAVE *STEP_WAVES_PER_WG) void batch_kernel(const BatchArgs ba)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int nw = gridDim.x * STEP_WAVES_PER_WG;
    const int gw = blockIdx.x * STEP_WAVES_PER_WG + threadIdx.x / WAVE;
    const unsigned nblocks = gridDim.x;
    int nchecks = 0;
    for (int64_t it = 0; it < ba.max_iters; ++it) {
        const bool check = ((it + 1) % ba.check_every == 0) || (it + 1 == ba.max_iters);
        const int par = int(it & 1);
        const int wcur = nchecks & 1;
        const int var = par * 4 + wcur * 2 + (check ? 1 : 0);

        // one iteration of every unfinished problem
        for (int t = gw; t < ba.total_tiles; t += nw) {
            const int p = __builtin_amdgcn_readfirstlane(ba.tile_pair[t]);
            if (__hip_atomic_load(&ba.state[p].done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) continue;
            const BatchPair &bp = ba.pairs[p];
            const int local = t - bp.tile0;
            strip_by_type<R, COMP>(bp.type, bp.template args<R>(var), local % bp.ncolw, local / bp.ncolw, lane);
        }
        if (grid_sync(ba.bar, nblocks)) return;
        if (!check) continue;

        // metrics of the step just taken, tile by tile
        for (int t = gw; t < ba.total_mtiles; t += nw) {
            const int p = __builtin_amdgcn_readfirstlane(ba.mtile_pair[t]);
            if (__hip_atomic_load(&ba.state[p].done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) continue;
            const BatchPair &bp = ba.pairs[p];
            const int local = t - bp.mtile0;
            double v[NMET];
            metrics_by_type<R, COMP>(bp.type, bp.template args<R>(var), local % bp.mcolw, local / bp.mcolw, lane, v);
#pragma unroll
            for (int q = 0; q < NMET; ++q) {
                const double s = wave_sum(v[q]);
                if (lane == 0) ba.partials[(int64_t)t * NMET + q] = s;
            }
        }
        if (grid_sync(ba.bar, nblocks)) return;

        // per problem: reduce its tiles and take the stopping decision
        for (int p = gw; p < ba.B; p += nw) {
            BatchPairState &st = ba.state[p];
            if (__hip_atomic_load(&st.done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) continue;
            const BatchPair &bp = ba.pairs[p];
            reduce_tiles(ba.partials, bp.mtile0, bp.mtiles, lane, st.met);
            if (lane == 0) {
                const double *m = st.met;
                const double Rk = m[0] / bp.mu + (bp.l > 0 ? m[1] / bp.nu : 0.0) + m[2] / bp.tau - 2.0 * m[3];
                const bool conv = ba.tol > 0.0 && Rk <= ba.tol * ba.tol * bp.R0;
                const bool bad = !isfinite(Rk) || !isfinite(m[4]);
                st.iters = it + 1;
                st.checks = nchecks + 1;
                st.cur = 1 - par;
                st.wcur = 1 - wcur;
                if (conv || bad || it + 1 == ba.max_iters) {
                    st.converged = conv ? 1 : 0;
                    __hip_atomic_store(&st.done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_add(&ba.bar[3], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        if (grid_sync(ba.bar, nblocks)) return;
        ++nchecks;
        if (ld_acq(&ba.bar[3]) >= unsigned(ba.B)) break;  // every problem has stopped
    }
}

// ------------------------------------------------ one launch per iteration
//
// The same work without grid barriers: one launch advances every unfinished
// problem by one iteration (one wave per strip), a second launch computes the
// metrics tiles at a check, and a third lets one wave per problem reduce its
// tiles and take the stopping decision.  The host replays a check interval of
// these launches as one HIP graph and reads back only the count of stopped
// problems after each interval.

__device__ __forceinline__ int remap_block(int b, int nwg)
{
    // contiguous tiles (one problem's strips) on one XCD: workgroups are
    // dealt round-robin to the 8 XCDs
    constexpr int NX = 8;
    const int x = b % NX, idx = b / NX;
    const int q = nwg / NX, r = nwg % NX;
    return (x < r) ? x * (q + 1) + idx : r * (q + 1) + (x - r) * q + idx;
}

// One launch advances every unfinished problem by T iterations: T = 1 walks
// the list of 64-column strips, T = 2 the list of (64 - 2T)-column strips
// (pipelined, halo lanes and rows recomputed); var selects the step
// arguments (T = 1: parity * 4 + w buffer * 2 + check; T = 2: 8 + parity * 2 +
// w buffer).
template <typename R, bool COMP, int T>
__global__ __launch_bounds__(WAVE *STEP_WAVES_PER_WG) void batch_step_kernel(const BatchArgs ba, int var)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int t = remap_block(blockIdx.x, gridDim.x) * STEP_WAVES_PER_WG + threadIdx.x / WAVE;
    if (t >= (T == 1 ? ba.total_tiles : ba.total_tiles2)) return;
    const int p = __builtin_amdgcn_readfirstlane(T == 1 ? ba.tile_pair[t] : ba.tile_pair2[t]);
    if (ba.state[p].done) return;
    const BatchPair &bp = ba.pairs[p];
    const int ncolw = T == 1 ? bp.ncolw : bp.ncolw2;
    const int local = t - (T == 1 ? bp.tile0 : bp.tile0_2);
    strip_by_type<R, COMP, T>(bp.type, bp.template args<R>(var), local % ncolw, local / ncolw, lane);
}

template <typename R, bool COMP>
__global__ __launch_bounds__(WAVE *STEP_WAVES_PER_WG) void batch_metrics_kernel(const BatchArgs ba, int var)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int t = blockIdx.x * STEP_WAVES_PER_WG + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    if (t >= ba.total_mtiles) return;
    const int p = __builtin_amdgcn_readfirstlane(ba.mtile_pair[t]);
    if (ba.state[p].done) return;
    const BatchPair &bp = ba.pairs[p];
    const int local = t - bp.mtile0;
    double v[NMET];
    metrics_by_type<R, COMP>(bp.type, bp.template args<R>(var), local % bp.mcolw, local / bp.mcolw, lane, v);
#pragma unroll
    for (int q = 0; q < NMET; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) ba.partials[(int64_t)t * NMET + q] = s;
    }
}

// One wave per problem: add up the tiles, count the iterations, decide.
// last: this check follows the final iteration of the solve; cur / wcur:
// the buffers that hold the iterate after this interval, relative to the
// solve's start.
__global__ __launch_bounds__(WAVE *STEP_WAVES_PER_WG) void batch_decide_kernel(const BatchArgs ba, int iters,
                                                                                 int last, int cur, int wcur)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int p = blockIdx.x * STEP_WAVES_PER_WG + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    if (p >= ba.B) return;
    BatchPairState &st = ba.state[p];
    if (st.done) return;
    const BatchPair &bp = ba.pairs[p];
    reduce_tiles(ba.partials, bp.mtile0, bp.mtiles, lane, st.met);
    if (lane == 0) {
        const double *m = st.met;
        const double R = m[0] / bp.mu + (bp.l > 0 ? m[1] / bp.nu : 0.0) + m[2] / bp.tau - 2.0 * m[3];
        const bool conv = ba.tol > 0.0 && R <= ba.tol * ba.tol * bp.R0;
        const bool bad = !isfinite(R) || !isfinite(m[4]);
        st.iters += iters;
        st.checks += 1;
        st.cur = cur;
        st.wcur = wcur;
        if (conv || bad || last) {
            st.converged = conv ? 1 : 0;
            st.done = 1;
            atomicAdd(&ba.bar[3], 1u);
        }
    }
}

}  // namespace

template <int T>
hipError_t launch_batch_step_T(const BatchArgs &a, int dtype, bool comp, int var, hipStream_t s)
{
    const int tiles = T == 1 ? a.total_tiles : a.total_tiles2;
    if (tiles <= 0) return hipSuccess;
    const dim3 grid((tiles + STEP_WAVES_PER_WG - 1) / STEP_WAVES_PER_WG), block(WAVE * STEP_WAVES_PER_WG);
    if (dtype == 1)
        hipLaunchKernelGGL((batch_step_kernel<double, false, T>), grid, block, 0, s, a, var);
    else if (comp)
        hipLaunchKernelGGL((batch_step_kernel<float, true, T>), grid, block, 0, s, a, var);
    else
        hipLaunchKernelGGL((batch_step_kernel<float, false, T>), grid, block, 0, s, a, var);
    return hipGetLastError();
}

hipError_t launch_batch_step(const BatchArgs &a, int dtype, bool comp, int var, hipStream_t s, int T)
{
    if (T == 2) return launch_batch_step_T<2>(a, dtype, comp, var, s);
    if (T != 1) return hipErrorInvalidValue;
    return launch_batch_step_T<1>(a, dtype, comp, var, s);
}

hipError_t launch_batch_check(const BatchArgs &a, int dtype, bool comp, int var, int iters, bool last, int cur,
                              int wcur, hipStream_t s)
{
    const dim3 grid((a.total_mtiles + STEP_WAVES_PER_WG - 1) / STEP_WAVES_PER_WG), block(WAVE * STEP_WAVES_PER_WG);
    if (dtype == 1)
        hipLaunchKernelGGL((batch_metrics_kernel<double, false>), grid, block, 0, s, a, var);
    else if (comp)
        hipLaunchKernelGGL((batch_metrics_kernel<float, true>), grid, block, 0, s, a, var);
    else
        hipLaunchKernelGGL((batch_metrics_kernel<float, false>), grid, block, 0, s, a, var);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nd = (a.B + STEP_WAVES_PER_WG - 1) / STEP_WAVES_PER_WG;
    hipLaunchKernelGGL(batch_decide_kernel, dim3(nd), block, 0, s, a, iters, last ? 1 : 0, cur, wcur);
    return hipGetLastError();
}

int batch_type(int k, int gk, int lb)
{
    if (k == 1 && gk == G_NONE && lb == 0) return 0;
    if (k == 2 && gk == G_PATH && lb == 1) return 1;
    if (k == 3 && gk == G_COMPLETE && lb == 3) return 2;
    if (k == 3 && gk == G_PATH && lb == 2) return 3;
    return -1;
}

hipError_t batch_blocks_per_cu(int dtype, bool comp, int *blocks)
{
    const int bs = WAVE * STEP_WAVES_PER_WG;
    if (dtype == 1) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, batch_kernel<double, false>, bs, 0);
    if (comp) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, batch_kernel<float, true>, bs, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, batch_kernel<float, false>, bs, 0);
}

hipError_t launch_batch(const BatchArgs &a, int dtype, bool comp, int nblocks, hipStream_t s)
{
    const dim3 block(WAVE * STEP_WAVES_PER_WG);
    if (dtype == 1)
        hipLaunchKernelGGL((batch_kernel<double, false>), dim3(nblocks), block, 0, s, a);
    else if (comp)
        hipLaunchKernelGGL((batch_kernel<float, true>), dim3(nblocks), block, 0, s, a);
    else
        hipLaunchKernelGGL((batch_kernel<float, false>), dim3(nblocks), block, 0, s, a);
    return hipGetLastError();
}

}  // namespace omt
