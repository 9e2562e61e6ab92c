// Device code of the fused PDHG iteration, shared by the per-launch step
// kernel and the persistent batched kernel.
#pragma once

#include "omt_kernels.h"

namespace omt {
namespace dev {

// ------------------------------------------------------------ lane moves
//
// The value of the neighbouring lane (column), by a DPP wavefront shift of
// one lane: a modifier of a vector move, with no round trip through the LDS
// crossbar and no counter to wait on.  A lane with no neighbour (lane 63
// for lane_next, lane 0 for lane_prev) keeps its own value, as a shuffle
// that leaves the wave does.
constexpr int DPP_WAVE_SHL1 = 0x130;  // lane l reads lane l + 1
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane l reads lane l - 1
template <int CTRL>
__device__ __forceinline__ int dpp_shift(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}
__device__ __forceinline__ float lane_next(float v) { return __int_as_float(dpp_shift<DPP_WAVE_SHL1>(__float_as_int(v))); }
__device__ __forceinline__ float lane_prev(float v) { return __int_as_float(dpp_shift<DPP_WAVE_SHR1>(__float_as_int(v))); }
__device__ __forceinline__ double lane_next(double v)
{
    return __hiloint2double(dpp_shift<DPP_WAVE_SHL1>(__double2hiint(v)), dpp_shift<DPP_WAVE_SHL1>(__double2loint(v)));
}
__device__ __forceinline__ double lane_prev(double v)
{
    return __hiloint2double(dpp_shift<DPP_WAVE_SHR1>(__double2hiint(v)), dpp_shift<DPP_WAVE_SHR1>(__double2loint(v)));
}

// Field accesses outside the step's row buffers (the metrics kernel) go
// through a global-address-space pointer.  The batched kernels read their
// field pointers from a table in memory, where the compiler cannot infer the
// address space and would otherwise emit flat accesses, which wait on both
// the vector-memory and the LDS counters.
#define OMT_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const OMT_GLOBAL T *gptr(const T *p)
{
    return (const OMT_GLOBAL T *)p;
}
template <typename R>
__device__ __forceinline__ R ld_field(const R *p)
{
    return *gptr(p);
}

// ------------------------------------------------------------ row buffers
//
// A strip reads and writes each field (all planes of phi, u, w, f) one row
// at a time.  Every such access goes through a raw buffer descriptor that
// starts at that row of the field's first plane and covers the field's
// planes in use (row_rsrc); a lane reaches plane c, column j at byte offset
// (c P + j) s.  The hardware range check returns 0 for a load and drops a
// store whenever that offset lies past the descriptor: a lane outside the
// grid, or one that must not store, carries offset OFF_NONE, and a row that
// must not be touched gets a descriptor of length 0.  So no memory
// instruction needs a branch, every one issues on every path, and the
// compiler can wait on exactly the loads it needs instead of on every store
// still in flight.  Descriptors are wave-uniform (scalar registers).
constexpr int RSRC_WORD3 = 0x00020000;      // raw 32-bit data, gfx9-family buffer descriptor
constexpr unsigned OFF_NONE = 0x80000000u;  // a byte offset past every row
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

// Descriptor from element `elem` (row r of plane 0) of a field whose planes
// are P elements apart; plane c of that row is at byte offset c P s + j s.
// `bytes` = ((planes - 1) P + n) s covers exactly the planes in use, and is
// below 2^31 (checked by the host), so OFF_NONE + c P s stays past it.
template <typename R>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const R *base, int64_t elem, bool valid, int bytes)
{
    // a zero-length descriptor never touches memory; its base stays at the
    // field's start so that no pointer past the allocation is formed
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<R *>(base) + (valid ? elem : 0), (short)0,
                                             valid ? bytes : 0, RSRC_WORD3);
}
// bytes a row descriptor of a field with `planes` planes must cover
__device__ __forceinline__ int field_bytes(int planes, int64_t P, int n, int s)
{
    return int(((int64_t)(planes - 1) * P + n) * s);
}
template <typename R>
__device__ __forceinline__ R buf_ld(__amdgpu_buffer_rsrc_t rs, unsigned off)
{
    if constexpr (sizeof(R) == 8)
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
    else
        return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
}
template <typename R>
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t rs, unsigned off, R v)
{
    if constexpr (sizeof(R) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), rs, off, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, off, 0, 0);
}

// value of lane L (a wave-uniform result)
__device__ __forceinline__ float lane_get(float v, int L)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), L));
}
__device__ __forceinline__ double lane_get(double v, int L)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), L);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), L);
    return __hiloint2double(hi, lo);
}

// ------------------------------------------------------------ shrinks (App. B)

template <typename R>
__device__ __forceinline__ R shrink_scale(R r, R t)
{
    // (1 - t/r) for r >= t, else 0: the factor applied to the block.
    return (r >= t && r > R(0)) ? R(1) - t / r : R(0);
}

template <typename R, int K>
__device__ __forceinline__ void shrink_u(int unorm, R (&bx)[K], R (&by)[K], R t)
{
    if (unorm == 0) {  // sum over channels of ||(u_x, u_y)||_2
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const R s = shrink_scale(sqrt(bx[c] * bx[c] + by[c] * by[c]), t);
            bx[c] = bx[c] * s;
            by[c] = by[c] * s;
        }
    } else if (unorm == 1) {  // element-wise
#pragma unroll
        for (int c = 0; c < K; ++c) {
            bx[c] = bx[c] * shrink_scale(fabs(bx[c]), t);
            by[c] = by[c] * shrink_scale(fabs(by[c]), t);
        }
    } else {  // one block of all 2k components
        R r2 = R(0);
#pragma unroll
        for (int c = 0; c < K; ++c) r2 = r2 + bx[c] * bx[c];
#pragma unroll
        for (int c = 0; c < K; ++c) r2 = r2 + by[c] * by[c];
        const R s = shrink_scale(sqrt(r2), t);
#pragma unroll
        for (int c = 0; c < K; ++c) {
            bx[c] = bx[c] * s;
            by[c] = by[c] * s;
        }
    }
}

template <typename R, int L>
__device__ __forceinline__ void shrink_w(int wnorm, R (&w)[L], R t)
{
    if (wnorm == 0) {
#pragma unroll
        for (int e = 0; e < L; ++e) w[e] = w[e] * shrink_scale(fabs(w[e]), t);
    } else {
        R r2 = R(0);
#pragma unroll
        for (int e = 0; e < L; ++e) r2 = r2 + w[e] * w[e];
        const R s = shrink_scale(sqrt(r2), t);
#pragma unroll
        for (int e = 0; e < L; ++e) w[e] = w[e] * s;
    }
}

// Grouped entry-wise norm sum_g wt_g ||x_g||_2 over groups of one or two
// coordinates (wt > 0 starts a group; a following 0 joins it): the factor
// of the shrink with threshold wt_g * t for every coordinate.
template <typename R, int N>
__device__ __forceinline__ void group_scales(const R *wt, const R (&x)[N], R t, R (&sc)[N])
{
#pragma unroll
    for (int c = 0; c < N; ++c) {
        if (wt[c] > R(0)) {
            const bool pair = (c + 1 < N) && wt[c + 1] == R(0);
            const R r = pair ? sqrt(x[c] * x[c] + x[c + 1] * x[c + 1]) : fabs(x[c]);
            const R s = shrink_scale<R>(r, wt[c] * t);
            sc[c] = s;
            if (c + 1 < N && pair) sc[c + 1] = s;
        }
    }
}

}  // namespace dev
}  // namespace omt

#include "matrix_device.h"

namespace omt {
namespace dev {

// Shrink of the u block of one direction of a matrix problem: the grouped
// entry-wise norm (u norm 3) or the nuclear norm (u norm 4).
template <typename R, int K, bool NUC>
__device__ __forceinline__ void matrix_u_shrink(int unorm, const R *uwt, R (&x)[K], R t)
{
    if (!NUC || unorm == 3) {
        R sc[K];
#pragma unroll
        for (int c = 0; c < K; ++c) sc[c] = R(0);
        group_scales<R, K>(uwt, x, t, sc);
#pragma unroll
        for (int c = 0; c < K; ++c) x[c] = x[c] * sc[c];
    } else {
        herm_nuc_shrink<R, K>(x, t);
    }
}

// ------------------------------------------------------------ channel graph

// Endpoints (a_e, b_e), a_e < b_e, of edge e of the compiled graph kinds.
constexpr int complete_row_start(int K, int a) { return a * (K - 1) - a * (a - 1) / 2; }
template <int GK, int K>
constexpr int edge_a(int e)
{
    if (GK == G_PATH) return e;
    int a = 0;
    while (a + 1 < K && complete_row_start(K, a + 1) <= e) ++a;
    return a;
}
template <int GK, int K>
constexpr int edge_b(int e)
{
    if (GK == G_PATH) return e + 1;
    const int a = edge_a<GK, K>(e);
    return a + 1 + (e - complete_row_start(K, a));
}

// ------------------------------------------------------------ check terms
//
// For one step (u, w, phi) -> (u', w', phi') every pixel contributes, in
// FP64, the terms listed in metrics_device.h.

// div_G of w' - w (dgd) and of w' (dg1) at channel c, in edge order:
// D diag(1/c) applied to the transfer (div_G is its negative).
template <typename R, int K, int GK, int LA, typename W>
__device__ __forceinline__ void graph_div_terms(const StepArgs<R> &a, int c, const W (&we0)[LA], const W (&we1)[LA],
                                                double &dgd, double &dg1)
{
    dgd = 0.0;
    dg1 = 0.0;
#pragma unroll
    for (int e = 0; e < LA; ++e) {
        if constexpr (GK == G_DENSE || is_matrix_kind(GK)) {
            dgd += double(a.gm[c * LMAX + e]) * (double(we1[e]) - double(we0[e]));
            dg1 += double(a.gm[c * LMAX + e]) * double(we1[e]);
        } else {
            if (edge_a<GK, K>(e) == c) {
                dgd += double(a.ic[e]) * (double(we1[e]) - double(we0[e]));
                dg1 += double(a.ic[e]) * double(we1[e]);
            }
            if (edge_b<GK, K>(e) == c) {
                dgd -= double(a.ic[e]) * (double(we1[e]) - double(we0[e]));
                dg1 -= double(a.ic[e]) * double(we1[e]);
            }
        }
    }
}

// The check terms of one channel of one pixel, added to the pixel's sums
// acc in a fixed order.  Arguments are the old (0) and new (1) values:
// potential p, flux (ux, uy) at the pixel, u_x of the pixel above (xl) and
// u_y of the pixel to the left (yl), each already zero where App. A's ghost
// rules make it so; dgd, dg1 from graph_div_terms; fc the source.  sq and
// u2 collect squares for the regulariser and the ||u||_2 norm.  Every path
// that takes a check (the separate metrics pass and the check fused into
// the step) calls this, then pixel_terms, then adds the pixel's sums to its
// column's, so both give the same bits.
__device__ __forceinline__ void chan_terms(double (&acc)[NMET], double &sq, double &u2, int unorm, double inv_h,
                                           double p0, double p1, double ux0, double ux1, double uy0, double uy1,
                                           double xl0, double xl1, double yl0, double yl1, double dgd, double dg1,
                                           double fc)
{
    const double dp = p1 - p0;
    const double dux = ux1 - ux0, duy = uy1 - uy0;
    const double ddiv = ((dux - (xl1 - xl0)) + duy - (yl1 - yl0)) * inv_h;
    const double div1 = ((ux1 - xl1) + uy1 - yl1) * inv_h;
    acc[0] += dux * dux + duy * duy;
    acc[2] += dp * dp;
    acc[3] += dp * (ddiv - dgd);
    acc[5] += p1 * fc;
    const double r = (div1 - dg1) + fc;
    acc[6] += r * r;
    acc[7] += p1;
    sq += ux1 * ux1 + uy1 * uy1;
    if (unorm == 0)
        acc[4] += sqrt(ux1 * ux1 + uy1 * uy1);
    else if (unorm == 1)
        acc[4] += fabs(ux1) + fabs(uy1);
    else
        u2 += ux1 * ux1 + uy1 * uy1;
}

// The transfer and norm terms of one pixel of the vector method, after its
// channels: ||u||_2 (u norm 2), |w' - w|^2, alpha ||w'||_w and the
// regulariser.  Transfers past the l in use (a dense graph's bucket) are 0.
template <int LA, typename W>
__device__ __forceinline__ void pixel_terms(double (&acc)[NMET], double sq, double u2, int unorm, int wnorm,
                                            double alpha, double eps, int l, const W (&we0)[LA], const W (&we1)[LA])
{
    if (unorm == 2) acc[4] += sqrt(u2);
    double wn = 0.0, w2 = 0.0;
#pragma unroll
    for (int e = 0; e < LA; ++e) {
        const double x0 = e < l ? double(we0[e]) : 0.0, x1 = e < l ? double(we1[e]) : 0.0;
        acc[1] += (x1 - x0) * (x1 - x0);
        wn += fabs(x1);
        w2 += x1 * x1;
    }
    acc[4] += alpha * (wnorm == 0 ? wn : sqrt(w2));
    if (eps > 0.0) acc[4] += eps * (sq + w2);  // quadratic regularisation
}

// Sum over the 64 lanes of a wave; lane 0 holds the result.  The tree adds
// neighbouring lanes first (offsets 1, 2, 4, ..., 32), so lane 4q holds the
// sum of its quad of columns after the first two levels: a check fused into
// a strip of any width (a whole number of 4-column quads) reproduces those
// quad sums, and quads_to_tiles the remaining levels.
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) x += __shfl_down(x, off, WAVE);
    return x;
}

// ------------------------------------------------------------ fused check
//
// A check launch (CHK) takes the check of Sec. 6.1 in the same pass as the
// iteration: the last stage, which holds both the old and the new iterate of
// every pixel it stores, adds the pixel's check terms (chan_terms and
// pixel_terms above, the same code as the separate metrics pass) to
// per-column sums over an aligned block of MET_ROWS rows, and at
// the end of each block adds the columns of every aligned 4-column quad as
// the first two levels of wave_sum do.  Every launch shape stores whole
// quads (strips are 64 - 2T columns wide from column (64 - 2T) wc, and
// 64 - 2T is a multiple of 4 for T = 1, 2, 4, 8), so the quad sums, and the
// tiles and totals formed from them in a fixed order, do not depend on the
// launch shape and equal those of the separate pass bit for bit.  (The host
// takes checks in single-iteration launches only: with the check, a
// two-iteration launch at k = 8 needs more than 256 registers.)
template <typename R, int K>
struct ChkState {
    R xo[K], xn[K];       // old and new u_x of this lane's pixel on the row above
    double col[NMET];     // this column's sums over the current row block
    int qlane;            // lane % 4 of the first column of each quad
};

// ------------------------------------------------------------ one stage

// Columns just outside an aligned strip, lane c holding channel c: the
// potential one column to the right (row r) and, one column to the left,
// the potential on rows r and r+1 and the flux on row r.
template <typename R>
struct Edges {
    R RA, RAl, LA, LAl, LB, LBl, Lux, Luy;
    bool hasL;
};

// Iteration of one pixel row r for this lane's column.  pA/pB: potential
// on rows r and r+1 (hi and, if COMP, lo parts); ux, uy, w: state on row r;
// carry: 2u'_x - u_x of row r-1 on entry, of row r on exit.  Outputs go to
// pO/pOl/uxO/uyO/wO and to memory: row r of each output plane (element
// offset ro = r * pitch within the plane, planes P elements apart) if st_row
// is set, at this lane's byte offset soff (OFF_NONE for a lane that must not
// store).  In
// the aligned mode (ALN) lane 63 takes its right potential and lane 0 its
// left flux from E instead of the neighbouring lane; the left flux is
// recomputed with the same expressions as every other pixel's.
//
// CHK (a check launch's last stage): also add this row's check terms to ck
// (pixel row r, column j, counted where it is stored) and, at the end of an
// aligned block of MET_ROWS rows, store the block's quad sums to a.qpart.
template <typename R, int K, int GK, int L, int LA, bool COMP, bool ALN, bool CHK = false>
__device__ __forceinline__ void stage(const StepArgs<R> &a, int lane, bool lane_ok, bool last_row, bool last_col,
                                      const R (&pA)[K], const R (&pAl)[K], const R (&pB)[K], const R (&pBl)[K],
                                      const R (&ux)[K], const R (&uy)[K], const R (&w)[LA], const R (&f)[K],
                                      const Edges<R> &E, bool st_row, int64_t ro, unsigned soff, int64_t P,
                                      R (&carry)[K], R (&pO)[K],
                                      R (&pOl)[K], R (&uxO)[K], R (&uyO)[K], R (&wO)[LA],
                                      ChkState<R, K> &ck, int r = 0, int j = 0)
{
    // this row of every output field (zero-length descriptors unless st_row)
    const unsigned Psz = unsigned(P) * unsigned(sizeof(R)), Pszl = unsigned(P) * 4u;
    const unsigned soffl = sizeof(R) == 4 ? soff : OFF_NONE;  // compensated potentials are FP32 only
    const auto rphi = row_rsrc(a.phi_out, ro, st_row, field_bytes(K, P, a.n, sizeof(R)));
    const auto ru = row_rsrc(a.u_out, ro, st_row, field_bytes(2 * K, P, a.n, sizeof(R)));
    const auto rw = row_rsrc(a.w_out, ro, st_row && L > 0, field_bytes(a.l, P, a.n, sizeof(R)));
    const auto rplo = row_rsrc(a.plo_out, ro, COMP && st_row, field_bytes(K, P, a.n, 4));
    // the matrix kinds only take the Frobenius (u 2, w 1) and grouped
    // entry-wise (u 3, w 2) norms: fold the others away at compile time
    const int unorm = GK == G_MATNUC ? (a.unorm >= 3 ? a.unorm : 2) : GK == G_MATRIX ? (a.unorm == 3 ? 3 : 2)
                                                                                     : a.unorm;
    const int wnorm = GK == G_MATNUC ? (a.wnorm >= 2 ? a.wnorm : 1) : GK == G_MATRIX ? (a.wnorm == 2 ? 2 : 1)
                                                                                     : a.wnorm;

    // w-update: shrink_w(w + nu grad_G phi, alpha nu); (grad_G phi)_e =
    // (phi_a - phi_b) / c_e (Sec. 3.1), or M^T phi for a dense graph
    R wb[LA];
    if constexpr (L > 0) {
        R wt[LA];
#pragma unroll
        for (int e = 0; e < LA; ++e) {
            R s = R(0);
            if constexpr (GK == G_DENSE || is_matrix_kind(GK)) {
#pragma unroll
                for (int c = 0; c < K; ++c) {
                    s = s + a.gm[c * LMAX + e] * pA[c];
                    if (COMP) s = s + a.gm[c * LMAX + e] * pAl[c];
                }
                wt[e] = (e < a.l) ? w[e] + a.nu * s : R(0);
            } else {
                const int ea = edge_a<GK, K>(e), eb = edge_b<GK, K>(e);
                s = pA[ea] - pA[eb];
                if (COMP) s = s + (pAl[ea] - pAl[eb]);
                wt[e] = w[e] + a.nu * (s * a.ic[e]);
            }
        }
        if constexpr (is_matrix_kind(GK)) {
            if (wnorm == 2) {
                R sc[LA];
                group_scales<R, LA>(a.wwt, wt, a.anu, sc);
#pragma unroll
                for (int e = 0; e < LA; ++e) wt[e] = wt[e] * sc[e];
            } else if (GK == G_MATNUC && wnorm == 3) {
                skew_nuc_shrink<R, K, LA>(wt, a.l, a.anu);
            } else {
                shrink_w<R, LA>(wnorm, wt, a.anu);
            }
        } else {
            shrink_w<R, LA>(wnorm, wt, a.anu);
        }
#pragma unroll
        for (int e = 0; e < LA; ++e) {
            wt[e] = wt[e] * a.wreg;  // regularised prox (factor 1 without regularisation)
            if (!lane_ok) wt[e] = R(0);
            wO[e] = wt[e];
            wb[e] = R(2) * wt[e] - w[e];
            if (L > 0) buf_st<R>(rw, soff + unsigned(e) * Psz, wt[e]);
        }
    }

    double cacc[NMET], csq = 0.0, cu2 = 0.0;
#pragma unroll
    for (int q = 0; q < NMET; ++q) cacc[q] = 0.0;

    // u~ = u + mu grad_x phi for this lane's pixel and, in the aligned mode,
    // for the pixel left of the strip (wave-uniform)
    auto utilde = [&](int c, R &tx, R &ty) {
        R pr = lane_next(pA[c]);
        R prl = COMP ? lane_next(pAl[c]) : R(0);
        if (ALN && lane == WAVE - 1) {
            pr = lane_get(E.RA, c);
            prl = COMP ? lane_get(E.RAl, c) : R(0);
        }
        R gx = pB[c] - pA[c];
        R gy = pr - pA[c];
        if (COMP) {
            gx = gx + (pBl[c] - pAl[c]);
            gy = gy + (prl - pAl[c]);
        }
        tx = last_row ? R(0) : ux[c] + a.mu_h * gx;
        ty = last_col ? R(0) : uy[c] + a.mu_h * gy;
    };
    auto utilde_left = [&](int c, R &tx, R &ty) {
        const R hA = lane_get(E.LA, c), hB = lane_get(E.LB, c), hR = lane_get(pA[c], 0);
        R gx = hB - hA;
        R gy = hR - hA;
        if (COMP) {
            const R hAl = lane_get(E.LAl, c), hBl = lane_get(E.LBl, c), hRl = lane_get(pAl[c], 0);
            gx = gx + (hBl - hAl);
            gy = gy + (hRl - hAl);
        }
        tx = last_row ? R(0) : lane_get(E.Lux, c) + a.mu_h * gx;
        ty = lane_get(E.Luy, c) + a.mu_h * gy;  // the left column is never the last one
    };
    // ||u||_2 over all 2k components needs the norm of the whole block first
    R s_all = R(0), s_left = R(0);
    if (unorm == 2) {
        R r2 = R(0), r2l = R(0), tx, ty;
#pragma unroll
        for (int c = 0; c < K; ++c) {
            utilde(c, tx, ty);
            r2 = r2 + tx * tx;
            if (ALN) {
                utilde_left(c, tx, ty);
                r2l = r2l + tx * tx;
            }
        }
#pragma unroll
        for (int c = 0; c < K; ++c) {
            utilde(c, tx, ty);
            r2 = r2 + ty * ty;
            if (ALN) {
                utilde_left(c, tx, ty);
                r2l = r2l + ty * ty;
            }
        }
        s_all = shrink_scale<R>(sqrt(r2), a.mu);
        s_left = shrink_scale<R>(sqrt(r2l), a.mu);
    }
    // grouped entry-wise norm of the matrix kinds (u norm 3): per-coordinate
    // factors of this pixel and, in the aligned mode, of the pixel left of
    // the strip
    R gsx[K], gsy[K], gsxl[K], gsyl[K];
#pragma unroll
    for (int c = 0; c < K; ++c) gsx[c] = gsy[c] = gsxl[c] = gsyl[c] = R(0);
    if constexpr (GK == G_MATRIX) {
        if (unorm == 3) {
            R qx[K], qy[K];
#pragma unroll
            for (int c = 0; c < K; ++c) utilde(c, qx[c], qy[c]);
            group_scales<R, K>(a.uwt, qx, a.mu, gsx);
            group_scales<R, K>(a.uwt, qy, a.mu, gsy);
            if (ALN) {
#pragma unroll
                for (int c = 0; c < K; ++c) utilde_left(c, qx[c], qy[c]);
                group_scales<R, K>(a.uwt, qx, a.mu, gsxl);
                group_scales<R, K>(a.uwt, qy, a.mu, gsyl);
            }
        }
    }
    // the matrix kind with nuclear norms (u norm 3 or 4): the shrunk
    // coordinates of each direction, as the shrink is no per-coordinate factor
    R mx[K], my[K], mxl[K], myl[K];
#pragma unroll
    for (int c = 0; c < K; ++c) mx[c] = my[c] = mxl[c] = myl[c] = R(0);
    if constexpr (GK == G_MATNUC) {
        if (unorm >= 3) {
#pragma unroll
            for (int c = 0; c < K; ++c) utilde(c, mx[c], my[c]);
            matrix_u_shrink<R, K, true>(unorm, a.uwt, mx, a.mu);
            matrix_u_shrink<R, K, true>(unorm, a.uwt, my, a.mu);
            if (ALN) {
#pragma unroll
                for (int c = 0; c < K; ++c) utilde_left(c, mxl[c], myl[c]);
                matrix_u_shrink<R, K, true>(unorm, a.uwt, mxl, a.mu);
                matrix_u_shrink<R, K, true>(unorm, a.uwt, myl, a.mu);
            }
        }
    }
    auto shrink_pair = [&](R tx, R ty, R sblock, R &bx, R &by) {
        if (unorm == 0) {  // sum over channels of ||(u_x, u_y)||_2 (App. B shrink_2 per channel)
            const R s = shrink_scale<R>(sqrt(tx * tx + ty * ty), a.mu);
            bx = tx * s;
            by = ty * s;
        } else if (unorm == 1) {  // element-wise shrink_1
            bx = tx * shrink_scale<R>(fabs(tx), a.mu);
            by = ty * shrink_scale<R>(fabs(ty), a.mu);
        } else {
            bx = tx * sblock;
            by = ty * sblock;
        }
    };

    // per channel: u-update, extrapolation, divergences, phi-update
#pragma unroll
    for (int c = 0; c < K; ++c) {
        R tx, ty, bx, by;
        utilde(c, tx, ty);
        if (GK == G_MATRIX && unorm == 3) {
            bx = tx * gsx[c];
            by = ty * gsy[c];
        } else if (GK == G_MATNUC && unorm >= 3) {
            bx = mx[c];
            by = my[c];
        } else {
            shrink_pair(tx, ty, s_all, bx, by);
        }
        bx = bx * a.ureg;  // regularised prox (factor 1 without regularisation)
        by = by * a.ureg;
        if (!lane_ok) bx = by = R(0);
        const R ubx = R(2) * bx - ux[c];
        const R uby = R(2) * by - uy[c];
        R ubl = lane_prev(uby);
        R ynl = CHK ? lane_prev(by) : R(0), yol = CHK ? lane_prev(uy[c]) : R(0);  // u_y left: new, old
        if (ALN) {
            R ex, ey, ebx, eby;
            utilde_left(c, ex, ey);
            if (GK == G_MATRIX && unorm == 3) {
                ebx = ex * gsxl[c];
                eby = ey * gsyl[c];
            } else if (GK == G_MATNUC && unorm >= 3) {
                ebx = mxl[c];
                eby = myl[c];
            } else {
                shrink_pair(ex, ey, s_left, ebx, eby);
            }
            eby = eby * a.ureg;
            const R el = E.hasL ? R(2) * eby - lane_get(E.Luy, c) : R(0);
            if (lane == 0) ubl = el;
            if (CHK && lane == 0) {
                ynl = E.hasL ? eby : R(0);
                yol = E.hasL ? lane_get(E.Luy, c) : R(0);
            }
        }
        const R dx = (((ubx - carry[c]) + uby) - ubl) * a.inv_h;
        // div_G(w) = -D diag(1/c) w: dg is D diag(1/c) w, accumulated in edge order
        R dg = R(0);
        if constexpr (L > 0) {
#pragma unroll
            for (int e = 0; e < LA; ++e) {
                if constexpr (GK == G_DENSE || is_matrix_kind(GK)) {
                    dg = dg + a.gm[c * LMAX + e] * wb[e];
                } else {
                    if (edge_a<GK, K>(e) == c) dg = dg + a.ic[e] * wb[e];
                    if (edge_b<GK, K>(e) == c) dg = dg - a.ic[e] * wb[e];
                }
            }
        }
        const R inc = a.tau * ((dx - dg) + f[c]);
        R po, pol = R(0);
        if (COMP) {
            // error-free sum of (hi, lo) and the increment (TwoSum)
            const R t = pAl[c] + inc;
            const R s = pA[c] + t;
            const R bb = s - pA[c];
            const R err = (pA[c] - (s - bb)) + (t - bb);
            po = lane_ok ? s : R(0);
            pol = lane_ok ? err : R(0);
        } else {
            po = lane_ok ? pA[c] + inc : R(0);
        }
        carry[c] = ubx;
        pO[c] = po;
        pOl[c] = pol;
        uxO[c] = bx;
        uyO[c] = by;
        buf_st<R>(rphi, soff + unsigned(c) * Psz, po);
        if (COMP) buf_st<float>(rplo, soffl + unsigned(c) * Pszl, float(pol));
        buf_st<R>(ru, soff + unsigned(c) * Psz, bx);
        buf_st<R>(ru, soff + unsigned(K + c) * Psz, by);
        if constexpr (CHK) {
            // the values the separate metrics pass reads back, ghosts zeroed
            const double p0 = COMP ? double(pA[c]) + double(pAl[c]) : double(pA[c]);
            const double p1 = COMP ? double(po) + double(pol) : double(po);
            const bool gx = r < a.m - 1, gy = j < a.n - 1;
            const double ux0 = gx ? double(ux[c]) : 0.0, ux1 = gx ? double(bx) : 0.0;
            const double uy0 = gy ? double(uy[c]) : 0.0, uy1 = gy ? double(by) : 0.0;
            const double xl0 = r > 0 ? double(ck.xo[c]) : 0.0, xl1 = r > 0 ? double(ck.xn[c]) : 0.0;
            const double yl0 = j > 0 ? double(yol) : 0.0, yl1 = j > 0 ? double(ynl) : 0.0;
            double dgd = 0.0, dg1 = 0.0;
            if constexpr (L > 0) graph_div_terms<R, K, GK, LA>(a, c, w, wO, dgd, dg1);
            chan_terms(cacc, csq, cu2, unorm, double(a.inv_h), p0, p1, ux0, ux1, uy0, uy1, xl0, xl1, yl0, yl1, dgd,
                       dg1, double(f[c]));
            ck.xo[c] = ux[c];
            ck.xn[c] = bx;
        }
    }
    if constexpr (CHK) {
        pixel_terms<LA>(cacc, csq, cu2, unorm, wnorm, a.alpha, a.eps, L > 0 ? a.l : 0, w, wO);
        // a pixel this launch stores is counted, once
        const bool mine = st_row && soff != OFF_NONE;
#pragma unroll
        for (int q = 0; q < NMET; ++q) ck.col[q] += mine ? cacc[q] : 0.0;
        // end of an aligned row block (wave-uniform): quad sums of the columns
        if (st_row && (r % MET_ROWS == MET_ROWS - 1 || r == a.m - 1)) {
            // a quad's first column sits on lanes with lane % 4 == ck.qlane;
            // it stores if its column is one this strip stores
            const bool base = (lane & 3) == ck.qlane && soff != OFF_NONE;
            double *dst = a.qpart + (int64_t)(r / MET_ROWS) * a.nq + (j >> 2);
#pragma unroll
            for (int q = 0; q < NMET; ++q) {
                double x = ck.col[q];
                x += __shfl_down(x, 1u, WAVE);
                x += __shfl_down(x, 2u, WAVE);
                if (base) dst[q * a.qstride] = x;
                ck.col[q] = 0.0;
            }
        }
    }
}

__device__ __forceinline__ int xcd_remap(int b, int nwg)
{
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD one
    // contiguous range of tiles (a band of rows) so that halo rows and
    // columns shared by neighbouring waves hit in that XCD's L2.
    constexpr int NX = 8;
    const int x = b % NX, idx = b / NX;
    const int q = nwg / NX, r = nwg % NX;
    return (x < r) ? x * (q + 1) + idx : r * (q + 1) + (x - r) * q + idx;
}

// T iterations on the strip (column block wc, row chunk wr) of one wave.
// CHK: a check launch (rows per wave a multiple of MET_ROWS; a.qpart set).
template <typename R, int K, int GK, int L, int T, bool COMP, bool CHK = false>
__device__ __forceinline__ void process_strip(const StepArgs<R> &a, int wc, int wr, int lane)
{
    constexpr int LA = L > 0 ? L : 1;
    constexpr bool ALN = (T == 1);  // aligned 64-column strips

    // the strip's coordinates are wave-uniform: every row bound and buffer
    // descriptor derived from them lives in scalar registers
    wc = __builtin_amdgcn_readfirstlane(wc);
    wr = __builtin_amdgcn_readfirstlane(wr);
    const int j = ALN ? wc * WAVE + lane : wc * (WAVE - 2 * T) - T + lane;
    const bool jin = (j >= 0) && (j < a.n);
    const bool jout = ALN ? jin : (jin && lane >= T && lane < WAVE - T);
    const bool last_col = (j == a.n - 1);
    const int i0 = wr * a.rows;
    const int i1 = min(i0 + a.rows, a.m);
    const int rs = max(i0 - T, 0);
    const int re = min(i1 + T - 1, a.m);
    const int64_t P = a.plane;
    const int pitch = a.pitch;

    // this lane's byte offset in a row (past the row for a column outside
    // the grid), and where it stores (only the strip's own columns)
    const unsigned voff = jin ? unsigned(j) * unsigned(sizeof(R)) : OFF_NONE;
    const unsigned voffl = jin ? unsigned(j) * 4u : OFF_NONE;  // compensated low parts (float)
    const unsigned soff = jout ? voff : OFF_NONE;
    const int nb_phi = field_bytes(K, P, a.n, sizeof(R)), nb_u = field_bytes(2 * K, P, a.n, sizeof(R));
    const int nb_w = field_bytes(a.l, P, a.n, sizeof(R)), nb_lo = field_bytes(K, P, a.n, 4);

    // plane stride in bytes, made opaque at every row step so that the
    // compiler forms each plane's offset where it is used rather than
    // keeping one per plane for the whole strip
    unsigned Psz = unsigned(P) * unsigned(sizeof(R)), Pszl = unsigned(P) * 4u;

    // aligned mode: columns just outside the strip, lane c holding channel c
    // (plane c of the field at that column; lanes >= K read nothing)
    const int jL = wc * WAVE - 1, jR = wc * WAVE + WAVE;
    const bool hasL = ALN && jL >= 0, hasR = ALN && jR < a.n;
    const bool hl = lane < K;
    const unsigned hcP = unsigned(hl ? lane : 0) * unsigned(P);
    const unsigned eR = hl && hasR ? (hcP + unsigned(jR)) * unsigned(sizeof(R)) : OFF_NONE;
    const unsigned eL = hl && hasL ? (hcP + unsigned(jL)) * unsigned(sizeof(R)) : OFF_NONE;
    const unsigned eRl = hl && hasR ? (hcP + unsigned(jR)) * 4u : OFF_NONE;
    const unsigned eLl = hl && hasL ? (hcP + unsigned(jL)) * 4u : OFF_NONE;
    auto ld_edge = [&](unsigned eoff, int r, const R *base, int nb, int plane0, bool ok) -> R {
        return buf_ld<R>(row_rsrc(base, (int64_t)r * pitch, ok, nb), eoff + unsigned(plane0) * Psz);
    };
    auto ld_edge_lo = [&](unsigned eoff, int r, bool ok) -> R {
        return R(buf_ld<float>(row_rsrc(a.plo_in, (int64_t)r * pitch, ok, nb_lo), eoff));
    };
    // next-row values (prefetched) of the edge columns
    R nRA = R(0), nRAl = R(0);                    // phi(r, jR)
    R nLA = R(0), nLAl = R(0), nLB = R(0), nLBl = R(0);  // phi(r, jL), phi(r+1, jL)
    R nLux = R(0), nLuy = R(0);                   // u(r, jL)

    // stage-0 inputs of the next row, loaded one step ahead
    R nA[K], nAl[K], nB[K], nBl[K], nux[K], nuy[K], nw[LA], nf[K];
    // row r of the potential (ok: the row exists and is wanted)
    auto load_phi = [&](int r, bool ok, R (&hi)[K], R (&lo)[K]) {
        ok = ok && r < a.m;
        const int64_t o = (int64_t)r * pitch;
        const auto rp = row_rsrc(a.phi_in, o, ok, nb_phi);
        const auto rl = row_rsrc(a.plo_in, o, COMP && ok, nb_lo);
#pragma unroll
        for (int c = 0; c < K; ++c) {
            hi[c] = buf_ld<R>(rp, voff + unsigned(c) * Psz);
            lo[c] = COMP ? R(buf_ld<float>(rl, voffl + unsigned(c) * Pszl)) : R(0);
        }
    };
    // row r of the fluxes, transfers and source; a single-iteration launch
    // needs no w or f on its top halo row
    auto load_rest = [&](int r, bool ok) {
        const int64_t o = (int64_t)r * pitch;
        const bool full = ok && (!ALN || r >= i0);
        const auto ru = row_rsrc(a.u_in, o, ok, nb_u);
        const auto rf = row_rsrc(a.f, o, full, nb_phi);
        const auto rw = row_rsrc(a.w_in, o, L > 0 && full, nb_w);
#pragma unroll
        for (int c = 0; c < K; ++c) {
            nux[c] = buf_ld<R>(ru, voff + unsigned(c) * Psz);
            nuy[c] = buf_ld<R>(ru, voff + unsigned(K + c) * Psz);
            nf[c] = buf_ld<R>(rf, voff + unsigned(c) * Psz);
        }
#pragma unroll
        for (int e = 0; e < LA; ++e) nw[e] = (L > 0) ? buf_ld<R>(rw, voff + unsigned(e) * Psz) : R(0);
    };
    auto load_edges_first = [&](int r) {
        nRA = ld_edge(eR, r, a.phi_in, nb_phi, 0, true);
        if (COMP) nRAl = ld_edge_lo(eRl, r, true);
        nLA = ld_edge(eL, r, a.phi_in, nb_phi, 0, true);
        if (COMP) nLAl = ld_edge_lo(eLl, r, true);
        nLB = ld_edge(eL, r + 1, a.phi_in, nb_phi, 0, r + 1 < a.m);
        if (COMP) nLBl = ld_edge_lo(eLl, r + 1, r + 1 < a.m);
        nLux = ld_edge(eL, r, a.u_in, nb_u, 0, true);
        nLuy = ld_edge(eL, r, a.u_in, nb_u, K, true);
    };
    load_phi(rs, true, nA, nAl);
    load_phi(rs + 1, true, nB, nBl);
    load_rest(rs, true);
    if (ALN) load_edges_first(rs);

    // pipeline registers: outputs of stage t on the previous (P) and the
    // current (N) step, and each stage's carry and source term
    R phP[T][K], plP[T][K], phN[T][K], plN[T][K];
    R uxP[T][K], uyP[T][K], wP[T][LA];
    R uxN[T][K], uyN[T][K], wN[T][LA];
    R carry[T][K], fq[T][K];
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
        for (int c = 0; c < K; ++c) {
            phP[t][c] = plP[t][c] = phN[t][c] = plN[t][c] = R(0);
            uxP[t][c] = uyP[t][c] = uxN[t][c] = uyN[t][c] = R(0);
            carry[t][c] = fq[t][c] = R(0);
        }
#pragma unroll
        for (int e = 0; e < LA; ++e) wP[t][e] = wN[t][e] = R(0);
    }

    ChkState<R, K> ck;
#pragma unroll
    for (int c = 0; c < K; ++c) ck.xo[c] = ck.xn[c] = R(0);
#pragma unroll
    for (int q = 0; q < NMET; ++q) ck.col[q] = 0.0;
    ck.qlane = ALN ? 0 : (T & 3);  // the strip's first stored column is on lane T (lane 0 aligned)

    const int nsteps = (re - rs) + T - 1;
    for (int s = 0; s < nsteps; ++s) {
        const int r0 = rs + s;
        Psz = unsigned(P) * unsigned(sizeof(R));
        Pszl = unsigned(P) * 4u;
        asm volatile("" : "+s"(Psz), "+s"(Pszl));
        // current stage-0 inputs
        R cA[K], cAl[K], cB[K], cBl[K], cux[K], cuy[K], cw[LA];
#pragma unroll
        for (int c = 0; c < K; ++c) {
            cA[c] = nA[c];
            cAl[c] = nAl[c];
            cB[c] = nB[c];
            cBl[c] = nBl[c];
            cux[c] = nux[c];
            cuy[c] = nuy[c];
        }
#pragma unroll
        for (int e = 0; e < LA; ++e) cw[e] = nw[e];
#pragma unroll
        for (int t = T - 1; t > 0; --t) {
#pragma unroll
            for (int c = 0; c < K; ++c) fq[t][c] = fq[t - 1][c];
        }
#pragma unroll
        for (int c = 0; c < K; ++c) fq[0][c] = nf[c];
        const R cRA = nRA, cRAl = nRAl, cLA = nLA, cLAl = nLAl, cLB = nLB, cLBl = nLBl, cLux = nLux, cLuy = nLuy;

        // prefetch the next row while this one is computed: issued on every
        // step (zero-length descriptors past the strip's last row), so that
        // no path skips a memory instruction and the waits count exactly
        const bool more = r0 + 1 < re;
#pragma unroll
        for (int c = 0; c < K; ++c) {
            nA[c] = cB[c];
            nAl[c] = cBl[c];
        }
        load_phi(r0 + 2, more, nB, nBl);
        load_rest(r0 + 1, more);
        if (ALN) {
            nRA = ld_edge(eR, r0 + 1, a.phi_in, nb_phi, 0, more);
            if (COMP) nRAl = ld_edge_lo(eRl, r0 + 1, more);
            nLA = cLB;
            nLAl = cLBl;
            nLB = ld_edge(eL, r0 + 2, a.phi_in, nb_phi, 0, more && r0 + 2 < a.m);
            if (COMP) nLBl = ld_edge_lo(eLl, r0 + 2, more && r0 + 2 < a.m);
            nLux = ld_edge(eL, r0 + 1, a.u_in, nb_u, 0, more);
            nLuy = ld_edge(eL, r0 + 1, a.u_in, nb_u, K, more);
        }

#pragma unroll
        for (int t = 0; t < T; ++t) {
            const int r = r0 - t;
            // one iteration per launch: every step is a row of the strip
            if (T == 1 || (r >= rs && r < re)) {
                const bool last_row = (r == a.m - 1);
                const bool st_row = (t == T - 1) && r >= i0 && r < i1;
                const int64_t ro = (int64_t)r * pitch;
                // the last stage of a check launch also takes the check
                constexpr bool CK0 = CHK && T == 1;
                if (t == 0) {
                    Edges<R> E{cRA, cRAl, cLA, cLAl, cLB, cLBl, cLux, cLuy, hasL};
                    stage<R, K, GK, L, LA, COMP, ALN, CK0>(a, lane, jin, last_row, last_col, cA, cAl, cB, cBl, cux,
                                                           cuy, cw, fq[0], E, st_row, ro, soff, P, carry[0], phN[0],
                                                           plN[0], uxN[0], uyN[0], wN[0], ck, r, j);
                } else if (CHK && t == T - 1) {
                    Edges<R> E{R(0), R(0), R(0), R(0), R(0), R(0), R(0), R(0), false};
                    stage<R, K, GK, L, LA, COMP, false, CHK>(a, lane, jin, last_row, last_col, phP[t - 1],
                                                             plP[t - 1], phN[t - 1], plN[t - 1], uxP[t - 1], uyP[t - 1],
                                                             wP[t - 1], fq[t], E, st_row, ro, soff, P, carry[t], phN[t],
                                                             plN[t], uxN[t], uyN[t], wN[t], ck, r, j);
                } else {
                    Edges<R> E{R(0), R(0), R(0), R(0), R(0), R(0), R(0), R(0), false};
                    stage<R, K, GK, L, LA, COMP, false>(a, lane, jin, last_row, last_col, phP[t - 1], plP[t - 1],
                                                        phN[t - 1], plN[t - 1], uxP[t - 1], uyP[t - 1], wP[t - 1],
                                                        fq[t], E, st_row, ro, soff, P, carry[t], phN[t], plN[t], uxN[t], uyN[t],
                                                        wN[t], ck, r, j);
                }
            }
        }
        // rotate: this step's outputs become the next step's inputs
#pragma unroll
        for (int t = 0; t < T; ++t) {
#pragma unroll
            for (int c = 0; c < K; ++c) {
                phP[t][c] = phN[t][c];
                plP[t][c] = plN[t][c];
                uxP[t][c] = uxN[t][c];
                uyP[t][c] = uyN[t][c];
            }
#pragma unroll
            for (int e = 0; e < LA; ++e) wP[t][e] = wN[t][e];
        }
    }
}

}  // namespace dev
}  // namespace omt
