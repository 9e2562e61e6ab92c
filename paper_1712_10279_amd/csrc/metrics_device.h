// Device code of the check-iteration metrics, shared by the per-problem
// solve and the persistent batched kernel so that both take identical
// stopping decisions.
//
// For one step (u, w, phi) -> (u', w', phi') every pixel contributes, in
// FP64 (Sec. 6.1 fixed-point residual with 1/nu on the w block, App. A
// objectives):
//   v[0] = |u' - u|^2             v[1] = |w' - w|^2        v[2] = |phi' - phi|^2
//   v[3] = <phi' - phi, div_x(u' - u) + div_G(w' - w)>
//   v[4] = ||u'||_u + alpha ||w'||_w (+ eps (|u'|^2 + |w'|^2))  (primal objective)
//   v[5] = <phi', f>                                         (dual objective)
//   v[6] = |div_x u' + div_G w' + f|^2                       (constraint residual)
//   v[7] = sum of phi'
// The terms of a pixel are formed by chan_terms / pixel_terms (step_device.h)
// in a fixed order.  A tile is 64 aligned columns by MET_ROWS rows: each lane
// adds its column's pixels row by row, the wave adds its lanes with
// wave_sum (neighbours first), and a single wave adds the tiles of a problem
// in tile order.  A check fused into a single-iteration step launch forms
// the same column and quad sums in registers and quads_to_tiles the same
// tiles, so both ways of taking a check give identical values.
#pragma once

#include "step_device.h"

namespace omt {
namespace dev {


// sum_g wt_g ||x_g||_2 of a grouped entry-wise norm (see group_scales)
template <int N, typename W>
__device__ __forceinline__ double group_norm(const W *wt, const double (&x)[N])
{
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        if (wt[c] > W(0)) {
            const bool pair = (c + 1 < N) && wt[c + 1] == W(0);
            const double r = pair ? sqrt(x[c] * x[c] + x[c + 1] * x[c + 1]) : fabs(x[c]);
            s += double(wt[c]) * r;
        }
    }
    return s;
}

template <typename R, int K, int GK, int L, bool COMP>
__device__ __forceinline__ void tile_metrics(const StepArgs<R> &a, int wc, int wr, int lane, double (&v)[NMET])
{
    constexpr int LA = L > 0 ? L : 1;
#pragma unroll
    for (int q = 0; q < NMET; ++q) v[q] = 0.0;
    // Tiles are 64-column aligned, so every lane's column is inside the
    // padded pitch: all lanes load (unconditionally, from in-bounds
    // addresses) and lanes past the grid add nothing.
    constexpr int MET_CH_UNROLL = 2;
    const int j = wc * WAVE + lane;
    const bool jok = j < a.n;
    const int i0 = wr * MET_ROWS, i1 = min(i0 + MET_ROWS, a.m);
    const int64_t P = a.plane;
    const R *phi0 = a.phi_in, *phi1 = a.phi_out, *u0 = a.u_in, *u1 = a.u_out, *w0 = a.w_in, *w1 = a.w_out;
    const double inv_h = double(a.inv_h);
    for (int i = i0; i < i1; ++i) {
        const int64_t o = (int64_t)i * a.pitch + j;
        const int64_t oi = i > 0 ? o - a.pitch : o, oj = j > 0 ? o - 1 : o;
        double acc[NMET];
#pragma unroll
        for (int q = 0; q < NMET; ++q) acc[q] = 0.0;
        double we0[LA], we1[LA];
#pragma unroll
        for (int e = 0; e < LA; ++e) {
            const bool on = L > 0 && e < a.l;
            we0[e] = on ? double(ld_field(&w0[e * P + o])) : 0.0;
            we1[e] = on ? double(ld_field(&w1[e * P + o])) : 0.0;
        }
        double u2 = 0.0, sq = 0.0;
        // grouped entry-wise norm of the matrix kinds, accumulated channel by
        // channel: an open two-coordinate group keeps its first squares and
        // its weight until its second coordinate arrives
        double gpx = 0.0, gpy = 0.0, gw = 0.0;
        // two channels at a time keep the live registers (and so the resident
        // waves) in check
#pragma unroll MET_CH_UNROLL
        for (int c = 0; c < K; ++c) {
            double p0 = double(ld_field(&phi0[c * P + o])), p1 = double(ld_field(&phi1[c * P + o]));
            if (COMP) {
                p0 += double(ld_field(&a.plo_in[c * P + o]));
                p1 += double(ld_field(&a.plo_out[c * P + o]));
            }
            const double lx0 = double(ld_field(&u0[c * P + o])), lx1 = double(ld_field(&u1[c * P + o]));
            const double ly0 = double(ld_field(&u0[(K + c) * P + o])), ly1 = double(ld_field(&u1[(K + c) * P + o]));
            const double lxl0 = double(ld_field(&u0[c * P + oi])), lxl1 = double(ld_field(&u1[c * P + oi]));
            const double lyl0 = double(ld_field(&u0[(K + c) * P + oj]));
            const double lyl1 = double(ld_field(&u1[(K + c) * P + oj]));
            const double ux0 = i < a.m - 1 ? lx0 : 0.0, ux1 = i < a.m - 1 ? lx1 : 0.0;
            const double uy0 = j < a.n - 1 ? ly0 : 0.0, uy1 = j < a.n - 1 ? ly1 : 0.0;
            const double xl0 = i > 0 ? lxl0 : 0.0, xl1 = i > 0 ? lxl1 : 0.0;
            const double yl0 = j > 0 ? lyl0 : 0.0, yl1 = j > 0 ? lyl1 : 0.0;
            double dgd = 0.0, dg1 = 0.0;
            if constexpr (L > 0) graph_div_terms<R, K, GK, LA>(a, c, we0, we1, dgd, dg1);
            const double fc = double(ld_field(&a.f[c * P + o]));
            chan_terms(acc, sq, u2, a.unorm, inv_h, p0, p1, ux0, ux1, uy0, uy1, xl0, xl1, yl0, yl1, dgd, dg1, fc);
            if constexpr (is_matrix_kind(GK)) {
                if (a.unorm == 3) {
                    const double wc = double(a.uwt[c]);
                    if (wc > 0.0) {
                        const bool pair = (c + 1 < K) && a.uwt[c + 1] == R(0);
                        if (pair) {
                            gpx = ux1 * ux1;
                            gpy = uy1 * uy1;
                            gw = wc;
                        } else {
                            acc[4] += wc * (fabs(ux1) + fabs(uy1));
                        }
                    } else {
                        acc[4] += gw * (sqrt(gpx + ux1 * ux1) + sqrt(gpy + uy1 * uy1));
                    }
                }
            }
        }
        if constexpr (is_matrix_kind(GK)) {
            if (a.unorm == 2) acc[4] += sqrt(u2);
            if constexpr (GK == G_MATNUC) {
                if (a.unorm == 4) {  // nuclear norm of each direction of u'
                    double cx[K], cy[K];
#pragma unroll
                    for (int c = 0; c < K; ++c) {
                        const double vx = double(ld_field(&u1[c * P + o])), vy = double(ld_field(&u1[(K + c) * P + o]));
                        cx[c] = i < a.m - 1 ? vx : 0.0;
                        cy[c] = j < a.n - 1 ? vy : 0.0;
                    }
                    acc[4] += herm_nuc<double, K>(cx) + herm_nuc<double, K>(cy);
                }
            }
            double wn = 0.0, w2 = 0.0;
#pragma unroll
            for (int e = 0; e < LA; ++e) {
                acc[1] += (we1[e] - we0[e]) * (we1[e] - we0[e]);
                wn += fabs(we1[e]);
                w2 += we1[e] * we1[e];
            }
            if (a.wnorm == 2)
                acc[4] += a.alpha * group_norm<LA>(a.wwt, we1);
            else if (GK == G_MATNUC && a.wnorm == 3)
                acc[4] += a.alpha * skew_nuc<K, LA>(we1, a.l);
            else
                acc[4] += a.alpha * (a.wnorm == 0 ? wn : sqrt(w2));
            if (a.eps > 0.0) acc[4] += a.eps * (sq + w2);
        } else {
            pixel_terms<LA>(acc, sq, u2, a.unorm, a.wnorm, a.alpha, a.eps, L > 0 ? a.l : 0, we0, we1);
        }
        // lanes past the grid add nothing (their terms are dropped as a whole)
#pragma unroll
        for (int q = 0; q < NMET; ++q) v[q] += jok ? acc[q] : 0.0;
    }
}

// One wave: out[q] = sum over tiles t0..t0+nt-1 of partials[t][q], in a fixed
// order (lane l takes tiles l, l+64, ...; then the wave tree).
__device__ __forceinline__ void reduce_tiles(const double *partials, int t0, int nt, int lane, double *out)
{
    // all NMET sums advance together (one pass over the tiles, the loads of
    // a tile's row independent of each other); each sum still adds its
    // tiles in increasing order, so the result does not depend on this
    double s[NMET];
#pragma unroll
    for (int q = 0; q < NMET; ++q) s[q] = 0.0;
    // unrolled so that the loads of several tiles are in flight at once;
    // every sum still takes its tiles one after another in increasing order
#pragma unroll 4
    for (int t = lane; t < nt; t += WAVE) {
        const double *row = partials + (int64_t)(t0 + t) * NMET;
#pragma unroll
        for (int q = 0; q < NMET; ++q) s[q] += row[q];
    }
#pragma unroll
    for (int q = 0; q < NMET; ++q) {
        const double v = wave_sum(s[q]);
        if (lane == 0) out[q] = v;
    }
}

}  // namespace dev
}  // namespace omt
