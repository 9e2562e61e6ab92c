// Fused PDHG iteration of the vector-OMT method (Sec. 7.2) on 3-D grids,
// for gfx950.  The paper leaves 3-D imaging as future work (Sec. 8.2); the
// discretisation is App. A's along each of the three axes: u has three
// components per channel, u_x between i and i+1, u_y between j and j+1, u_z
// between z and z+1, with the ghost components u_x(m-1,.,.), u_y(.,n-1,.),
// u_z(.,.,p-1) zero.
//
// One wavefront owns a register tile of G3_ROWS rows by 64 aligned columns
// and marches it through a chunk of slices along z.  Lanes are columns
// (every access is a coalesced row segment, and every store covers whole
// cache lines).  The two neighbours from outside the tile come from side
// loads in which lane c carries channel c: the potential right of the tile
// (the u_y gradient of lane 63), and, left of it, the potential and flux
// from which the left pixel's flux update is recomputed (the u_y divergence
// of lane 0), with the same expressions as in its own tile.  The tile carries
// one halo row above (its flux update gives the u_x neighbour of the first
// row) and one below (its potential gives the gradient of the last row).
// The u_z neighbour of a slice is the previous slice's, kept in registers; a
// chunk starts one slice early to compute it.  Every pixel is computed by
// the same expressions wherever it sits in a tile, so any tiling gives the
// same iterates bit for bit.

#include <type_traits>

#include "grid3.h"
#include "step_device.h"

namespace omt {
namespace {

using namespace dev;

// Shrink of the flux block of one pixel, (u_x, u_y, u_z) of k channels
// (App. B): per channel on the spatial 3-vector (u norm 0), element-wise
// (1), or one block of all 3k components (2).
template <typename R, int K>
__device__ __forceinline__ void shrink3(int unorm, R (&x)[K], R (&y)[K], R (&z)[K], R t)
{
    if (unorm == 0) {
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const R s = shrink_scale<R>(sqrt(x[c] * x[c] + y[c] * y[c] + z[c] * z[c]), t);
            x[c] = x[c] * s;
            y[c] = y[c] * s;
            z[c] = z[c] * s;
        }
    } else if (unorm == 1) {
#pragma unroll
        for (int c = 0; c < K; ++c) {
            x[c] = x[c] * shrink_scale<R>(fabs(x[c]), t);
            y[c] = y[c] * shrink_scale<R>(fabs(y[c]), t);
            z[c] = z[c] * shrink_scale<R>(fabs(z[c]), t);
        }
    } else {
        R r2 = R(0);
#pragma unroll
        for (int c = 0; c < K; ++c) r2 = r2 + x[c] * x[c];
#pragma unroll
        for (int c = 0; c < K; ++c) r2 = r2 + y[c] * y[c];
#pragma unroll
        for (int c = 0; c < K; ++c) r2 = r2 + z[c] * z[c];
        const R s = shrink_scale<R>(sqrt(r2), t);
#pragma unroll
        for (int c = 0; c < K; ++c) {
            x[c] = x[c] * s;
            y[c] = y[c] * s;
            z[c] = z[c] * s;
        }
    }
}

template <typename R, int K, int GK, int L>
__global__ __launch_bounds__(WAVE *STEP_WAVES_PER_WG) void pdhg_step3_kernel(const Step3Args<R> a)
{
    constexpr int LA = L > 0 ? L : 1;
    constexpr int RT = G3_ROWS;
    const int lane = threadIdx.x & (WAVE - 1);
    const int g = xcd_remap(blockIdx.x, a.nwg) * STEP_WAVES_PER_WG + int(threadIdx.x / WAVE);
    if (g >= a.ncolw * a.nroww * a.nzw) return;  // whole wave leaves; no barriers follow
    const int wc = __builtin_amdgcn_readfirstlane(g % a.ncolw);
    const int wr = __builtin_amdgcn_readfirstlane((g / a.ncolw) % a.nroww);
    const int wz = __builtin_amdgcn_readfirstlane(g / (a.ncolw * a.nroww));

    const int j = wc * G3_COLS + lane;
    const bool jin = j < a.n;
    const bool last_col = j == a.n - 1;
    // side columns: jL left of the tile, jR right of it; lane c < K reads
    // channel c there (plane c), other lanes read nothing
    const int jL = wc * G3_COLS - 1, jR = wc * G3_COLS + G3_COLS;
    const bool hasL = jL >= 0, hasR = jR < a.n;
    const unsigned hcP = unsigned(lane < K ? lane : 0) * unsigned(a.plane);
    const unsigned eL = lane < K && hasL ? (hcP + unsigned(jL)) * unsigned(sizeof(R)) : OFF_NONE;
    const unsigned eR = lane < K && hasR ? (hcP + unsigned(jR)) * unsigned(sizeof(R)) : OFF_NONE;
    const int i0 = wr * RT;
    const int z0 = wz * a.zch, z1 = min(z0 + a.zch, a.p);
    const int zs = max(z0 - 1, 0);
    const int64_t P = a.plane;
    const unsigned Psz = unsigned(P) * unsigned(sizeof(R));
    const unsigned voff = jin ? unsigned(j) * unsigned(sizeof(R)) : OFF_NONE;
    const unsigned soff = voff;  // every lane in the grid stores
    const int nb_phi = field_bytes(K, P, a.n, sizeof(R)), nb_u = field_bytes(3 * K, P, a.n, sizeof(R));
    const int nb_w = field_bytes(a.l, P, a.n, sizeof(R));
    auto roff = [&](int z, int i) -> int64_t { return ((int64_t)z * a.m + i) * a.pitch; };
    auto row_ok = [&](int i) { return i >= 0 && i < a.m; };

    // potential of the current slice and of the next, rows i0 - 1 .. i0 + RT
    R pc[RT + 2][K], pn[RT + 2][K];
    R carry[RT][K];  // 2 u_z' - u_z of the previous slice, tile rows
    // fluxes (rows i0 - 1 .. i0 + RT - 1), transfers and source (tile rows)
    // of the current slice
    R ux[RT + 1][K], uy[RT + 1][K], uz[RT + 1][K];
    R wv[RT][LA], fv[RT][K];
    // side values (lane c: channel c): the potential left and right of the
    // tile on the current and the next slice, and the flux left of it
    R eLc[RT + 2], eLn[RT + 2], eRc[RT + 2], eRn[RT + 2];
    R eUx[RT + 1], eUy[RT + 1], eUz[RT + 1];
#pragma unroll
    for (int q = 0; q < RT; ++q)
#pragma unroll
        for (int c = 0; c < K; ++c) carry[q][c] = R(0);
    // loads of one row of a slice; ok = false gives a zero-length
    // descriptor (zeros, no memory access)
    auto ld_phi = [&](R (&dst)[K], R &dl, R &dr, int z, int i, bool ok) {
        const auto rp = row_rsrc(a.phi_in, roff(z, i), ok && row_ok(i) && z < a.p, nb_phi);
#pragma unroll
        for (int c = 0; c < K; ++c) dst[c] = buf_ld<R>(rp, voff + unsigned(c) * Psz);
        dl = buf_ld<R>(rp, eL);
        dr = buf_ld<R>(rp, eR);
    };
    auto ld_u = [&](int q, int z, bool ok) {
        const int i = i0 - 1 + q;
        const auto ru = row_rsrc(a.u_in, roff(z, i), ok && row_ok(i), nb_u);
#pragma unroll
        for (int c = 0; c < K; ++c) {
            ux[q][c] = buf_ld<R>(ru, voff + unsigned(c) * Psz);
            uy[q][c] = buf_ld<R>(ru, voff + unsigned(K + c) * Psz);
            uz[q][c] = buf_ld<R>(ru, voff + unsigned(2 * K + c) * Psz);
        }
        eUx[q] = buf_ld<R>(ru, eL);
        eUy[q] = buf_ld<R>(ru, eL + unsigned(K) * Psz);
        eUz[q] = buf_ld<R>(ru, eL + unsigned(2 * K) * Psz);
    };
    auto ld_wf = [&](int r, int z, bool ok) {
        const int i = i0 + r;
        ok = ok && row_ok(i);
        const auto rw = row_rsrc(a.w_in, roff(z, i), ok && L > 0, nb_w);
        const auto rf = row_rsrc(a.f, roff(z, i), ok, nb_phi);
#pragma unroll
        for (int e = 0; e < LA; ++e) wv[r][e] = L > 0 ? buf_ld<R>(rw, soff + unsigned(e) * Psz) : R(0);
#pragma unroll
        for (int c = 0; c < K; ++c) fv[r][c] = buf_ld<R>(rf, voff + unsigned(c) * Psz);
    };
    // the first slice: its potential, the next slice's, its fluxes, and
    // (if the wave stores it) its transfers and source
#pragma unroll
    for (int q = 0; q < RT + 2; ++q) ld_phi(pc[q], eLc[q], eRc[q], zs, i0 - 1 + q, true);
#pragma unroll
    for (int q = 0; q < RT + 2; ++q) ld_phi(pn[q], eLn[q], eRn[q], zs + 1, i0 - 1 + q, true);
#pragma unroll
    for (int q = 0; q < RT + 1; ++q) ld_u(q, zs, true);
#pragma unroll
    for (int r = 0; r < RT; ++r) ld_wf(r, zs, zs >= z0);

    for (int z = zs; z < z1; ++z) {
        const bool inner = z >= z0;  // a slice this wave stores (else the halo slice)
        const bool zlast = z == a.p - 1;
        // the next slice is loaded row by row as this one frees its
        // registers, so its loads are in flight while this slice computes
        const bool more = z + 1 < z1;
        R ubxp[K];  // 2 u_x' - u_x of the row above
#pragma unroll
        for (int c = 0; c < K; ++c) ubxp[c] = R(0);
#pragma unroll
        for (int q = 0; q < RT + 1; ++q) {
            const int i = i0 - 1 + q;
            const bool rin = row_ok(i);
            const bool lane_ok = jin && rin;
            const bool last_row = i == a.m - 1;
            // u-update: shrink_u(u + mu grad phi, mu), ghosts zero
            R tx[K], ty[K], tz[K];
#pragma unroll
            for (int c = 0; c < K; ++c) {
                R pr = lane_next(pc[q][c]);
                if (lane == WAVE - 1) pr = lane_get(eRc[q], c);
                tx[c] = last_row ? R(0) : ux[q][c] + a.mu_h * (pc[q + 1][c] - pc[q][c]);
                ty[c] = last_col ? R(0) : uy[q][c] + a.mu_h * (pr - pc[q][c]);
                tz[c] = zlast ? R(0) : uz[q][c] + a.mu_h * (pn[q][c] - pc[q][c]);
            }
            shrink3<R, K>(a.unorm, tx, ty, tz, a.mu);
            R ubx[K], uby[K], ubz[K];
#pragma unroll
            for (int c = 0; c < K; ++c) {
                tx[c] = lane_ok ? tx[c] * a.ureg : R(0);
                ty[c] = lane_ok ? ty[c] * a.ureg : R(0);
                tz[c] = lane_ok ? tz[c] * a.ureg : R(0);
                ubx[c] = R(2) * tx[c] - ux[q][c];
                uby[c] = R(2) * ty[c] - uy[q][c];
                ubz[c] = R(2) * tz[c] - uz[q][c];
            }
            if (q >= 1) {
                const int r = q - 1;
                if (inner) {
                    // the pixel left of the tile: its flux update, as in
                    // its own tile, for the u_y divergence of lane 0
                    R lb[K];
                    {
                        R ex[K], ey[K], ez[K];
#pragma unroll
                        for (int c = 0; c < K; ++c) {
                            const R hA = lane_get(eLc[q], c), hB = lane_get(eLc[q + 1], c);
                            const R hZ = lane_get(eLn[q], c), hR = lane_get(pc[q][c], 0);
                            ex[c] = last_row ? R(0) : lane_get(eUx[q], c) + a.mu_h * (hB - hA);
                            ey[c] = lane_get(eUy[q], c) + a.mu_h * (hR - hA);  // never the last column
                            ez[c] = zlast ? R(0) : lane_get(eUz[q], c) + a.mu_h * (hZ - hA);
                        }
                        shrink3<R, K>(a.unorm, ex, ey, ez, a.mu);
#pragma unroll
                        for (int c = 0; c < K; ++c) {
                            const R yl = hasL ? ey[c] * a.ureg : R(0);
                            lb[c] = R(2) * yl - (hasL ? lane_get(eUy[q], c) : R(0));
                        }
                    }
                    const bool st = rin;
                    const int64_t ro = roff(z, i);
                    const auto rphi = row_rsrc(a.phi_out, ro, st, nb_phi);
                    const auto ruo = row_rsrc(a.u_out, ro, st, nb_u);
                    const auto rwo = row_rsrc(a.w_out, ro, st && L > 0, nb_w);
                    // w-update: shrink_w(w + nu grad_G phi, alpha nu), Sec. 3.1
                    R wb[LA];
                    if constexpr (L > 0) {
                        R wt[LA];
#pragma unroll
                        for (int e = 0; e < LA; ++e) {
                            if constexpr (GK == G_DENSE) {
                                R s = R(0);
#pragma unroll
                                for (int c = 0; c < K; ++c) s = s + a.gm[c * LMAX + e] * pc[q][c];
                                wt[e] = (e < a.l) ? wv[r][e] + a.nu * s : R(0);
                            } else {
                                const int ea = edge_a<GK, K>(e), eb = edge_b<GK, K>(e);
                                wt[e] = wv[r][e] + a.nu * ((pc[q][ea] - pc[q][eb]) * a.ic[e]);
                            }
                        }
                        shrink_w<R, LA>(a.wnorm, wt, a.anu);
#pragma unroll
                        for (int e = 0; e < LA; ++e) {
                            wt[e] = lane_ok ? wt[e] * a.wreg : R(0);
                            wb[e] = R(2) * wt[e] - wv[r][e];
                            buf_st<R>(rwo, soff + unsigned(e) * Psz, wt[e]);
                        }
                    }
                    // phi-update: phi + tau (div_x u_bar + div_G w_bar + f)
#pragma unroll
                    for (int c = 0; c < K; ++c) {
                        R ubl = lane_prev(uby[c]);
                        if (lane == 0) ubl = lb[c];
                        const R dx = ((((ubx[c] - ubxp[c]) + uby[c]) - ubl) + (ubz[c] - carry[r][c])) * a.inv_h;
                        R dg = R(0);
                        if constexpr (L > 0) {
#pragma unroll
                            for (int e = 0; e < LA; ++e) {
                                if constexpr (GK == G_DENSE) {
                                    dg = dg + a.gm[c * LMAX + e] * wb[e];
                                } else {
                                    if (edge_a<GK, K>(e) == c) dg = dg + a.ic[e] * wb[e];
                                    if (edge_b<GK, K>(e) == c) dg = dg - a.ic[e] * wb[e];
                                }
                            }
                        }
                        const R po = lane_ok ? pc[q][c] + a.tau * ((dx - dg) + fv[r][c]) : R(0);
                        buf_st<R>(rphi, soff + unsigned(c) * Psz, po);
                        buf_st<R>(ruo, soff + unsigned(c) * Psz, tx[c]);
                        buf_st<R>(ruo, soff + unsigned(K + c) * Psz, ty[c]);
                        buf_st<R>(ruo, soff + unsigned(2 * K + c) * Psz, tz[c]);
                    }
                }
#pragma unroll
                for (int c = 0; c < K; ++c) carry[r][c] = ubz[c];
            }
#pragma unroll
            for (int c = 0; c < K; ++c) ubxp[c] = ubx[c];
            // row q of this slice is done with its flux, potential and
            // (row q - 1) transfer and source: load the next slice's
            ld_u(q, z + 1, more);
            if (q >= 1) ld_wf(q - 1, z + 1, more);
#pragma unroll
            for (int c = 0; c < K; ++c) pc[q][c] = pn[q][c];
            eLc[q] = eLn[q];
            eRc[q] = eRn[q];
            ld_phi(pn[q], eLn[q], eRn[q], z + 2, i0 - 1 + q, more);
        }
#pragma unroll
        for (int c = 0; c < K; ++c) pc[RT + 1][c] = pn[RT + 1][c];
        eLc[RT + 1] = eLn[RT + 1];
        eRc[RT + 1] = eRn[RT + 1];
        ld_phi(pn[RT + 1], eLn[RT + 1], eRn[RT + 1], z + 2, i0 + RT, more);
    }
}

// ------------------------------------------------------------- the check

// div_G of w' - w (dgd) and of w' (dg1) at channel c: D diag(1/c) applied
// to the transfers, in edge order (div_G is its negative, Sec. 3.1).
template <typename R, int K, int GK, int LA>
__device__ __forceinline__ void graph_div3(const Step3Args<R> &a, int c, const double (&we0)[LA],
                                           const double (&we1)[LA], double &dgd, double &dg1)
{
    dgd = 0.0;
    dg1 = 0.0;
#pragma unroll
    for (int e = 0; e < LA; ++e) {
        if constexpr (GK == G_DENSE) {
            dgd += double(a.gm[c * LMAX + e]) * (we1[e] - we0[e]);
            dg1 += double(a.gm[c * LMAX + e]) * we1[e];
        } else {
            if (edge_a<GK, K>(e) == c) {
                dgd += double(a.ic[e]) * (we1[e] - we0[e]);
                dg1 += double(a.ic[e]) * we1[e];
            }
            if (edge_b<GK, K>(e) == c) {
                dgd -= double(a.ic[e]) * (we1[e] - we0[e]);
                dg1 -= double(a.ic[e]) * we1[e];
            }
        }
    }
}

// Check terms (Sec. 6.1 R^k with 1/nu on the w block, App. A objectives,
// constraint residual) of one tile: 64 aligned columns by MET_ROWS rows of
// one slice; every lane adds its column row by row, lanes past the grid
// add nothing.
template <typename R, int K, int GK, int L>
__global__ __launch_bounds__(WAVE *STEP_WAVES_PER_WG) void tile_metrics3_kernel(const Step3Args<R> a, double alpha,
                                                                                 double eps, int ncolw, int ntiles,
                                                                                 double *partials)
{
    constexpr int LA = L > 0 ? L : 1;
    const int lane = threadIdx.x & (WAVE - 1);
    const int t = blockIdx.x * STEP_WAVES_PER_WG + __builtin_amdgcn_readfirstlane(int(threadIdx.x / WAVE));
    if (t >= ntiles) return;
    const int nrt = (a.m + MET_ROWS - 1) / MET_ROWS;
    const int wc = t % ncolw, wr = (t / ncolw) % nrt, z = t / (ncolw * nrt);
    const int j = wc * WAVE + lane;
    const bool jok = j < a.n;
    const int i0 = wr * MET_ROWS, i1 = min(i0 + MET_ROWS, a.m);
    const int64_t P = a.plane;
    const double inv_h = double(a.inv_h);
    const R *phi0 = a.phi_in, *phi1 = a.phi_out, *u0 = a.u_in, *u1 = a.u_out, *w0 = a.w_in, *w1 = a.w_out;
    double v[NMET];
#pragma unroll
    for (int q = 0; q < NMET; ++q) v[q] = 0.0;
    for (int i = i0; i < i1; ++i) {
        // every lane reads in-bounds addresses (column j < pitch); lanes past
        // the grid drop their terms
        const int64_t o = ((int64_t)z * a.m + i) * a.pitch + j;
        const int64_t oi = i > 0 ? o - a.pitch : o, oj = j > 0 ? o - 1 : o;
        const int64_t oz = z > 0 ? o - (int64_t)a.m * a.pitch : o;
        double acc[NMET];
#pragma unroll
        for (int q = 0; q < NMET; ++q) acc[q] = 0.0;
        // every load is issued unconditionally (the addresses are clamped
        // into the field), so they all can be in flight at once; ghost and
        // outside neighbours are zeroed afterwards
        double we0[LA], we1[LA];
#pragma unroll
        for (int e = 0; e < LA; ++e) {
            we0[e] = we1[e] = 0.0;
            if constexpr (L > 0) {
                // a type compiled for more edges than in use reads plane 0
                // again for the missing ones and drops it
                const bool on = e < a.l;
                const int64_t oe = on ? e * P + o : o;
                const double v0 = double(ld_field(&w0[oe])), v1 = double(ld_field(&w1[oe]));
                we0[e] = on ? v0 : 0.0;
                we1[e] = on ? v1 : 0.0;
            }
        }
        double u2 = 0.0, sq = 0.0;
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const double p0 = double(ld_field(&phi0[c * P + o])), p1 = double(ld_field(&phi1[c * P + o]));
            const double lx0 = double(ld_field(&u0[c * P + o])), lx1 = double(ld_field(&u1[c * P + o]));
            const double ly0 = double(ld_field(&u0[(K + c) * P + o])), ly1 = double(ld_field(&u1[(K + c) * P + o]));
            const double lz0 = double(ld_field(&u0[(2 * K + c) * P + o]));
            const double lz1 = double(ld_field(&u1[(2 * K + c) * P + o]));
            const double lxl0 = double(ld_field(&u0[c * P + oi])), lxl1 = double(ld_field(&u1[c * P + oi]));
            const double lyl0 = double(ld_field(&u0[(K + c) * P + oj]));
            const double lyl1 = double(ld_field(&u1[(K + c) * P + oj]));
            const double lzl0 = double(ld_field(&u0[(2 * K + c) * P + oz]));
            const double lzl1 = double(ld_field(&u1[(2 * K + c) * P + oz]));
            const double ux0 = i < a.m - 1 ? lx0 : 0.0, ux1 = i < a.m - 1 ? lx1 : 0.0;
            const double uy0 = j < a.n - 1 ? ly0 : 0.0, uy1 = j < a.n - 1 ? ly1 : 0.0;
            const double uz0 = z < a.p - 1 ? lz0 : 0.0, uz1 = z < a.p - 1 ? lz1 : 0.0;
            const double xl0 = i > 0 ? lxl0 : 0.0, xl1 = i > 0 ? lxl1 : 0.0;
            const double yl0 = j > 0 ? lyl0 : 0.0, yl1 = j > 0 ? lyl1 : 0.0;
            const double zl0 = z > 0 ? lzl0 : 0.0, zl1 = z > 0 ? lzl1 : 0.0;
            double dgd = 0.0, dg1 = 0.0;
            if constexpr (L > 0) graph_div3<R, K, GK, LA>(a, c, we0, we1, dgd, dg1);
            const double fc = double(ld_field(&a.f[c * P + o]));
            const double dp = p1 - p0;
            const double dux = ux1 - ux0, duy = uy1 - uy0, duz = uz1 - uz0;
            const double ddiv = (((dux - (xl1 - xl0)) + duy - (yl1 - yl0)) + duz - (zl1 - zl0)) * inv_h;
            const double div1 = (((ux1 - xl1) + uy1 - yl1) + uz1 - zl1) * inv_h;
            acc[0] += dux * dux + duy * duy + duz * duz;
            acc[2] += dp * dp;
            acc[3] += dp * (ddiv - dgd);
            acc[5] += p1 * fc;
            const double rr = (div1 - dg1) + fc;
            acc[6] += rr * rr;
            acc[7] += p1;
            sq += ux1 * ux1 + uy1 * uy1 + uz1 * uz1;
            if (a.unorm == 0)
                acc[4] += sqrt(ux1 * ux1 + uy1 * uy1 + uz1 * uz1);
            else if (a.unorm == 1)
                acc[4] += fabs(ux1) + fabs(uy1) + fabs(uz1);
            else
                u2 += ux1 * ux1 + uy1 * uy1 + uz1 * uz1;
        }
        pixel_terms<LA>(acc, sq, u2, a.unorm, a.wnorm, alpha, eps, L > 0 ? a.l : 0, we0, we1);
#pragma unroll
        for (int q = 0; q < NMET; ++q) v[q] += jok ? acc[q] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NMET; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) partials[(int64_t)t * NMET + q] = s;
    }
}

template <typename R, int K, int GK, int L>
hipError_t launch3(const void *args, hipStream_t s)
{
    const Step3Args<R> &a = *static_cast<const Step3Args<R> *>(args);
    hipLaunchKernelGGL((pdhg_step3_kernel<R, K, GK, L>), dim3(a.nwg), dim3(WAVE * STEP_WAVES_PER_WG), 0, s, a);
    return hipGetLastError();
}

template <typename R, int K, int GK, int L>
hipError_t met3(const Metrics3Launch &Lc)
{
    const Step3Args<R> &a = *static_cast<const Step3Args<R> *>(Lc.args);
    const int nb = (Lc.ntiles + STEP_WAVES_PER_WG - 1) / STEP_WAVES_PER_WG;
    hipLaunchKernelGGL((tile_metrics3_kernel<R, K, GK, L>), dim3(nb), dim3(WAVE * STEP_WAVES_PER_WG), 0, Lc.stream, a,
                       Lc.alpha, Lc.eps, Lc.ncolw, Lc.ntiles, Lc.partials);
    return hipGetLastError();
}

// Compiled problem types on 3-D grids: k = 1 without edges, k = 2 with one
// edge, k = 3 on the path, the triangle or another graph of up to 3 edges.
template <typename F>
hipError_t by_type(int dtype, int k, int gk, int lb, F &&f)
{
    if (k == 1 && gk == G_NONE && lb == 0) return f(std::integral_constant<int, 0>{});
    if (k == 2 && gk == G_PATH && lb == 1) return f(std::integral_constant<int, 1>{});
    if (k == 3 && gk == G_PATH && lb == 2) return f(std::integral_constant<int, 2>{});
    if (k == 3 && gk == G_COMPLETE && lb == 3) return f(std::integral_constant<int, 3>{});
    if (k == 3 && gk == G_DENSE && lb == 2) return f(std::integral_constant<int, 4>{});
    if (k == 3 && gk == G_DENSE && lb == 3) return f(std::integral_constant<int, 5>{});
    (void)dtype;
    return hipErrorInvalidValue;
}

}  // namespace

bool step3_supported(int dtype, int k, int gk, int lb)
{
    return (dtype == 0 || dtype == 1) &&
           by_type(dtype, k, gk, lb, [](auto) { return hipSuccess; }) == hipSuccess;
}

hipError_t launch_step3(int dtype, int k, int gk, int lb, const void *args, hipStream_t stream)
{
    return by_type(dtype, k, gk, lb, [&](auto ty) -> hipError_t {
        constexpr int T = decltype(ty)::value;
        constexpr int K = T == 0 ? 1 : T == 1 ? 2 : 3;
        constexpr int GK = T == 0 ? G_NONE : (T == 1 || T == 2) ? G_PATH : T == 3 ? G_COMPLETE : G_DENSE;
        constexpr int L = T == 0 ? 0 : T == 1 ? 1 : T == 2 ? 2 : T == 3 ? 3 : T == 4 ? 2 : 3;
        return dtype == 1 ? launch3<double, K, GK, L>(args, stream) : launch3<float, K, GK, L>(args, stream);
    });
}

hipError_t launch_metrics3(const Metrics3Launch &Lc)
{
    return by_type(Lc.dtype, Lc.k, Lc.gk, Lc.lb, [&](auto ty) -> hipError_t {
        constexpr int T = decltype(ty)::value;
        constexpr int K = T == 0 ? 1 : T == 1 ? 2 : 3;
        constexpr int GK = T == 0 ? G_NONE : (T == 1 || T == 2) ? G_PATH : T == 3 ? G_COMPLETE : G_DENSE;
        constexpr int L = T == 0 ? 0 : T == 1 ? 1 : T == 2 ? 2 : T == 3 ? 3 : T == 4 ? 2 : 3;
        return Lc.dtype == 1 ? met3<double, K, GK, L>(Lc) : met3<float, K, GK, L>(Lc);
    });
}

}  // namespace omt
