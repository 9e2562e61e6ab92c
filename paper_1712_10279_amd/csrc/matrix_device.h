// Device code of the nuclear-norm shrinks of the matrix method (App. B), on
// the orthonormal coordinates the kernels carry: a Hermitian k x k matrix X
// is (X_aa; sqrt2 Re X_ab, sqrt2 Im X_ab for a < b), a skew-Hermitian N is
// (Im N_aa; the same pairs); real symmetric / skew matrices drop the
// imaginary parts.  The nuclear shrink of a Hermitian X soft-thresholds the
// moduli of its eigenvalues and keeps their signs; that of a skew-Hermitian
// N is -i times the shrink of the Hermitian iN.
#pragma once

#include "omt_kernels.h"

namespace omt {
namespace dev {

// coordinates of one transfer matrix W_s for K coordinates of the potential
template <int K>
constexpr int skew_coords()
{
    return K == 3 ? 1 : K == 4 ? 4 : K == 6 ? 3 : K == 9 ? 9 : 0;
}

template <typename R>
__device__ __forceinline__ R soft(R lam, R t)
{
    const R r = fabs(lam) - t;
    return r > R(0) ? (lam > R(0) ? r : -r) : R(0);
}

// Hermitian 2 x 2 from (d0, d1, p, q) = (X_00, X_11, sqrt2 Re X_01, sqrt2 Im X_01):
// X = a I + (X - a I) with eigenvalues a +- r, r = |X - a I|_2; the spectral
// function g maps X to (g(a+r) + g(a-r))/2 I + (g(a+r) - g(a-r))/(2r) (X - a I).
template <typename R>
__device__ __forceinline__ void herm2_shrink(R &d0, R &d1, R &p, R &q, R t)
{
    const R a = (d0 + d1) * R(0.5), dl = (d0 - d1) * R(0.5);
    const R r = sqrt(dl * dl + (p * p + q * q) * R(0.5));
    const R gp = soft(a + r, t), gm = soft(a - r, t);
    const R al = (gp + gm) * R(0.5);
    const R be = r > R(0) ? (gp - gm) * R(0.5) / r : R(0);
    d0 = al + be * dl;
    d1 = al - be * dl;
    p = be * p;
    q = be * q;
}

template <typename R>
__device__ __forceinline__ R herm2_nuc(R d0, R d1, R p, R q)
{
    const R a = (d0 + d1) * R(0.5), dl = (d0 - d1) * R(0.5);
    const R r = sqrt(dl * dl + (p * p + q * q) * R(0.5));
    return fabs(a + r) + fabs(a - r);
}

// Real symmetric 3 x 3 by cyclic Jacobi (a fixed number of sweeps, enough
// for the working precision): A = V diag(lam) V^T.
template <typename R>
__device__ __forceinline__ void sym3_eig(const R (&c)[6], R (&lam)[3], R (&V)[3][3])
{
    constexpr int SWEEPS = sizeof(R) == 8 ? 8 : 6;
    const R ir2 = R(0.70710678118654752440);
    R A[3][3] = {{c[0], c[3] * ir2, c[4] * ir2}, {c[3] * ir2, c[1], c[5] * ir2}, {c[4] * ir2, c[5] * ir2, c[2]}};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? R(1) : R(0);
#pragma unroll
    for (int sw = 0; sw < SWEEPS; ++sw) {
#pragma unroll
        for (int pq = 0; pq < 3; ++pq) {
            const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
            const R apq = A[p][q];
            const bool z = apq == R(0);
            const R th = (A[q][q] - A[p][p]) / (R(2) * (z ? R(1) : apq));
            const R tt = (th >= R(0) ? R(1) : R(-1)) / (fabs(th) + sqrt(th * th + R(1)));
            const R t = z ? R(0) : tt;
            const R cs = R(1) / sqrt(t * t + R(1)), sn = t * cs;
#pragma unroll
            for (int r = 0; r < 3; ++r) {  // A <- A J
                const R arp = A[r][p], arq = A[r][q];
                A[r][p] = cs * arp - sn * arq;
                A[r][q] = sn * arp + cs * arq;
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) {  // A <- J^T A
                const R apr = A[p][r], aqr = A[q][r];
                A[p][r] = cs * apr - sn * aqr;
                A[q][r] = sn * apr + cs * aqr;
            }
#pragma unroll
            for (int r = 0; r < 3; ++r) {  // V <- V J
                const R vrp = V[r][p], vrq = V[r][q];
                V[r][p] = cs * vrp - sn * vrq;
                V[r][q] = sn * vrp + cs * vrq;
            }
        }
    }
    lam[0] = A[0][0];
    lam[1] = A[1][1];
    lam[2] = A[2][2];
}

template <typename R>
__device__ __forceinline__ void sym3_shrink(R (&c)[6], R t)
{
    R lam[3], V[3][3];
    sym3_eig<R>(c, lam, V);
    const R g[3] = {soft(lam[0], t), soft(lam[1], t), soft(lam[2], t)};
    const R r2 = R(1.4142135623730950488);
    auto f = [&](int a, int b) { return V[a][0] * g[0] * V[b][0] + V[a][1] * g[1] * V[b][1] + V[a][2] * g[2] * V[b][2]; };
    c[0] = f(0, 0);
    c[1] = f(1, 1);
    c[2] = f(2, 2);
    c[3] = r2 * f(0, 1);
    c[4] = r2 * f(0, 2);
    c[5] = r2 * f(1, 2);
}

template <typename R>
__device__ __forceinline__ R sym3_nuc(const R (&c)[6])
{
    R lam[3], V[3][3];
    sym3_eig<R>(c, lam, V);
    return fabs(lam[0]) + fabs(lam[1]) + fabs(lam[2]);
}

// Nuclear shrink of one Hermitian matrix given by its K coordinates
// (K = 3 real 2 x 2, 4 complex 2 x 2, 6 real 3 x 3).
template <typename R, int K>
__device__ __forceinline__ void herm_nuc_shrink(R (&x)[K], R t)
{
    if constexpr (K == 3) {
        R q = R(0);
        herm2_shrink<R>(x[0], x[1], x[2], q, t);
    } else if constexpr (K == 4) {
        herm2_shrink<R>(x[0], x[1], x[2], x[3], t);
    } else if constexpr (K == 6) {
        sym3_shrink<R>(x, t);
    }
}

template <typename R, int K>
__device__ __forceinline__ R herm_nuc(const R (&x)[K])
{
    if constexpr (K == 3) return herm2_nuc<R>(x[0], x[1], x[2], R(0));
    if constexpr (K == 4) return herm2_nuc<R>(x[0], x[1], x[2], x[3]);
    if constexpr (K == 6) return sym3_nuc<R>(x);
    return R(0);
}

// Nuclear shrink of the l transfer matrices W_s held in w[s * KS + q].
// A real skew matrix has singular values in equal pairs: 2 x 2 and 3 x 3
// ones have the nuclear norm sqrt2 |coordinates|, whose prox is a block
// shrink with threshold sqrt2 t; a complex 2 x 2 skew N is i times the
// Hermitian H = -iN with coordinates (c0, c1, c3, -c2).
template <typename R, int K, int LA>
__device__ __forceinline__ void skew_nuc_shrink(R (&w)[LA], int l, R t)
{
    constexpr int KS = skew_coords<K>();
    const R r2 = R(1.4142135623730950488);
#pragma unroll
    for (int s = 0; s * KS < LA; ++s) {
        if (s * KS >= l) break;
        if constexpr (K == 3 || K == 6) {
            R n2 = R(0);
#pragma unroll
            for (int q = 0; q < KS; ++q) n2 = n2 + w[s * KS + q] * w[s * KS + q];
            const R n = sqrt(n2);
            const R sc = shrink_scale<R>(n, r2 * t);
#pragma unroll
            for (int q = 0; q < KS; ++q) w[s * KS + q] = w[s * KS + q] * sc;
        } else if constexpr (K == 4) {
            R d0 = w[s * 4 + 0], d1 = w[s * 4 + 1], p = w[s * 4 + 3], q = -w[s * 4 + 2];
            herm2_shrink<R>(d0, d1, p, q, t);
            w[s * 4 + 0] = d0;
            w[s * 4 + 1] = d1;
            w[s * 4 + 2] = -q;
            w[s * 4 + 3] = p;
        }
    }
}

template <int K, int LA>
__device__ __forceinline__ double skew_nuc(const double (&w)[LA], int l)
{
    constexpr int KS = skew_coords<K>();
    double s_ = 0.0;
#pragma unroll
    for (int s = 0; s * KS < LA; ++s) {
        if (s * KS >= l) break;
        if constexpr (K == 3 || K == 6) {
            double n2 = 0.0;
#pragma unroll
            for (int q = 0; q < KS; ++q) n2 += w[s * KS + q] * w[s * KS + q];
            s_ += 1.4142135623730950488 * sqrt(n2);
        } else if constexpr (K == 4) {
            s_ += herm2_nuc<double>(w[s * 4 + 0], w[s * 4 + 1], w[s * 4 + 3], -w[s * 4 + 2]);
        }
    }
    return s_;
}

}  // namespace dev
}  // namespace omt
