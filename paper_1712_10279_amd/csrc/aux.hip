// Set-up, reduction and layout kernels around the fused PDHG step: FP64
// sums of the input densities (mass check), the source term f, the
// reductions of the per-check metrics (computed in metrics_device.h), the
// exported potential and the
// conversions between the caller's layout (m x n x k, channel fastest) and
// the SoA planes the step kernel streams.
//
// Every reduction writes one row of partial sums per workgroup (wavefront
// shuffles, then LDS, in a fixed order) and a single-workgroup kernel sums
// the rows in a fixed order, so results are deterministic.

#include "metrics_device.h"

namespace omt {
namespace {

constexpr int RB = 256;  // threads per reduction workgroup

template <typename R>
__device__ __forceinline__ double ld(const void *p, int64_t i)
{
    return double(static_cast<const R *>(p)[i]);
}

__device__ __forceinline__ double ldv(const void *p, int dtype, int64_t i)
{
    return dtype == 1 ? ld<double>(p, i) : ld<float>(p, i);
}

__device__ __forceinline__ void stv(void *p, int dtype, int64_t i, double v)
{
    if (dtype == 1)
        static_cast<double *>(p)[i] = v;
    else
        static_cast<float *>(p)[i] = float(v);
}

// Sum v[0..W) over the workgroup into out[0..W) (thread 0 writes).
template <int W>
__device__ void block_sum(double (&v)[W], double *out)
{
    __shared__ double sm[RB / WAVE][W];
#pragma unroll
    for (int q = 0; q < W; ++q) {
        double x = v[q];
#pragma unroll
        for (int off = WAVE / 2; off > 0; off >>= 1) x += __shfl_down(x, off, WAVE);
        v[q] = x;
    }
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < W; ++q) sm[wv][q] = v[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < W; ++q) {
            double s = 0.0;
            for (int w = 0; w < RB / WAVE; ++w) s += sm[w][q];
            out[q] = s;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------- set-up

__global__ __launch_bounds__(RB) void sums_kernel(SumsArgs a)
{
    // channel by channel: sum rho0, sum rho1, sum |rho0|, sum |rho1|; the last
    // column counts non-finite entries
    const int W = 4 * a.k + 1;
    double bad = 0.0;
    for (int c = 0; c < a.k; ++c) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t p = blockIdx.x * (int64_t)RB + threadIdx.x; p < a.npix; p += (int64_t)a.nblocks * RB) {
            const double x0 = ldv(a.rho0, a.dtype, p * a.k + c);
            const double x1 = ldv(a.rho1, a.dtype, p * a.k + c);
            if (!isfinite(x0) || !isfinite(x1)) {
                bad += 1.0;
                continue;
            }
            v[0] += x0;
            v[1] += x1;
            v[2] += fabs(x0);
            v[3] += fabs(x1);
        }
        double o[4];
        block_sum<4>(v, o);
        if (threadIdx.x == 0) {
            for (int q = 0; q < 4; ++q) a.partials[(int64_t)blockIdx.x * W + 4 * c + q] = o[q];
        }
    }
    double b[1] = {bad};
    double o1[1];
    block_sum<1>(b, o1);
    if (threadIdx.x == 0) a.partials[(int64_t)blockIdx.x * W + 4 * a.k] = o1[0];
}

// Pixel pp of the caller's layout (i, j and, on a 3-D grid, z; channel
// fastest) -> its offset within a plane: row z m + i, column j.
__device__ __forceinline__ int64_t plane_offset(int64_t pp, int m, int n, int p3, int pitch, int &i, int &j, int &z)
{
    z = int(pp % p3);
    const int64_t t = pp / p3;
    j = int(t % n);
    i = int(t / n);
    return ((int64_t)z * m + i) * pitch + j;
}

__global__ void make_f_kernel(MakeFArgs a)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= (int64_t)a.m * a.n * a.p) return;
    int i, j, z;
    const int64_t o = plane_offset(p, a.m, a.n, a.p, a.pitch, i, j, z);
    for (int c = 0; c < a.k; ++c) {
        const double x0 = ldv(a.rho0, a.dtype, p * a.k + c);
        const double x1 = ldv(a.rho1, a.dtype, p * a.k + c);
        stv(a.f, a.dtype, c * a.plane + o, (x1 - x0) - a.shift[c]);
    }
}

// ---------------------------------------------------------------- reductions

__global__ __launch_bounds__(RB) void reduce_rows_kernel(const double *partials, int nblocks, int width, double *out)
{
    __shared__ double sm[RB];
    for (int q = 0; q < width; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += RB) s += partials[(int64_t)b * width + q];
        sm[threadIdx.x] = s;
        __syncthreads();
        for (int h = RB / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[q] = sm[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(WAVE) void reduce_tiles_kernel(const double *partials, int ntiles, double *out)
{
    dev::reduce_tiles(partials, 0, ntiles, threadIdx.x, out);
}

// One wave per (row block, four column tiles): lanes 16 u .. 16 u + 15 hold
// the quads of tile 4 x + u and add them with shuffle offsets 1, 2, 4, 8
// (the last four levels of wave_sum); quads past the grid count as zero.
__global__ __launch_bounds__(WAVE) void quads_to_tiles_kernel(const double *qpart, int64_t qstride, int nq, int ncolw,
                                                              double *partials)
{
    const int blk = blockIdx.y;
    const int tile = blockIdx.x * 4 + int(threadIdx.x) / 16;
    const int quad = tile * 16 + int(threadIdx.x) % 16;
    const bool ok = tile < ncolw && quad < nq;
    for (int q = 0; q < NMET; ++q) {
        double x = ok ? qpart[q * qstride + (int64_t)blk * nq + quad] : 0.0;
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) x += __shfl_down(x, off, WAVE);
        if (threadIdx.x % 16 == 0 && tile < ncolw) partials[((int64_t)blk * ncolw + tile) * NMET + q] = x;
    }
}

__global__ __launch_bounds__(RB) void plane_sums_kernel(PlaneSumArgs a)
{
    for (int c = 0; c < a.k; ++c) {
        double v[1] = {0.0};
        for (int64_t p = blockIdx.x * (int64_t)RB + threadIdx.x; p < (int64_t)a.m * a.n; p += (int64_t)a.nblocks * RB) {
            const int i = int(p / a.n), j = int(p % a.n);
            const int64_t o = c * a.plane + (int64_t)i * a.pitch + j;
            v[0] += ldv(a.phi, a.dtype, o) + (a.plo ? double(a.plo[o]) : 0.0);
        }
        double o1[1];
        block_sum<1>(v, o1);
        if (threadIdx.x == 0) a.partials[(int64_t)blockIdx.x * a.k + c] = o1[0];
    }
}

__global__ void xfer_kernel(XferArgs a)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= (int64_t)a.m * a.n * a.p) return;
    int i, j, z;
    const int64_t o = plane_offset(p, a.m, a.n, a.p, a.pitch, i, j, z);
    const int k = a.k;
    const int nc = a.p > 1 ? 3 : 2;  // flux components per channel
    switch (a.mode) {
        case 0:  // exported potential: sign * (-(phi - mean))
            for (int c = 0; c < k; ++c) {
                double x = ldv(a.src, a.dtype, c * a.plane + o);
                if (a.plo) x += double(a.plo[c * a.plane + o]);
                stv(a.dst, a.dtype, p * k + c, a.sign * (-(x - a.mean[c])));
            }
            break;
        case 1:  // u planes -> m x n (x p) x k x nc
            for (int c = 0; c < k; ++c)
                for (int d = 0; d < nc; ++d)
                    stv(a.dst, a.dtype, (p * k + c) * nc + d, ldv(a.src, a.dtype, (d * k + c) * a.plane + o));
            break;
        case 2:  // planes -> m x n x k (w, or phi when plo is null)
            for (int c = 0; c < k; ++c) {
                double x = ldv(a.src, a.dtype, c * a.plane + o);
                if (a.plo) x += double(a.plo[c * a.plane + o]);
                stv(a.dst, a.dtype, p * k + c, x);
            }
            break;
        case 3:  // m x n x k -> planes (phi or w); low parts cleared
            for (int c = 0; c < k; ++c) {
                stv(a.dst, a.dtype, c * a.plane + o, a.src ? ldv(a.src, a.dtype, p * k + c) : 0.0);
                if (a.plo_out) a.plo_out[c * a.plane + o] = 0.0f;
            }
            break;
        case 4:  // m x n (x p) x k x nc -> u planes, ghosts zeroed (App. A)
            for (int c = 0; c < k; ++c) {
                const double x = (a.src && i < a.m - 1) ? ldv(a.src, a.dtype, (p * k + c) * nc + 0) : 0.0;
                const double y = (a.src && j < a.n - 1) ? ldv(a.src, a.dtype, (p * k + c) * nc + 1) : 0.0;
                stv(a.dst, a.dtype, c * a.plane + o, x);
                stv(a.dst, a.dtype, (k + c) * a.plane + o, y);
                if (nc == 3) {
                    const double zz = (a.src && z < a.p - 1) ? ldv(a.src, a.dtype, (p * k + c) * nc + 2) : 0.0;
                    stv(a.dst, a.dtype, (2 * k + c) * a.plane + o, zz);
                }
            }
            break;
        default:
            break;
    }
}

__device__ __forceinline__ int matrix_ncoord(int k, int real, int herm)
{
    return real ? (herm ? k * (k + 1) / 2 : k * (k - 1) / 2) : k * k;
}

__global__ void matrix_xfer_kernel(MatrixXferArgs a)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;  // (pixel, matrix)
    if (q >= a.npix * a.count) return;
    const int k = a.k, nc = matrix_ncoord(k, a.real, a.herm);
    const int ent = a.real ? 1 : 2;                  // values per matrix entry
    const int64_t mbase = q * k * k * ent;           // first entry of this matrix
    const int64_t cbase = q * nc;                    // first coordinate of this group
    const double r2 = 1.4142135623730951, ir2 = 0.70710678118654752;
    auto cidx = [&](int c) { return (cbase + c) * a.cstride + a.coff; };
    auto midx = [&](int r, int c) { return mbase + (int64_t(r) * k + c) * ent; };
    // diagonal
    const int nd = (a.herm || !a.real) ? k : 0;
    for (int d = 0; d < nd; ++d) {
        if (a.pack) {
            const double v = a.herm ? ldv(a.src, a.dtype, midx(d, d)) : ldv(a.src, a.dtype, midx(d, d) + 1);
            stv(a.dst, a.dtype, cidx(d), v);
        } else {
            const double v = ldv(a.src, a.dtype, cidx(d));
            if (a.real) {
                stv(a.dst, a.dtype, midx(d, d), v);
            } else {
                stv(a.dst, a.dtype, midx(d, d), a.herm ? v : 0.0);
                stv(a.dst, a.dtype, midx(d, d) + 1, a.herm ? 0.0 : v);
            }
        }
    }
    if (!a.pack && a.real && !a.herm)
        for (int d = 0; d < k; ++d) stv(a.dst, a.dtype, midx(d, d), 0.0);
    // pairs a < b
    int c = nd;
    for (int r = 0; r < k; ++r)
        for (int s = r + 1; s < k; ++s) {
            if (a.pack) {
                stv(a.dst, a.dtype, cidx(c), r2 * ldv(a.src, a.dtype, midx(r, s)));
                if (!a.real) stv(a.dst, a.dtype, cidx(c + 1), r2 * ldv(a.src, a.dtype, midx(r, s) + 1));
            } else {
                const double re = ir2 * ldv(a.src, a.dtype, cidx(c));
                const double im = a.real ? 0.0 : ir2 * ldv(a.src, a.dtype, cidx(c + 1));
                // X_rs = re + i im; X_sr = conj (Hermitian) or -conj (skew)
                stv(a.dst, a.dtype, midx(r, s), re);
                stv(a.dst, a.dtype, midx(s, r), a.herm ? re : -re);
                if (!a.real) {
                    stv(a.dst, a.dtype, midx(r, s) + 1, im);
                    stv(a.dst, a.dtype, midx(s, r) + 1, a.herm ? -im : im);
                }
            }
            c += a.real ? 1 : 2;
        }
}

__global__ void zero_kernel(uint32_t *p, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
        p[q] = 0u;
}

// Every 32-bit word of nplanes planes (stride_words apart) that lies outside
// the grid -- past rows * row_words in the plane, or at a word column >=
// n_words of a row -- becomes all ones, a NaN in FP32 and FP64 alike.
__global__ void poison_kernel(uint32_t *p, int64_t nplanes, int64_t stride_words, int64_t row_words, int64_t rows,
                              int64_t n_words)
{
    const int64_t total = nplanes * stride_words;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = q % stride_words;
        if (o / row_words >= rows || o % row_words >= n_words) p[q] = 0xFFFFFFFFu;
    }
}

}  // namespace

hipError_t launch_sums(const SumsArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(sums_kernel, dim3(a.nblocks), dim3(RB), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_make_f(const MakeFArgs &a, hipStream_t s)
{
    const int64_t n = (int64_t)a.m * a.n * a.p;
    hipLaunchKernelGGL(make_f_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce_rows(const double *partials, int nblocks, int width, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_rows_kernel, dim3(1), dim3(RB), 0, s, partials, nblocks, width, out);
    return hipGetLastError();
}

hipError_t launch_reduce_tiles(const double *partials, int ntiles, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(reduce_tiles_kernel, dim3(1), dim3(WAVE), 0, s, partials, ntiles, out);
    return hipGetLastError();
}

hipError_t launch_quads_to_tiles(const double *qpart, int64_t qstride, int nq, int nblk, int ncolw, double *partials,
                                 hipStream_t s)
{
    hipLaunchKernelGGL(quads_to_tiles_kernel, dim3(unsigned((ncolw + 3) / 4), unsigned(nblk)), dim3(WAVE), 0, s, qpart,
                       qstride, nq, ncolw, partials);
    return hipGetLastError();
}

hipError_t launch_plane_sums(const PlaneSumArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(plane_sums_kernel, dim3(a.nblocks), dim3(RB), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_xfer(const XferArgs &a, hipStream_t s)
{
    if (a.p < 1) return hipErrorInvalidValue;
    const int64_t n = (int64_t)a.m * a.n * a.p;
    hipLaunchKernelGGL(xfer_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_matrix_xfer(const MatrixXferArgs &a, hipStream_t s)
{
    const int64_t n = a.npix * a.count;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(matrix_xfer_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_poison(void *p, int64_t nplanes, size_t plane_stride_bytes, int row_elems, int64_t rows, int n,
                         int esz, hipStream_t s)
{
    if (nplanes <= 0 || plane_stride_bytes % 4 != 0 || esz % 4 != 0) return nplanes <= 0 ? hipSuccess : hipErrorInvalidValue;
    const int64_t stride_words = int64_t(plane_stride_bytes / 4), total = nplanes * stride_words;
    const int64_t blocks = (total + 255) / 256;
    hipLaunchKernelGGL(poison_kernel, dim3(unsigned(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s,
                       static_cast<uint32_t *>(p), nplanes, stride_words, int64_t(row_elems) * (esz / 4), rows,
                       int64_t(n) * (esz / 4));
    return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    const int64_t n = int64_t(bytes / 4);
    if (n == 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(zero_kernel, dim3(unsigned(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s,
                       static_cast<uint32_t *>(p), n);
    return hipGetLastError();
}

}  // namespace omt
