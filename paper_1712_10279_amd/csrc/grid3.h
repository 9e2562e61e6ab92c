// Interface between the host driver and the 3-D grid kernels (step3.hip).
//
// A 3-D field is stored as SoA planes like a 2-D one, each plane holding the
// p slices of m rows one after another: element (i, j, z) of a plane at
// (z m + i) pitch + j.  u has 3k planes (u_x, then u_y, then u_z).
#pragma once

#include "omt_kernels.h"

namespace omt {

// rows of the register tile one wavefront updates per slice
constexpr int G3_ROWS = 4;
// columns a wavefront stores: all 64 lanes, an aligned block of columns
constexpr int G3_COLS = 64;

template <typename R>
struct Step3Args {
    const R *phi_in;
    R *phi_out;
    const R *u_in;
    R *u_out;
    const R *w_in;
    R *w_out;
    const R *f;
    int64_t plane;         // elements per plane
    int32_t m, n, p, pitch;
    int32_t l;             // edges in use
    int32_t unorm, wnorm;
    int32_t ncolw, nroww;  // waves across (64-column strips) and down (row tiles)
    int32_t zch, nzw;      // slices per wave and z chunks
    int32_t nwg;           // workgroups launched
    R mu, mu_h, nu, anu, tau, inv_h, ureg, wreg;
    R ic[LMAX];
    R gm[KMAX * LMAX];
};

// Check quantities of a 3-D step (in -> out buffers of the args): one row of
// NMET FP64 partial sums per tile (64 columns x MET_ROWS rows of one slice).
struct Metrics3Launch {
    int dtype, k, gk, lb;
    const void *args;  // Step3Args<float> or <double>
    double alpha, eps;
    int ncolw, ntiles;
    double *partials;
    hipStream_t stream;
};

bool step3_supported(int dtype, int k, int gk, int lb);
hipError_t launch_step3(int dtype, int k, int gk, int lb, const void *args, hipStream_t stream);
hipError_t launch_metrics3(const Metrics3Launch &L);

}  // namespace omt
