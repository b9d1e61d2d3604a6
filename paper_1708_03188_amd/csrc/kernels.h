// Kernel launch wrappers for the tensor-product transform passes (not ABI).
#pragma once
#include "common.h"

namespace sgm {

// Per-axis device tables of the Chebyshev/Shen direction.
struct ChebDev {
    int basis, N, nb;
    int npar[2], mpar[2];
    const double2* theta;   // N
    const double* beta;     // N
    const double* gamma;    // N
    const double* bscale;   // N
    const double* fscale;   // N
    const double* rot[2];   // 4 * npar
    const double* rtab[2];  // 3 * npar
    const double* qtab[2];  // 2 * mpar
    const double* solve[2]; // 20 * npar
    // segmented biharmonic projection: per-row state coefficients (2 * npar)
    // and per-segment 2 x 2 maps (4 * segments) of the Givens and
    // back-substitution sweeps
    const double* gal[2];
    const double* gmat[2];
    const double* bal[2];
    const double* bmat[2];
};

// rows per segment of the parallel biharmonic projection (the plan tables
// are built for the same value)
constexpr int kProjSegRowsDev = 16;

enum ChebFwdMode { kScalarProduct = 0, kProject = 1 };

// Column geometry of the spectral array seen by the x pass and the solves:
// ncols columns, column c = (iy, iz) with iy = c / nlast, iz = c % nlast.
struct ColGeom {
    int ncols;
    int nlast;       // length of the last spectral axis (M2/2+1, M2, or for ndim=2 the y axis)
    int Mmid;        // FFT length of the middle axis (ndim=3), 1 for ndim=2
    int Mlast;       // FFT length of the last axis
    int last_r2c;    // 1 if the last axis holds n = 0..M/2 only
    double sy, sz;   // (2 pi / Ly)^2 and (2 pi / Lz)^2 factors of kappa^2 (sy unused for ndim=2)
};

hipError_t launch_lines_r2c(const double* in, double2* out, int L, int nlines, int G, const RadixPlan& rp,
                            double scale, hipStream_t s);
hipError_t launch_lines_c2r(const double2* in, double* out, int L, int nlines, int G, const RadixPlan& rp,
                            hipStream_t s);
hipError_t launch_lines_c2c(const double2* in, double2* out, int L, int nlines, int G, const RadixPlan& rp,
                            int sign, double scale, hipStream_t s);
hipError_t launch_strided_c2c(const double2* in, double2* out, int L, int outer, int inner, int W,
                              const RadixPlan& rp, int sign, double scale, hipStream_t s);
hipError_t launch_cheb_fwd(const double2* in, double2* out, const ChebDev& cd, int ncols, int W,
                           const RadixPlan& rp, int mode, hipStream_t s);
hipError_t launch_cheb_bwd(const double2* in, double2* out, const ChebDev& cd, int ncols, int W,
                           const RadixPlan& rp, hipStream_t s);
hipError_t launch_solve(const double2* in, double2* out, const ChebDev& cd, const ColGeom& g, int W,
                        int kind, double alpha, hipStream_t s);

size_t lds_bytes_lines(int L, int G);
size_t lds_bytes_strided(int L, int W);
size_t lds_bytes_cheb(int N, int W);
size_t lds_bytes_solve(int N, int W, int basis);

}  // namespace sgm
