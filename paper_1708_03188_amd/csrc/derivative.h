// Spectral derivative + projection pass (not ABI).
#pragma once
#include "kernels.h"

namespace sgm {

// Arguments of the derivative pass over the columns of a spectral array
// [N][ncols] (column c = (iy, iz) as in ColGeom).
struct DxArgs {
    int N;
    int ncols;
    int src_basis;        // basis of the input coefficients
    int nb_src;           // its number of basis functions
    const double* beta;   // recombination T_{l+2} coefficients of the source (N)
    const double* gamma;  // recombination T_{l+4} coefficients of the source (N)
    int dst_basis;        // SGM_CHEBYSHEV, SGM_SHEN_DIRICHLET, SGM_SHEN_NEUMANN, or the
                          // Legendre ones SGM_LEGENDRE, SGM_LEG_DIRICHLET, SGM_LEG_NEUMANN
    int leg;              // 1: Legendre family (coefficients of L_k), 0: Chebyshev (of T_k)
    // Neumann target: sum over the even / odd k < N of q_k^2 h_k, with q_k the
    // derivative of the k-th polynomial at x = 1 up to a constant (Chebyshev k^2,
    // Legendre k(k+1)) and h_k the inverse of its squared norm up to a constant
    // (Chebyshev 1 for k >= 1, Legendre (2k+1)/2)
    double k4[2];
    int ox, oy, oz;       // derivative orders along x, y (middle or last), z (last, ndim = 3)
    int ndim;
    int nlast, Mmid, Mlast, last_r2c;
    double ky, kz;        // 2 pi / Ly and 2 pi / Lz
};

// Largest N the pass supports.
constexpr int kDxMaxN = 512;

hipError_t launch_dx_project(const double2* in, double2* out, const DxArgs& a, hipStream_t s);

}  // namespace sgm
