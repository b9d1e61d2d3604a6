// Small 2D spaces in one kernel (not ABI): for N, M <= 64 a whole field fits in
// one work-group's LDS, and a transform is two dense products there (the
// periodic axis as a DFT, the x axis as the plan's projection, scalar-product or
// synthesis matrix), one launch per call instead of a pass per axis.
#pragma once
#include <string>
#include <vector>

#include "kernels.h"

namespace sgm {

constexpr int kSmallMaxN = 64;
constexpr int kSmallMaxM = 64;

// Device view of the tables: F [M][Mc] forward DFT e^{-2 pi i n y / M} / M of the
// Mc stored coefficients; G [Mc][M] backward DFT e^{+2 pi i n y / M}, times the
// Hermitian weight (1 for n = 0 and n = M/2, 2 otherwise) on an R2C axis;
// P[0] projection, P[1] scalar product (both N x N, rows >= the basis size zero),
// P[2] synthesis (N x N, columns >= the basis size zero), row-major.
struct SmallDev {
    int N, M, Mc, r2c;
    const double2* F;
    const double2* G;
    const double* P[3];
};

enum SmallMode { kSmallForward = 0, kSmallScalar = 1, kSmallBackward = 2 };

// Doubles of the packed tables: F, G (complex), then the three N x N matrices.
size_t small_table_doubles(int N, int M, bool r2c);
// Build the packed tables for a Chebyshev-family basis (SGM_CHEBYSHEV,
// SGM_SHEN_DIRICHLET, SGM_SHEN_NEUMANN) on the Gauss-Chebyshev points, or take
// the x matrices of a Legendre-family space from fwd / sp / bwd (row-major
// N x N, as built for its dense pass).
bool build_small_tables(int basis, int N, int M, bool r2c, const std::vector<double>* leg_fwd,
                        const std::vector<double>* leg_sp, const std::vector<double>* leg_bwd,
                        std::vector<double>& out, std::string& err);
// Dynamic LDS bytes of the kernel for a space.
size_t small_lds_bytes(int N, int M, bool r2c);
// One transform of the field in -> out (forward / scalar product: physical to
// spectral; backward: spectral to physical).  in and out must not overlap.
hipError_t launch_small_pass(const void* in, void* out, const SmallDev& sd, int mode, hipStream_t s);

}  // namespace sgm
