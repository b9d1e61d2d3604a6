// Register-FFT pass kernels for the compile-time lengths (not ABI).
#pragma once
#include "kernels.h"

namespace sgm {

enum RegChebMode { kProjCheb = 2, kProjDirichlet = 3, kProjBiharmonic = 4, kScalarSolve = 5 };

// Extra arguments of the fused scalar-product + Dirichlet Helmholtz solve pass
// (boundary-state table of the segmented solve for this alpha); unused by the
// other Chebyshev-axis modes.
struct ChebSolve {
    const double* tab;
    ColGeom g;
    double alpha;
};

struct RegKernels {
    int L = 0;
    int W = 0;       // lines per block
    int threads = 0; // block size (W * threads per line)
    size_t lds = 0;      // dynamic LDS bytes of the Fourier-line kernels
    size_t lds_cheb = 0; // dynamic LDS bytes of the Chebyshev-axis kernels (two tiles)
    size_t lds_str = 0;  // dynamic LDS bytes of the strided kernels (exchange + twiddles)
    int variant = 0;
    void (*r2c)(const double*, double2*, int, const double2*, double) = nullptr;
    void (*c2r)(const double2*, double*, int, const double2*) = nullptr;
    void (*c2c_f)(const double2*, double2*, int, const double2*, double) = nullptr;
    void (*c2c_b)(const double2*, double2*, int, const double2*, double) = nullptr;
    void (*str_f)(const double2*, double2*, int, int, const double2*, double) = nullptr;
    void (*str_b)(const double2*, double2*, int, int, const double2*, double) = nullptr;
    void (*cf_sp)(const double2*, double2*, ChebDev, int, const double2*, ChebSolve) = nullptr;
    void (*cf_cheb)(const double2*, double2*, ChebDev, int, const double2*, ChebSolve) = nullptr;
    void (*cf_dir)(const double2*, double2*, ChebDev, int, const double2*, ChebSolve) = nullptr;
    void (*cf_bih)(const double2*, double2*, ChebDev, int, const double2*, ChebSolve) = nullptr;
    // fused scalar product + Dirichlet Helmholtz solve (L = 256 with 8-column
    // tiles only: chains of at most 128 rows on 8 lanes; nullptr elsewhere)
    void (*cf_spsolve)(const double2*, double2*, ChebDev, int, const double2*, ChebSolve) = nullptr;
    void (*cb)(const double2*, double2*, ChebDev, int, const double2*) = nullptr;
};

constexpr int kRegVariants = 8;
// Fill `k` with variant `variant` of the kernels for length L; false if L (or
// that variant) has no compiled instance.
bool reg_kernels_for(int L, RegKernels& k, int variant = 0);

// Byte-offset range of the strided kernels' buffer accesses.
constexpr long kBufRange = 0x7ffffff0;
inline bool strided_fits(const RegKernels& k, int inner) { return (long)(k.W + 2L * inner) * k.L * 16 < kBufRange; }

// Strided pass (sign -1 forward, +1 backward) over `outer` slabs of L x inner
// complex values, line stride inner: persistent launch sized to the device's
// occupancy.  hipErrorInvalidValue if a slab pair exceeds the kernel's 2 GB
// buffer-offset range.
hipError_t launch_strided(const RegKernels& k, int sign, const double2* in, double2* out, int outer, int inner,
                          const double2* tw, double scale, hipStream_t s);

}  // namespace sgm
