// Host-side construction of the plan constants (long double arithmetic,
// rounded once to binary64 for upload).  Not part of the ABI.
#pragma once
#include <complex>
#include <vector>

namespace sgm {

// exp(-2 pi i r / L), r = 0..L-1, from the exactly reduced index r.
std::vector<double> twiddles(int L);

constexpr int kProjSegRows = 16;

// Tables of one Chebyshev/Shen axis with N points; all vectors are flat
// binary64 arrays ready for upload.
struct ChebTables {
    int basis = 0;
    int N = 0;
    int nb = 0;              // number of basis functions
    int npar[2] = {0, 0};    // basis functions of parity 0 / 1
    int mpar[2] = {0, 0};    // Chebyshev modes of parity 0 / 1
    std::vector<double> theta;   // 2N: exp(-i pi k / (2N)), k = 0..N-1
    std::vector<double> beta;    // N: recombination coefficient of T_{l+2} in phi_l (0 if none)
    std::vector<double> gamma;   // N: coefficient of T_{l+4} in phi_l
    std::vector<double> bscale;  // N: sqrt(2 pi / c_k) / N  (DCT-II sum -> sqrt(D) * Chebyshev coefficient)
    std::vector<double> fscale;  // N: 2 / (c_k N)          (DCT-II sum -> Chebyshev coefficient)
    // Givens least-squares projection, per parity p, step i:
    // rot[p][4i..4i+3] = (c1, s1, c2, s2), rtab[p][3i..3i+2] = (1/R_ii, R_i,i+1, R_i,i+2)
    std::vector<double> rot[2];
    std::vector<double> rtab[2];
    // The two sweeps of that solve cut into segments of kProjSegRows rows
    // (biharmonic): per row i, gal[p][2i..] / bal[p][2i..] = how the Givens
    // output / back-substituted value of row i depends on the two-value state
    // entering its segment; per segment u, gmat[p][4u..] / bmat[p][4u..] = the
    // 2 x 2 map from the entering to the leaving state (row-major).
    std::vector<double> gal[2], gmat[2], bal[2], bmat[2];
    // Orthonormal basis of the boundary functionals in the D^{1/2}-scaled
    // coordinates, per parity: qtab[p][2t + r], r < nrot (1 Dirichlet, 2 biharmonic).
    std::vector<double> qtab[2];
    // Galerkin solver rows, per parity p, row i: 20 doubles
    // [t0(-2..2), t1(-2..2), t2(-2..2), U1, U2, V1, V2, pad]
    // M = T0 + mu1 T1 + mu2 T2 (band), plus sum_r U_r(i) V_r(j) for j >= i + s.
    std::vector<double> solve[2];
    int solve_s = 1;     // first parity offset of the separable tail
    int solve_rank = 1;  // number of separable terms
};

// Fill every table for `basis` (SGM_* constant) and N points.
// Returns false (with a message in err) for unsupported combinations.
bool build_cheb_tables(int basis, int N, ChebTables& t, std::string& err);

}  // namespace sgm
