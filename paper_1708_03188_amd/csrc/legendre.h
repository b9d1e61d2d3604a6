// Legendre-family x axis (Sec. 3.1 Legendre bases, Sec. 3.4.2 Legendre-Gauss
// quadrature): plan tables and the dense transform pass.  Not ABI.
#pragma once
#include <string>
#include <vector>

#include "common.h"

namespace sgm {

inline bool is_legendre_basis(int b) {
    return b == SGM_LEGENDRE || b == SGM_LEG_DIRICHLET || b == SGM_LEG_NEUMANN || b == SGM_LEG_BIHARMONIC;
}
inline int legendre_nbasis(int b, int N) {
    return b == SGM_LEGENDRE ? N : b == SGM_LEG_BIHARMONIC ? N - 4 : N - 2;
}

// Dense x-axis operators of one Legendre space with N points, each an N x N
// row-major binary64 matrix acting on a column of N values (rows or columns
// beyond the basis size are zero):
//   fwd  u_hat = F u   (weighted least-squares projection, eq. projection)
//   bwd  u = Phi u_hat (synthesis at the points, eq. fast_shen)
//   sp   f_tilde = Phi^T W f (scalar product, eq. quadrature)
struct LegTables {
    int basis = 0, N = 0, nb = 0;
    std::vector<double> x, w;   // points (descending) and weights
    std::vector<double> fwd, bwd, sp;
    // Galerkin rows per parity (the layout of ChebTables::solve), weight 1, banded
    // (no separable tail): Dirichlet and Neumann -A (diagonal) and B (tridiagonal per
    // parity); biharmonic S (diagonal), A (tridiagonal), B (pentadiagonal)
    int npar[2] = {0, 0}, mpar[2] = {0, 0};
    std::vector<double> solve[2];
    // recombination coefficients of L_{l+2} and L_{l+4} in phi_l (N each, zero past
    // the basis), for the derivative pass
    std::vector<double> beta, gamma;
};
bool build_leg_tables(int basis, int N, LegTables& t, std::string& err);

// The matrix-core pass reads its matrix in fragment order: for k-group g (4
// columns of the matrix) and row block r (16 rows), 64 consecutive doubles, entry
// q holding A[16 r + q % 16][4 g + q / 16]; leg_row_blocks(N) row blocks per
// k-group (a multiple of 4, rows past N zero).
int leg_row_blocks(int N);
std::vector<double> leg_pack(const std::vector<double>& A, int N);
size_t leg_packed_doubles(int N);

// out[r][c] = sum_k A[r][k] in[k][c] for the N x C real view of a spectral array
// (C = 2 * complex columns), A packed by leg_pack.  in and out may be the same
// array (a work-group reads all of its columns before writing them).
hipError_t launch_leg_pass(const double* Apk, const double* in, double* out, int N, long C, hipStream_t s);

// Largest N of the pass.
constexpr int kLegMaxN = 512;

}  // namespace sgm
