// Host tables of the small-space kernel (extended precision, rounded once).
#include <cmath>

#include "small.h"

namespace sgm {

namespace {

typedef long double ld;
const ld kPi = 3.141592653589793238462643383279502884L;

// T_k(x_j), x_j = cos((2j+1) pi / (2N)): cos(pi r / (2N)) with r = k(2j+1) reduced mod 4N
ld cheb_t(int k, int j, int N) {
    const long r = ((long)k * (2 * j + 1)) % (4L * N);
    return cosl(kPi * (ld)r / (2.0L * N));
}

// Chebyshev coefficient k of basis function l
ld cheb_recomb(int basis, int k, int l) {
    if (k == l) return 1;
    if (k == l + 2) {
        if (basis == SGM_SHEN_DIRICHLET) return -1;
        if (basis == SGM_SHEN_NEUMANN) {
            const ld q = (ld)l / (ld)(l + 2);
            return -q * q;
        }
    }
    return 0;
}

// X = A^{-1} B for A n x n, B n x r (Gaussian elimination, partial pivoting);
// false if A is singular.
bool solve(std::vector<ld> A, int n, std::vector<ld> B, int r, std::vector<ld>& X) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (fabsl(A[(size_t)i * n + c]) > fabsl(A[(size_t)piv * n + c])) piv = i;
        if (A[(size_t)piv * n + c] == 0) return false;
        if (piv != c) {
            for (int j = 0; j < n; ++j) std::swap(A[(size_t)c * n + j], A[(size_t)piv * n + j]);
            for (int j = 0; j < r; ++j) std::swap(B[(size_t)c * r + j], B[(size_t)piv * r + j]);
        }
        for (int i = c + 1; i < n; ++i) {
            const ld f = A[(size_t)i * n + c] / A[(size_t)c * n + c];
            if (f == 0) continue;
            for (int j = c; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)c * n + j];
            for (int j = 0; j < r; ++j) B[(size_t)i * r + j] -= f * B[(size_t)c * r + j];
        }
    }
    X.assign((size_t)n * r, 0);
    for (int c = n - 1; c >= 0; --c)
        for (int j = 0; j < r; ++j) {
            ld s = B[(size_t)c * r + j];
            for (int k = c + 1; k < n; ++k) s -= A[(size_t)c * n + k] * X[(size_t)k * r + j];
            X[(size_t)c * r + j] = s / A[(size_t)c * n + c];
        }
    return true;
}

}  // namespace

size_t small_table_doubles(int N, int M, bool r2c) {
    const int Mc = r2c ? M / 2 + 1 : M;
    return 2 * (size_t)M * Mc * 2 + 3 * (size_t)N * N;
}

size_t small_lds_bytes(int N, int M, bool r2c) {
    const int Mc = r2c ? M / 2 + 1 : M;
    // forward: input [N][M] + intermediate [N][Mc]; backward: two [N][Mc]
    return sizeof(double2) * (size_t)N * (size_t)std::max(M + Mc, 2 * Mc);
}

bool build_small_tables(int basis, int N, int M, bool r2c, const std::vector<double>* leg_fwd,
                        const std::vector<double>* leg_sp, const std::vector<double>* leg_bwd,
                        std::vector<double>& out, std::string& err) {
    if (N < 1 || N > kSmallMaxN || M < 1 || M > kSmallMaxM) {
        err = "space too large for the small-space kernel";
        return false;
    }
    const int Mc = r2c ? M / 2 + 1 : M;
    out.assign(small_table_doubles(N, M, r2c), 0.0);
    double* F = out.data();
    double* G = F + 2 * (size_t)M * Mc;
    double* P = G + 2 * (size_t)M * Mc;
    // DFTs with the phase index n y reduced mod M exactly
    for (int y = 0; y < M; ++y)
        for (int n = 0; n < Mc; ++n) {
            const long r = ((long)n * y) % M;
            const ld th = 2 * kPi * (ld)r / (ld)M;
            const ld cs = cosl(th), sn = sinl(th);
            F[2 * ((size_t)y * Mc + n)] = (double)(cs / M);
            F[2 * ((size_t)y * Mc + n) + 1] = (double)(-sn / M);
            const ld h = (!r2c || n == 0 || 2 * n == M) ? 1 : 2;
            // exact zeros where the phase is a multiple of pi
            const ld sn0 = (2 * r == M || r == 0) ? 0 : sn;
            G[2 * ((size_t)n * M + y)] = (double)(h * cs);
            G[2 * ((size_t)n * M + y) + 1] = (double)(h * sn0);
        }
    double* Pf = P;
    double* Ps = P + (size_t)N * N;
    double* Pb = P + 2 * (size_t)N * N;
    if (leg_fwd) {
        if (!leg_sp || !leg_bwd || leg_fwd->size() != (size_t)N * N) {
            err = "Legendre matrices missing";
            return false;
        }
        std::copy(leg_fwd->begin(), leg_fwd->end(), Pf);
        std::copy(leg_sp->begin(), leg_sp->end(), Ps);
        std::copy(leg_bwd->begin(), leg_bwd->end(), Pb);
        return true;
    }
    if (basis != SGM_CHEBYSHEV && basis != SGM_SHEN_DIRICHLET && basis != SGM_SHEN_NEUMANN) {
        err = "basis not handled by the small-space kernel";
        return false;
    }
    const int nb = basis == SGM_CHEBYSHEV ? N : N - 2;
    if (nb < 1) {
        err = "N too small for the basis";
        return false;
    }
    // Phi[j][l] = phi_l(x_j), weights pi / N
    std::vector<ld> Phi((size_t)N * nb, 0);
    for (int j = 0; j < N; ++j)
        for (int l = 0; l < nb; ++l) {
            ld s = 0;
            for (int k = l; k <= l + 2 && k < N; ++k) s += cheb_recomb(basis, k, l) * cheb_t(k, j, N);
            Phi[(size_t)j * nb + l] = s;
        }
    const ld w = kPi / N;
    // scalar product S = Phi^T W, mass B = Phi^T W Phi, projection B^{-1} S
    std::vector<ld> S((size_t)nb * N), B((size_t)nb * nb, 0), X;
    for (int l = 0; l < nb; ++l)
        for (int j = 0; j < N; ++j) S[(size_t)l * N + j] = Phi[(size_t)j * nb + l] * w;
    for (int l = 0; l < nb; ++l)
        for (int m = 0; m < nb; ++m) {
            ld s = 0;
            for (int j = 0; j < N; ++j) s += S[(size_t)l * N + j] * Phi[(size_t)j * nb + m];
            B[(size_t)l * nb + m] = s;
        }
    if (!solve(B, nb, S, N, X)) {
        err = "singular mass matrix";
        return false;
    }
    for (int l = 0; l < nb; ++l)
        for (int j = 0; j < N; ++j) {
            Pf[(size_t)l * N + j] = (double)X[(size_t)l * N + j];
            Ps[(size_t)l * N + j] = (double)S[(size_t)l * N + j];
        }
    for (int j = 0; j < N; ++j)
        for (int l = 0; l < nb; ++l) Pb[(size_t)j * N + l] = (double)Phi[(size_t)j * nb + l];
    return true;
}

}  // namespace sgm
