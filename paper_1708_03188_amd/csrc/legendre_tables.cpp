// Plan tables of the Legendre-family x axis (Sec. 3.1, Sec. 3.4.2), computed in
// long double on the host and rounded once to binary64.
//
// Points: the zeros of L_N by Newton's method from the usual cosine guesses,
// stored descending; weights w_j = 2 / ((1 - x_j^2) L_N'(x_j)^2).
// Forward operator: with L[j][k] = L_k(x_j) and g_k = 2 / (2k + 1), Gauss
// quadrature gives L^T W L = diag(g), so the interpolant's Legendre
// coefficients are c = diag(1/g) L^T W u and, for u_hat in a basis with
// Legendre recombination P, sum_j w_j |(L P u_hat)_j - u_j|^2 =
// sum_k g_k |(P u_hat)_k - c_k|^2 for the interpolated part.  The weighted
// least-squares projection (eq. projection) is therefore the least-squares
// solution of diag(g)^{1/2} P u_hat = diag(g)^{1/2} c, which splits into the two
// parity classes; each is solved by a Householder QR in long double.
#include <cmath>
#include <string>
#include <vector>

#include "legendre.h"

namespace sgm {

using ld = long double;
static const ld PI_LL = 3.141592653589793238462643383279502884L;

// (L_n(x), L_n'(x)) by the three-term recurrence.
static void legendre_pd(int n, ld x, ld& p, ld& dp) {
    ld p0 = 1, p1 = x;
    if (n == 0) { p = 1; dp = 0; return; }
    for (int k = 1; k < n; ++k) {
        ld p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    dp = n * (p0 - x * p1) / (1 - x * x);
}

// Legendre coefficient k of basis function l (0 outside the recombination).
static ld recomb(int basis, int k, int l) {
    if (k == l) return 1;
    if (basis == SGM_LEG_DIRICHLET && k == l + 2) return -1;
    if (basis == SGM_LEG_NEUMANN && k == l + 2) return -(ld)(l * (l + 1)) / (ld)((l + 2) * (l + 3));
    if (basis == SGM_LEG_BIHARMONIC) {
        if (k == l + 2) return -(ld)(2 * (2 * l + 5)) / (ld)(2 * l + 7);
        if (k == l + 4) return (ld)(2 * l + 3) / (ld)(2 * l + 7);
    }
    return 0;
}

// Least-squares solution X (n x r) of A X = B for A m x n (m >= n, full rank) and
// B m x r, by Householder QR; A and B are overwritten.
static void lstsq(std::vector<ld>& A, int m, int n, std::vector<ld>& B, int r, std::vector<ld>& X) {
    auto a = [&](int i, int j) -> ld& { return A[(size_t)i * n + j]; };
    auto b = [&](int i, int j) -> ld& { return B[(size_t)i * r + j]; };
    std::vector<ld> v(m);
    for (int c = 0; c < n; ++c) {
        ld nrm = 0;
        for (int i = c; i < m; ++i) nrm += a(i, c) * a(i, c);
        nrm = sqrtl(nrm);
        const ld alpha = a(c, c) > 0 ? -nrm : nrm;
        for (int i = c; i < m; ++i) v[i] = a(i, c);
        v[c] -= alpha;
        ld vn = 0;
        for (int i = c; i < m; ++i) vn += v[i] * v[i];
        if (vn == 0) continue;
        for (int j = c; j < n; ++j) {
            ld d = 0;
            for (int i = c; i < m; ++i) d += v[i] * a(i, j);
            d = 2 * d / vn;
            for (int i = c; i < m; ++i) a(i, j) -= d * v[i];
        }
        for (int j = 0; j < r; ++j) {
            ld d = 0;
            for (int i = c; i < m; ++i) d += v[i] * b(i, j);
            d = 2 * d / vn;
            for (int i = c; i < m; ++i) b(i, j) -= d * v[i];
        }
    }
    X.assign((size_t)n * r, 0);
    for (int j = 0; j < r; ++j)
        for (int i = n - 1; i >= 0; --i) {
            ld s = b(i, j);
            for (int q = i + 1; q < n; ++q) s -= a(i, q) * X[(size_t)q * r + j];
            X[(size_t)i * r + j] = s / a(i, i);
        }
}

// Legendre series in extended precision: derivative of a coefficient vector,
// d_m = (2m + 1) sum_{k > m, k - m odd} c_k.
static std::vector<ld> leg_series_der(const std::vector<ld>& c) {
    const int n = (int)c.size();
    std::vector<ld> d(n, 0);
    ld s[2] = {0, 0};
    for (int k = n - 1; k >= 1; --k) {
        s[k & 1] += c[k];
        d[k - 1] = (ld)(2 * (k - 1) + 1) * s[k & 1];
    }
    return d;
}

// Galerkin rows per parity in the layout of the solver rows (20 doubles per row,
// offsets -2..2 in units of two modes): the Helmholtz bases (Dirichlet, Neumann)
// store -A, B; the biharmonic basis stores S, A, B with S_mj = (phi_j^(4), phi_m),
// A_mj = (phi_j'', phi_m), B_mj = (phi_j, phi_m), all with the Legendre weight 1:
// (L_k, L_n) = 2/(2n+1) delta_kn, derivatives exact in coefficient space.  No
// separable tail for these bases (the matrices are banded).
static void galerkin_rows(int basis, int N, int nb, LegTables& t) {
    const bool bih = basis == SGM_LEG_BIHARMONIC;
    std::vector<std::vector<ld>> d0(nb), d2(nb), d4(nb);
    for (int l = 0; l < nb; ++l) {
        std::vector<ld> c(N, 0);
        for (int k = l; k <= l + 4 && k < N; ++k) c[k] = recomb(basis, k, l);
        d2[l] = leg_series_der(leg_series_der(c));
        if (bih) d4[l] = leg_series_der(leg_series_der(d2[l]));
        d0[l] = std::move(c);
    }
    // (f, phi_m) for a Legendre series f
    auto inner = [&](const std::vector<ld>& f, int m) {
        ld s = 0;
        for (int k = m; k <= m + 4 && k < N; ++k) s += f[k] * recomb(basis, k, m) * (ld)2 / (ld)(2 * k + 1);
        return s;
    };
    for (int par = 0; par < 2; ++par) {
        const int n = t.npar[par];
        std::vector<double>& S = t.solve[par];
        S.assign(20 * (size_t)n, 0.0);
        for (int i = 0; i < n; ++i) {
            const int m = par + 2 * i;
            double* row = &S[20 * (size_t)i];
            for (int d = -2; d <= 2; ++d) {
                const int ii = i + d, j = m + 2 * d;
                if (ii < 0 || ii >= n) continue;
                if (bih) {
                    row[0 + d + 2] = (double)inner(d4[j], m);
                    row[5 + d + 2] = (double)inner(d2[j], m);
                    row[10 + d + 2] = (double)inner(d0[j], m);
                } else {
                    row[0 + d + 2] = (double)(-inner(d2[j], m));
                    row[5 + d + 2] = (double)inner(d0[j], m);
                }
            }
        }
    }
}

bool build_leg_tables(int basis, int N, LegTables& t, std::string& err) {
    if (!is_legendre_basis(basis)) { err = "not a Legendre basis"; return false; }
    const int nb = legendre_nbasis(basis, N);
    if (nb < 1) { err = "N too small for the basis"; return false; }
    if (N > kLegMaxN) { err = "Legendre spaces support N <= 512"; return false; }
    t.basis = basis;
    t.N = N;
    t.nb = nb;
    std::vector<ld> x(N), w(N);
    for (int j = 0; j < N; ++j) {
        ld xj = cosl(PI_LL * (4 * j + 3) / (4 * N + 2)), p, dp;
        for (int it = 0; it < 100; ++it) {
            legendre_pd(N, xj, p, dp);
            const ld dx = p / dp;
            xj -= dx;
            if (fabsl(dx) < 1e-30L) break;
        }
        legendre_pd(N, xj, p, dp);
        x[j] = xj;
        w[j] = 2 / ((1 - xj * xj) * dp * dp);
    }
    // L[j][k]
    std::vector<ld> L((size_t)N * N);
    for (int j = 0; j < N; ++j) {
        ld p0 = 1, p1 = x[j];
        L[(size_t)j * N] = 1;
        if (N > 1) L[(size_t)j * N + 1] = x[j];
        for (int k = 1; k + 1 < N; ++k) {
            const ld p2 = ((2 * k + 1) * x[j] * p1 - k * p0) / (k + 1);
            L[(size_t)j * N + k + 1] = p2;
            p0 = p1;
            p1 = p2;
        }
    }
    // Phi[j][l] = sum_k L_k(x_j) P[k][l]
    std::vector<ld> Phi((size_t)N * nb, 0);
    for (int j = 0; j < N; ++j)
        for (int l = 0; l < nb; ++l) {
            ld s = 0;
            for (int k = l; k <= l + 4 && k < N; ++k) s += L[(size_t)j * N + k] * recomb(basis, k, l);
            Phi[(size_t)j * nb + l] = s;
        }
    t.x.resize(N);
    t.w.resize(N);
    for (int j = 0; j < N; ++j) { t.x[j] = (double)x[j]; t.w[j] = (double)w[j]; }
    t.bwd.assign((size_t)N * N, 0.0);
    t.sp.assign((size_t)N * N, 0.0);
    for (int j = 0; j < N; ++j)
        for (int l = 0; l < nb; ++l) {
            t.bwd[(size_t)j * N + l] = (double)Phi[(size_t)j * nb + l];
            t.sp[(size_t)l * N + j] = (double)(Phi[(size_t)j * nb + l] * w[j]);
        }
    // discrete Legendre transform Lambda[k][j] = (2k + 1)/2 L_k(x_j) w_j
    std::vector<ld> Lam((size_t)N * N);
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j) Lam[(size_t)k * N + j] = (ld)(2 * k + 1) / 2 * L[(size_t)j * N + k] * w[j];
    for (int par = 0; par < 2; ++par) {
        t.npar[par] = nb > par ? (nb - par + 1) / 2 : 0;
        t.mpar[par] = N > par ? (N - par + 1) / 2 : 0;
    }
    if (basis != SGM_LEGENDRE) galerkin_rows(basis, N, nb, t);
    t.beta.assign(N, 0.0);
    t.gamma.assign(N, 0.0);
    for (int l = 0; l < nb; ++l) {
        if (l + 2 < N) t.beta[l] = (double)recomb(basis, l + 2, l);
        if (l + 4 < N) t.gamma[l] = (double)recomb(basis, l + 4, l);
    }
    t.fwd.assign((size_t)N * N, 0.0);
    if (basis == SGM_LEGENDRE) {
        for (size_t i = 0; i < Lam.size(); ++i) t.fwd[i] = (double)Lam[i];
        return true;
    }
    for (int par = 0; par < 2; ++par) {
        const int m = (N - par + 1) / 2, n = (nb - par + 1) / 2;
        if (n <= 0) continue;
        std::vector<ld> A((size_t)m * n, 0), B((size_t)m * N), X;
        for (int r = 0; r < m; ++r) {
            const int k = par + 2 * r;
            const ld sg = sqrtl((ld)2 / (2 * k + 1));
            for (int i = 0; i < n; ++i) A[(size_t)r * n + i] = sg * recomb(basis, k, par + 2 * i);
            for (int j = 0; j < N; ++j) B[(size_t)r * N + j] = sg * Lam[(size_t)k * N + j];
        }
        lstsq(A, m, n, B, N, X);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < N; ++j) t.fwd[(size_t)(par + 2 * i) * N + j] = (double)X[(size_t)i * N + j];
    }
    return true;
}

int leg_row_blocks(int N) {
    const int rb = (N + 15) / 16;
    return rb <= 4 ? 4 : rb <= 8 ? 8 : rb <= 16 ? 16 : 32;
}

size_t leg_packed_doubles(int N) { return (size_t)((N + 3) / 4) * leg_row_blocks(N) * 64; }

std::vector<double> leg_pack(const std::vector<double>& A, int N) {
    const int KG = (N + 3) / 4, RB = leg_row_blocks(N);
    std::vector<double> out(leg_packed_doubles(N), 0.0);
    for (int g = 0; g < KG; ++g)
        for (int r = 0; r < RB; ++r)
            for (int q = 0; q < 64; ++q) {
                const int row = 16 * r + q % 16, col = 4 * g + q / 16;
                if (row < N && col < N) out[((size_t)g * RB + r) * 64 + q] = A[(size_t)row * N + col];
            }
    return out;
}

}  // namespace sgm
