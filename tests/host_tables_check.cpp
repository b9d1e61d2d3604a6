// Host-side check of the plan-table builders, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py (no GPU needed):
// every table of every basis over a range of N, the Legendre operators and
// their fragment packing, the Fourier twiddles and the radix factorisation.
// Structural checks only (sizes, finiteness, products); the values themselves
// are checked against the oracle by the GPU parity tests.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "legendre.h"
#include "tables.h"

using namespace sgm;

static int fails = 0;
#define CHECK(c, ...)                       \
    do {                                    \
        if (!(c)) {                         \
            std::fprintf(stderr, __VA_ARGS__); \
            std::fprintf(stderr, "\n");     \
            ++fails;                        \
        }                                   \
    } while (0)

static bool finite(const std::vector<double>& v) {
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

int main() {
    // radix factorisation: the stage radices multiply to L
    for (int L = 1; L <= 4096; ++L) {
        int rad[kMaxStages];
        const int n = factor_radices(L, rad);
        long prod = 1;
        for (int i = 0; i < n; ++i) prod *= rad[i];
        CHECK(n >= 0 && n <= kMaxStages && prod == L, "factor_radices(%d)", L);
    }
    // twiddles: L unit-modulus values
    for (int L = 1; L <= 1100; L += (L < 64 ? 1 : 37)) {
        const std::vector<double> w = twiddles(L);
        CHECK((int)w.size() == 2 * L && finite(w), "twiddles(%d) size", L);
        for (int r = 0; r < L; ++r)
            CHECK(std::fabs(std::hypot(w[2 * r], w[2 * r + 1]) - 1.0) < 1e-15, "twiddles(%d)[%d]", L, r);
    }
    // Chebyshev-family tables
    const int cheb[4] = {SGM_SHEN_DIRICHLET, SGM_SHEN_BIHARMONIC, SGM_CHEBYSHEV, SGM_SHEN_NEUMANN};
    std::vector<int> Ns;
    for (int N = 2; N <= 80; ++N) Ns.push_back(N);
    for (int N : {127, 128, 129, 255, 256, 257, 300, 511, 512}) Ns.push_back(N);
    for (int basis : cheb)
        for (int N : Ns) {
            ChebTables t;
            std::string err;
            const int minN = basis == SGM_SHEN_BIHARMONIC ? 5 : basis == SGM_CHEBYSHEV ? 2 : 3;
            const bool ok = build_cheb_tables(basis, N, t, err);
            if (N < minN) continue;  // below the basis minimum the plan rejects N before building
            if (!ok) {
                // the Neumann basis is limited by its derivative-pass projection
                CHECK(basis == SGM_SHEN_NEUMANN && !err.empty(), "cheb tables basis %d N %d: %s", basis, N, err.c_str());
                continue;
            }
            CHECK(t.N == N && t.npar[0] + t.npar[1] == t.nb && t.mpar[0] + t.mpar[1] == N, "cheb counts %d %d", basis, N);
            CHECK((int)t.theta.size() == 2 * N && finite(t.theta), "theta %d %d", basis, N);
            CHECK(finite(t.beta) && finite(t.gamma) && finite(t.bscale) && finite(t.fscale), "scales %d %d", basis, N);
            for (int p = 0; p < 2; ++p) {
                CHECK(finite(t.rot[p]) && finite(t.rtab[p]) && finite(t.qtab[p]), "projection %d %d", basis, N);
                CHECK(finite(t.gal[p]) && finite(t.gmat[p]) && finite(t.bal[p]) && finite(t.bmat[p]), "segments %d %d",
                      basis, N);
                CHECK(finite(t.solve[p]), "solve rows %d %d", basis, N);
                if (basis != SGM_CHEBYSHEV)
                    CHECK(t.solve[p].size() == 20 * (size_t)t.npar[p], "solve size %d %d", basis, N);
            }
        }
    // Legendre-family operators
    const int leg[4] = {SGM_LEGENDRE, SGM_LEG_DIRICHLET, SGM_LEG_NEUMANN, SGM_LEG_BIHARMONIC};
    for (int basis : leg)
        for (int N : {5, 6, 7, 8, 13, 16, 33, 64, 100, 160}) {
            LegTables t;
            std::string err;
            CHECK(build_leg_tables(basis, N, t, err), "leg tables %d %d: %s", basis, N, err.c_str());
            const size_t NN = (size_t)N * N;
            CHECK((int)t.x.size() == N && (int)t.w.size() == N && finite(t.x) && finite(t.w), "leg points %d %d", basis, N);
            CHECK(t.fwd.size() == NN && t.bwd.size() == NN && t.sp.size() == NN, "leg sizes %d %d", basis, N);
            CHECK(finite(t.fwd) && finite(t.bwd) && finite(t.sp), "leg finite %d %d", basis, N);
            double wsum = 0;
            for (double w : t.w) wsum += w;
            CHECK(std::fabs(wsum - 2.0) < 1e-13, "leg weights sum %d %d", basis, N);
            const std::vector<double> pk = leg_pack(t.fwd, N);
            CHECK(pk.size() == leg_packed_doubles(N) && finite(pk), "leg pack %d %d", basis, N);
            if (basis == SGM_LEGENDRE) continue;
            // Galerkin rows against their closed forms (k the row's mode):
            // Dirichlet -A = 4k + 6; Neumann -A = (4k + 6) s_k with s_k = k(k+1)/((k+2)(k+3));
            // biharmonic S = 2 (2k+3)^2 (2k+5); Dirichlet / Neumann B diagonal
            for (int p = 0; p < 2; ++p) {
                CHECK(t.solve[p].size() == 20 * (size_t)t.npar[p] && finite(t.solve[p]), "leg solve %d %d", basis, N);
                for (int i = 0; i < t.npar[p]; ++i) {
                    const double k = p + 2 * i, *row = &t.solve[p][20 * (size_t)i];
                    const double sk = k * (k + 1) / ((k + 2) * (k + 3));
                    double want = 0, bdiag = 0;
                    if (basis == SGM_LEG_DIRICHLET) { want = 4 * k + 6; bdiag = 2 / (2 * k + 1) + 2 / (2 * k + 5); }
                    if (basis == SGM_LEG_NEUMANN) { want = (4 * k + 6) * sk; bdiag = 2 / (2 * k + 1) + sk * sk * 2 / (2 * k + 5); }
                    if (basis == SGM_LEG_BIHARMONIC) want = 2 * (2 * k + 3) * (2 * k + 3) * (2 * k + 5);
                    CHECK(std::fabs(row[2] - want) <= 1e-12 * std::fabs(want) + 1e-14, "leg row %d %d %d: %g vs %g", basis,
                          N, (int)k, row[2], want);
                    if (bdiag != 0) CHECK(std::fabs(row[7] - bdiag) <= 1e-13, "leg B %d %d %d", basis, N, (int)k);
                    for (int d : {0, 1, 3, 4}) CHECK(basis == SGM_LEG_BIHARMONIC || row[d] == 0.0 || std::fabs(row[d]) < 1e-12,
                                                     "leg -A off-diagonal %d %d %d", basis, N, (int)k);
                }
            }
        }
    if (fails) {
        std::printf("FAILED %d checks\n", fails);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
