// Plan constants for the Fourier and Chebyshev/Shen axes.
//
// Everything here is computed once per plan on the host in long double
// (x87, 64-bit significand) and rounded to binary64 when uploaded.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/sgm.h"
#include "common.h"

#include "tables.h"

namespace sgm {

using ld = long double;
static const ld PI_L = 3.141592653589793238462643383279502884L;

int factor_radices(int L, int* radix) {
    int n = 0;
    int a = 0;
    while (L % 2 == 0) { L /= 2; ++a; }
    // powers of two: as many radix-8 stages as possible, remainder as 4 / 4x4 / 2
    int r8 = a / 3, rem = a % 3;
    if (rem == 1 && r8 > 0) { --r8; radix[n++] = 4; radix[n++] = 4; }
    else if (rem == 1) radix[n++] = 2;
    else if (rem == 2) radix[n++] = 4;
    for (int i = 0; i < r8; ++i) radix[n++] = 8;
    for (int p : {3, 5, 7}) {
        while (L % p == 0) { radix[n++] = p; L /= p; }
    }
    for (int p = 11; L > 1; p += 2) {
        while (L % p == 0) { radix[n++] = p; L /= p; }
        if ((long)p * p > L && L > 1) { radix[n++] = L; L = 1; }
    }
    return n;
}

std::vector<double> twiddles(int L) {
    std::vector<double> t(2 * (size_t)L);
    for (int r = 0; r < L; ++r) {
        ld ang = -2 * PI_L * (ld)r / (ld)L;
        t[2 * r] = (double)cosl(ang);
        t[2 * r + 1] = (double)sinl(ang);
    }
    return t;
}

// ---- exact Chebyshev inner products -------------------------------------
// (T_n'', T_m)_w / (pi/2) = n (n^2 - m^2) for m <= n-2, n-m even, else 0.
static ld g2(long n, long m) {
    if (m > n - 2 || ((n - m) & 1)) return 0;
    return (ld)n * (ld)(n * n - m * m);
}
// (T_n'''', T_m)_w / (pi/2) = sum_{p=m+2, step 2}^{n-2} n (n^2-p^2) p (p^2-m^2), exact integers.
static ld g4(long n, long m) {
    if (m > n - 4 || ((n - m) & 1)) return 0;
    __int128 s = 0;
    for (long p = m + 2; p <= n - 2; p += 2) s += (__int128)n * (n * n - p * p) * p * (p * p - m * m);
    return (ld)s;
}
static ld g0(long n, long m) { return n == m ? (m == 0 ? 2 : 1) : 0; }

struct Comp {
    int cnt;
    long k[3];
    ld c[3];
};
static Comp composite(int basis, long l) {
    Comp c{};
    c.k[0] = l; c.c[0] = 1; c.cnt = 1;
    if (basis == SGM_SHEN_DIRICHLET) { c.k[1] = l + 2; c.c[1] = -1; c.cnt = 2; }
    if (basis == SGM_SHEN_BIHARMONIC) {
        c.k[1] = l + 2; c.c[1] = -(ld)(2 * (l + 2)) / (ld)(l + 3);
        c.k[2] = l + 4; c.c[2] = (ld)(l + 1) / (ld)(l + 3);
        c.cnt = 3;
    }
    if (basis == SGM_SHEN_NEUMANN) {
        c.k[1] = l + 2; c.c[1] = -((ld)l / (ld)(l + 2)) * ((ld)l / (ld)(l + 2)); c.cnt = 2;
    }
    return c;
}
// (phi_j^(d), phi_k)_w / (pi/2) for the composite basis, by the formulas above.
static ld entry(int basis, ld (*g)(long, long), long k, long j) {
    Comp a = composite(basis, j), b = composite(basis, k);
    ld s = 0;
    for (int x = 0; x < a.cnt; ++x)
        for (int y = 0; y < b.cnt; ++y) s += a.c[x] * b.c[y] * g(a.k[x], b.k[y]);
    return s;
}

bool build_cheb_tables(int basis, int N, ChebTables& t, std::string& err) {
    t.basis = basis;
    t.N = N;
    int nb = (basis == SGM_SHEN_DIRICHLET || basis == SGM_SHEN_NEUMANN) ? N - 2 : basis == SGM_SHEN_BIHARMONIC ? N - 4
                                                                                                      : N;
    if (nb < 1) { err = "N too small for the basis"; return false; }
    t.nb = nb;
    for (int p = 0; p < 2; ++p) {
        t.npar[p] = nb > p ? (nb - p + 1) / 2 : 0;
        t.mpar[p] = N > p ? (N - p + 1) / 2 : 0;
    }
    t.theta.resize(2 * (size_t)N);
    t.beta.assign(N, 0.0);
    t.gamma.assign(N, 0.0);
    t.bscale.resize(N);
    t.fscale.resize(N);
    for (int k = 0; k < N; ++k) {
        ld ang = -PI_L * (ld)k / (ld)(2 * N);
        t.theta[2 * k] = (double)cosl(ang);
        t.theta[2 * k + 1] = (double)sinl(ang);
        ld ck = k == 0 ? 2 : 1;
        t.bscale[k] = (double)(sqrtl(2 * PI_L / ck) / (ld)N);
        t.fscale[k] = (double)(2 / (ck * (ld)N));
    }
    for (int l = 0; l < nb; ++l) {
        Comp c = composite(basis, l);
        if (c.cnt > 1) t.beta[l] = (double)c.c[1];
        if (c.cnt > 2) t.gamma[l] = (double)c.c[2];
    }
    if (basis == SGM_SHEN_NEUMANN) {
        // Galerkin rows (layout of the solver rows below), Chebyshev weight, with
        // r_k = (k / (k+2))^2: -A_kk = 2 pi k^2 (k+1) / (k+2), -A_kj = pi (1 - r_k) j^2
        // for j >= k + 2 (rank one: U = pi (1 - r_k), V = j^2), B_kk = (pi/2)(c_k + r_k^2),
        // B_{k,k+2} = B_{k+2,k} = -(pi/2) r_k
        const ld h = PI_L / 2;
        for (int p = 0; p < 2; ++p) {
            const int n = t.npar[p];
            std::vector<double>& S = t.solve[p];
            S.assign(20 * (size_t)n, 0.0);
            for (int i = 0; i < n; ++i) {
                const long k = p + 2 * i;
                const ld rk = ((ld)k / (ld)(k + 2)) * ((ld)k / (ld)(k + 2));
                const ld ck = k == 0 ? 2 : 1;
                double* row = &S[20 * (size_t)i];
                row[2] = (double)(2 * PI_L * (ld)k * (ld)k * (ld)(k + 1) / (ld)(k + 2));
                row[7] = (double)(h * (ck + rk * rk));
                if (i + 1 < n) row[8] = (double)(-h * rk);
                if (i > 0) {
                    const ld rm = ((ld)(k - 2) / (ld)k) * ((ld)(k - 2) / (ld)k);
                    row[6] = (double)(-h * rm);
                }
                row[15] = (double)(PI_L * (1 - rk));
                row[17] = (double)((ld)k * (ld)k);
            }
        }
        t.solve_s = 1;
        t.solve_rank = 1;
    }
    // the regular basis needs no projection tables; the Neumann projection runs from
    // the Chebyshev coefficients in closed form (derivative pass)
    if (basis == SGM_CHEBYSHEV || basis == SGM_SHEN_NEUMANN) return true;

    // ---- Givens QR of D^{1/2} P per parity (banded least squares) ----------
    const int nrot = basis == SGM_SHEN_DIRICHLET ? 1 : 2;
    for (int p = 0; p < 2; ++p) {
        int n = t.npar[p], m = t.mpar[p];
        // band storage: row r keeps columns r-2 .. r+3
        const int W = 6, OFF = 2;
        std::vector<ld> A((size_t)m * W, 0), rot(4 * (size_t)n, 0), rt(3 * (size_t)n, 0);
        auto at = [&](int r, int c) -> ld& { return A[(size_t)r * W + (c - r + OFF)]; };
        for (int i = 0; i < n; ++i) {
            long l = p + 2 * i;
            Comp c = composite(basis, l);
            for (int x = 0; x < c.cnt; ++x) {
                long k = c.k[x];
                int r = (int)((k - p) / 2);
                ld Dk = (k == 0 ? PI_L : PI_L / 2);
                at(r, i) = sqrtl(Dk) * c.c[x];
            }
        }
        for (int i = 0; i < n; ++i) {
            for (int q = 1; q <= nrot; ++q) {
                int r = i + q;
                ld a = at(i, i), b = (r < m) ? at(r, i) : 0;
                ld h = hypotl(a, b);
                ld cc = a / h, ss = b / h;
                for (int col = i; col <= i + 3 && col < n; ++col) {
                    if (col - r + OFF < 0 || col - r + OFF >= W) continue;
                    ld x = at(i, col), y = (r < m) ? at(r, col) : 0;
                    at(i, col) = cc * x + ss * y;
                    if (r < m) at(r, col) = -ss * x + cc * y;
                }
                rot[4 * i + 2 * (q - 1)] = cc;
                rot[4 * i + 2 * (q - 1) + 1] = ss;
            }
            rt[3 * i] = 1 / at(i, i);
            rt[3 * i + 1] = (i + 1 < n) ? at(i, i + 1) : 0;
            rt[3 * i + 2] = (i + 2 < n) ? at(i, i + 2) : 0;
        }
        t.rot[p].assign(rot.begin(), rot.end());
        t.rtab[p].assign(rt.begin(), rt.end());
        if (nrot == 2) {
            // segment maps of both sweeps, from the binary64 factors the kernels use
            const int R = kProjSegRows, nseg = (n + R - 1) / R;
            const std::vector<double>& ro = t.rot[p];
            const std::vector<double>& rr = t.rtab[p];
            t.gal[p].assign(2 * (size_t)n, 0.0);
            t.bal[p].assign(2 * (size_t)n, 0.0);
            t.gmat[p].assign(4 * (size_t)nseg, 0.0);
            t.bmat[p].assign(4 * (size_t)nseg, 0.0);
            for (int u = 0; u < nseg; ++u) {
                const int lo = u * R, hi = std::min(n, lo + R);
                for (int cu = 0; cu < 2; ++cu) {
                    // Givens sweep: state (w0, w1) entering row lo, no fresh input
                    ld a = cu == 0, b = cu == 1;
                    for (int i = lo; i < hi; ++i) {
                        const ld c1 = ro[4 * i], s1 = ro[4 * i + 1], c2 = ro[4 * i + 2], s2 = ro[4 * i + 3];
                        const ld a1 = c1 * a + s1 * b, b1 = -s1 * a + c1 * b;
                        t.gal[p][2 * i + cu] = (double)(c2 * a1);
                        a = b1;
                        b = -s2 * a1;
                    }
                    t.gmat[p][4 * u + cu] = (double)a;
                    t.gmat[p][4 * u + 2 + cu] = (double)b;
                    // back substitution: (x_hi, x_hi+1) entering, rows hi-1 .. lo
                    std::vector<ld> x((size_t)(hi - lo + 2), 0);
                    x[hi - lo] = cu == 0;
                    x[hi - lo + 1] = cu == 1;
                    for (int i = hi - 1; i >= lo; --i) {
                        const ld v = (-(ld)rr[3 * i + 1] * x[i - lo + 1] - (ld)rr[3 * i + 2] * x[i - lo + 2]) * (ld)rr[3 * i];
                        x[i - lo] = v;
                        t.bal[p][2 * i + cu] = (double)v;
                    }
                    t.bmat[p][4 * u + cu] = (double)x[0];
                    t.bmat[p][4 * u + 2 + cu] = (double)x[1];
                }
            }
        }
        // Boundary functionals of parity p: sum_k c_k (u(1) +- u(-1)) and, for the
        // biharmonic basis, sum_k k^2 c_k (u'(1) -+ u'(-1)).  Range(P) is their null
        // space; in b = D^{1/2} c coordinates the functionals are D^{-1/2} C^T, with
        // D proportional to diag(c_k).  Gram-Schmidt (twice) gives an orthonormal basis.
        std::vector<ld> y[2];
        for (int r = 0; r < nrot; ++r) {
            y[r].resize(m);
            for (int tt = 0; tt < m; ++tt) {
                long k = p + 2 * tt;
                ld ck = k == 0 ? 2 : 1;
                y[r][tt] = (r == 0 ? 1.0L : (ld)k * (ld)k) / sqrtl(ck);
            }
            for (int pass = 0; pass < 2; ++pass)
                for (int q = 0; q < r; ++q) {
                    ld d = 0;
                    for (int tt = 0; tt < m; ++tt) d += y[q][tt] * y[r][tt];
                    for (int tt = 0; tt < m; ++tt) y[r][tt] -= d * y[q][tt];
                }
            ld nn = 0;
            for (int tt = 0; tt < m; ++tt) nn += y[r][tt] * y[r][tt];
            nn = sqrtl(nn);
            for (int tt = 0; tt < m; ++tt) y[r][tt] /= nn;
        }
        t.qtab[p].assign(2 * (size_t)m, 0.0);
        for (int tt = 0; tt < m; ++tt)
            for (int r = 0; r < nrot; ++r) t.qtab[p][2 * tt + r] = (double)y[r][tt];
    }

    // ---- Galerkin solver rows ---------------------------------------------
    const ld h = PI_L / 2;
    for (int p = 0; p < 2; ++p) {
        int n = t.npar[p];
        std::vector<double>& S = t.solve[p];
        S.assign(20 * (size_t)n, 0.0);
        for (int i = 0; i < n; ++i) {
            long k = p + 2 * i;
            double* row = &S[20 * (size_t)i];
            auto lidx = [&](int d) { return k + 2 * d; };  // column basis index at parity offset d
            if (basis == SGM_SHEN_DIRICHLET) {
                // T0 = -A: diagonal 2 pi (k+1)(k+2); tail -A_kj = 4 pi (k+1) for j > k (offset >= 1).
                row[0 + 2] = (double)(2 * PI_L * (ld)(k + 1) * (ld)(k + 2));
                // T1 = B: (pi/2)(c_k + 1) on the diagonal, -pi/2 at offsets +-1.
                for (int d = -2; d <= 2; ++d) {
                    int ii = i + d;
                    if (ii < 0 || ii >= n) continue;
                    row[5 + d + 2] = (double)(h * entry(basis, g0, k, lidx(d)));
                }
                row[15] = (double)(4 * PI_L * (ld)(k + 1));
                row[17] = 1.0;
            } else {
                // T0 = S (offsets 0, +1 explicit, >= 2 separable), T1 = A, T2 = B.
                for (int d = 0; d <= 1; ++d)
                    if (i + d < n) row[0 + d + 2] = (double)(h * entry(basis, g4, k, lidx(d)));
                for (int d = -2; d <= 2; ++d) {
                    int ii = i + d;
                    if (ii < 0 || ii >= n) continue;
                    row[5 + d + 2] = (double)(h * entry(basis, g2, k, lidx(d)));
                    row[10 + d + 2] = (double)(h * entry(basis, g0, k, lidx(d)));
                }
                // Separable tail: S_kj = (pi/2) [U3(k) V3(j) + U4(k) V4(j)], j >= k + 4, with
                // U3 = sum_b P_{k+b,k} (k+b)^4, U4 = sum_b P_{k+b,k} ((k+b)^6 - 8 (k+b)^4),
                // V3 = sum_a P_{j+a,j} 3 (j+a)^3 / 24, V4 = -sum_a P_{j+a,j} (j+a) / 24.
                // Numerators over (k+3) are exact 128-bit integers.
                auto num = [&](long kk, auto f) {
                    __int128 v = (__int128)(kk + 3) * f(kk) - (__int128)2 * (kk + 2) * f(kk + 2) +
                                 (__int128)(kk + 1) * f(kk + 4);
                    return (ld)v / (ld)(kk + 3);
                };
                auto p4 = [](long q) { return (__int128)q * q * q * q; };
                auto p64 = [](long q) { __int128 q2 = (__int128)q * q; return q2 * q2 * q2 - 8 * q2 * q2; };
                auto p3 = [](long q) { return (__int128)q * q * q; };
                auto p1 = [](long q) { return (__int128)q; };
                row[15] = (double)(h * num(k, p4));
                row[16] = (double)(h * num(k, p64));
                row[17] = (double)(3 * num(k, p3) / 24);
                row[18] = (double)(-num(k, p1) / 24);
            }
        }
    }
    t.solve_s = basis == SGM_SHEN_DIRICHLET ? 1 : 2;
    t.solve_rank = basis == SGM_SHEN_DIRICHLET ? 1 : 2;
    return true;
}

}  // namespace sgm
