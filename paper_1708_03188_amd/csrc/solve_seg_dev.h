// Device code of the segmented per-wavenumber Galerkin solves (header-only;
// used by the solve kernels and by the fused scalar-product + solve pass).
// The algorithm is described at the top of solve_seg.hip.
#pragma once
#include "kernels.h"

namespace sgm {
namespace segdev {

constexpr double kHalfPi = 1.5707963267948966192;

__device__ __forceinline__ int wnum(int q, int M) { return q < (M + 1) / 2 ? q : q - M; }

template <int KIND>
struct SegTraits {
    static constexpr int P = KIND == SGM_SHEN_BIHARMONIC ? 2 : 1;
    static constexpr int Q = P, S = P, NR = P;
    static constexpr int NC = Q + NR;      // c-state components
    static constexpr int WS = NC * P;      // w-state doubles
};

// Band, tail factors of row i < n of the chain of parity p (Chebyshev-Dirichlet,
// Chebyshev-Neumann and Legendre-Dirichlet in closed form, biharmonic from the
// plan's row table, 20 doubles per row).
template <int KIND>
__device__ __forceinline__ void row_coeffs(const double* rows, int p, int i, int n, double mu1, double mu2,
                                           double* band, double* U, double* V) {
    constexpr int P = SegTraits<KIND>::P, Q = SegTraits<KIND>::Q, NR = SegTraits<KIND>::NR;
    if constexpr (KIND == SGM_SHEN_DIRICHLET) {
        const double k = (double)(p + 2 * i);
        const double ck = (p + 2 * i) == 0 ? 2.0 : 1.0;
        band[0] = i >= 1 ? -mu1 * kHalfPi : 0.0;
        band[1] = 4.0 * kHalfPi * (k + 1.0) * (k + 2.0) + mu1 * kHalfPi * (ck + 1.0);
        band[2] = i + 1 < n ? -mu1 * kHalfPi : 0.0;
        U[0] = 8.0 * kHalfPi * (k + 1.0);
        V[0] = 1.0;
    } else if constexpr (KIND == SGM_SHEN_NEUMANN) {
        // r_k = (k/(k+2))^2: -A_kk = 4 (pi/2) k^2 (k+1)/(k+2), tail pi (1 - r_k) j^2;
        // B: (pi/2)(c_k + r_k^2) on the diagonal, -(pi/2) r_k right, -(pi/2) r_{k-2} left
        const double k = (double)(p + 2 * i);
        const double ck = (p + 2 * i) == 0 ? 2.0 : 1.0;
        const double q = k / (k + 2.0), rk = q * q;
        const double qm = (k - 2.0) / k;
        band[0] = i >= 1 ? -mu1 * kHalfPi * qm * qm : 0.0;
        band[1] = 4.0 * kHalfPi * k * k * (k + 1.0) / (k + 2.0) + mu1 * kHalfPi * (ck + rk * rk);
        band[2] = i + 1 < n ? -mu1 * kHalfPi * rk : 0.0;
        U[0] = 2.0 * kHalfPi * (1.0 - rk);
        V[0] = k * k;
    } else if constexpr (KIND == SGM_LEG_NEUMANN) {
        // s_k = k(k+1)/((k+2)(k+3)): -A = diag((4k + 6) s_k), B: 2/(2k+1) + s_k^2 2/(2k+5)
        // on the diagonal, -s_k 2/(2k+5) right, -s_{k-2} 2/(2k+1) left; no tail
        const double k = (double)(p + 2 * i);
        const double sk = k * (k + 1.0) / ((k + 2.0) * (k + 3.0));
        const double sm = (k - 2.0) * (k - 1.0) / (k * (k + 1.0));
        const double r1 = 2.0 / (2.0 * k + 1.0), r5 = 2.0 / (2.0 * k + 5.0);
        band[0] = i >= 1 ? -mu1 * sm * r1 : 0.0;
        band[1] = (4.0 * k + 6.0) * sk + mu1 * (r1 + sk * sk * r5);
        band[2] = i + 1 < n ? -mu1 * sk * r5 : 0.0;
        U[0] = 0.0;
        V[0] = 1.0;
    } else if constexpr (KIND == SGM_LEG_DIRICHLET) {
        // -A = diag(4k + 6), B: 2/(2k+1) + 2/(2k+5) on the diagonal, -2/(2k+5) and
        // -2/(2k+1) two places right and left; no tail
        const double k = (double)(p + 2 * i);
        const double r1 = 2.0 / (2.0 * k + 1.0), r5 = 2.0 / (2.0 * k + 5.0);
        band[0] = i >= 1 ? -mu1 * r1 : 0.0;
        band[1] = 4.0 * k + 6.0 + mu1 * (r1 + r5);
        band[2] = i + 1 < n ? -mu1 * r5 : 0.0;
        U[0] = 0.0;
        V[0] = 1.0;
    } else {
        const double2* row = reinterpret_cast<const double2*>(rows + 20 * i);
        double v[20];
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            const double2 t = row[j];
            v[2 * j] = t.x;
            v[2 * j + 1] = t.y;
        }
#pragma unroll
        for (int d = -P; d <= Q; ++d) band[d + P] = v[d + 2] + mu1 * v[7 + d] + mu2 * v[12 + d];
#pragma unroll
        for (int r = 0; r < NR; ++r) { U[r] = v[15 + r]; V[r] = v[17 + r]; }
    }
}

// 1/a for the pivots (well scaled, never denormal): hardware estimate and two
// Newton steps r <- r + r (1 - a r).
__device__ __forceinline__ double recip(double a) {
    double r = __builtin_amdgcn_rcp(a);
    double e = __builtin_fma(-a, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-a, r, 1.0);
    return __builtin_fma(r, e, r);
}

__device__ __forceinline__ void chain_mu(const ColGeom& g, int kind, int col, double alpha, double& mu1, double& mu2) {
    const int iy = col / g.nlast, iz = col - iy * g.nlast;
    const double m = g.Mmid > 1 ? (double)wnum(iy, g.Mmid) : 0.0;
    const double nn = g.last_r2c ? (double)iz : (double)wnum(iz, g.Mlast);
    const double k2 = g.sy * m * m + g.sz * nn * nn;
    const bool helm = kind != SGM_SHEN_BIHARMONIC;
    mu1 = helm ? k2 + alpha : -2.0 * k2;
    mu2 = helm ? 0.0 : k2 * k2;
}

// One step of the w recurrence (row i); returns 1/coef0 and b.
template <int KIND>
__device__ __forceinline__ double w_step(const double* band, const double* U, const double* V, const double* Vnext,
                                         bool inside, double (&wx)[SegTraits<KIND>::Q][SegTraits<KIND>::P],
                                         double (&ws)[SegTraits<KIND>::NR][SegTraits<KIND>::P],
                                         double (&b)[SegTraits<KIND>::P]) {
    constexpr int P = SegTraits<KIND>::P, Q = SegTraits<KIND>::Q, NR = SegTraits<KIND>::NR, S = SegTraits<KIND>::S;
    double coef[P + 1];
    coef[0] = band[P];
#pragma unroll
    for (int e = 1; e <= P; ++e) coef[e] = band[P - e];
#pragma unroll
    for (int d = 1; d <= Q; ++d)
#pragma unroll
        for (int e = 0; e < P; ++e) coef[e] += band[P + d] * wx[d - 1][e];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int e = 0; e < P; ++e) coef[e] += U[r] * ws[r][e];
    const double inv = recip(coef[0]);
#pragma unroll
    for (int e = 0; e < P; ++e) b[e] = -coef[e + 1] * inv;
    // new w of x_i, x_{i+1}, ..; rep substitution x_i -> b . window
    double nwx[Q][P];
#pragma unroll
    for (int e = 0; e < P; ++e) nwx[0][e] = b[e];
#pragma unroll
    for (int d = 1; d < Q; ++d)
#pragma unroll
        for (int e = 0; e < P; ++e) nwx[d][e] = wx[d - 1][0] * b[e] + (e + 1 < P ? wx[d - 1][e + 1] : 0.0);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const double Vt = S == 1 ? V[r] : Vnext[r];
        double o[P];
#pragma unroll
        for (int e = 0; e < P; ++e) o[e] = ws[r][0] * b[e] + (e + 1 < P ? ws[r][e + 1] : 0.0);
        if (inside)
#pragma unroll
            for (int e = 0; e < P; ++e) o[e] += Vt * nwx[S - 1][e];
#pragma unroll
        for (int e = 0; e < P; ++e) ws[r][e] = o[e];
    }
#pragma unroll
    for (int d = 0; d < Q; ++d)
#pragma unroll
        for (int e = 0; e < P; ++e) wx[d][e] = nwx[d][e];
    return inv;
}

template <int NC>
struct Aff {
    double2 h;
    double m[NC];
};

template <int NC>
__device__ __forceinline__ void aff_axpy(Aff<NC>& y, double s, const Aff<NC>& x) {
    y.h.x += s * x.h.x;
    y.h.y += s * x.h.y;
#pragma unroll
    for (int c = 0; c < NC; ++c) y.m[c] += s * x.m[c];
}

__device__ __forceinline__ void aff_axpy(double2& y, double s, const double2& x) {
    y.x += s * x.x;
    y.y += s * x.y;
}
template <int NC>
__device__ __forceinline__ void aff_scale(Aff<NC>& y, double s) {
    y.h.x *= s;
    y.h.y *= s;
#pragma unroll
    for (int c = 0; c < NC; ++c) y.m[c] *= s;
}
__device__ __forceinline__ void aff_scale(double2& y, double s) {
    y.x *= s;
    y.y *= s;
}

// One row of the bottom-up elimination for either c representation (Aff: c
// symbolic in the state entering the segment; double2: concrete).  On entry
// cst holds f_i; on exit it holds a_i, b the window coefficients of x_i.
template <int KIND, class CT>
__device__ __forceinline__ void elim_row(const double* band, const double* U, const double* V,
                                         double (&Vnext)[SegTraits<KIND>::NR], bool inside,
                                         double (&wx)[SegTraits<KIND>::Q][SegTraits<KIND>::P],
                                         double (&ws)[SegTraits<KIND>::NR][SegTraits<KIND>::P],
                                         CT (&cx)[SegTraits<KIND>::Q], CT (&cs)[SegTraits<KIND>::NR], CT& cst,
                                         double (&b)[SegTraits<KIND>::P]) {
    constexpr int P = SegTraits<KIND>::P, Q = SegTraits<KIND>::Q, NR = SegTraits<KIND>::NR, S = SegTraits<KIND>::S;
#pragma unroll
    for (int d = 1; d <= Q; ++d) aff_axpy(cst, -band[P + d], cx[d - 1]);
#pragma unroll
    for (int q = 0; q < NR; ++q) aff_axpy(cst, -U[q], cs[q]);
    double w0x[Q], w0s[NR];
#pragma unroll
    for (int d = 0; d < Q; ++d) w0x[d] = wx[d][0];
#pragma unroll
    for (int q = 0; q < NR; ++q) w0s[q] = ws[q][0];
    const double inv = w_step<KIND>(band, U, V, Vnext, inside, wx, ws, b);
    aff_scale(cst, inv);
    // x_i = a, x_{i+d} += w0 a, sigma_r += w0 a + V x_{i-1+S}
    CT ncx[Q];
    ncx[0] = cst;
#pragma unroll
    for (int d = 1; d < Q; ++d) {
        ncx[d] = cx[d - 1];
        aff_axpy(ncx[d], w0x[d - 1], cst);
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        aff_axpy(cs[q], w0s[q], cst);
        if (inside) aff_axpy(cs[q], S == 1 ? V[q] : Vnext[q], ncx[S - 1]);
    }
#pragma unroll
    for (int d = 0; d < Q; ++d) cx[d] = ncx[d];
#pragma unroll
    for (int q = 0; q < NR; ++q) Vnext[q] = V[q];
}

__device__ __forceinline__ double2 shfl_down2(double2 v, int d) {
    return make_double2(__shfl_down(v.x, d), __shfl_down(v.y, d));
}
__device__ __forceinline__ double2 shfl_up2(double2 v, int d) {
    return make_double2(__shfl_up(v.x, d), __shfl_up(v.y, d));
}

// Right-hand side rows read from global memory: f of chain row i (position
// p + 2 i) of column col.
struct GlobalRhs {
    const double2* in;
    int ncols;
    __device__ __forceinline__ double2 operator()(int p, int i, int col) const {
        return in[(long)(p + 2 * i) * ncols + col];
    }
};

// Solution rows to global memory: x of chain row i of column col, and the
// zero rows beyond the basis.
struct GlobalOut {
    double2* out;
    int ncols;
    __device__ __forceinline__ void operator()(int p, int i, int col, double2 v) const {
        out[(long)(p + 2 * i) * ncols + col] = v;
    }
    __device__ __forceinline__ void zero(int l, int col) const { out[(long)l * ncols + col] = make_double2(0.0, 0.0); }
};

// Solve the chains of wave gw (see k_solve_seg for the lane layout); f comes
// from rhs(p, i, col), x goes to out(p, i, col, x) and out.zero(l, col).
template <int KIND, int K, int R, class Rhs, class Out>
__device__ __forceinline__ void solve_wave(int gw, const Rhs& rhs, const Out& out, const double* tab,
                                           const ChebDev& cd, const ColGeom& g, double alpha,
                                           const double* rows0, const double* rows1) {
    using T = SegTraits<KIND>;
    constexpr int P = T::P, Q = T::Q, NR = T::NR, S = T::S, NC = T::NC, WS = T::WS;
    constexpr int C = 64 / K;
    const int lane = threadIdx.x & 63;
    const int ngroups = (g.ncols + C - 1) / C;
    const int p = gw / ngroups;
    const double* rows = p == 0 ? rows0 : rows1;
    const int seg = lane / C;
    const int col = (gw - p * ngroups) * C + (lane - seg * C);
    const bool act = col < g.ncols;
    const int ncols = g.ncols;
    const int n = cd.npar[p];
    const int lo = seg * R;
    double mu1, mu2;
    chain_mu(g, KIND, act ? col : 0, alpha, mu1, mu2);

    // 1. rows of the segment
    double2 fr[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
        fr[r] = (act && lo + r < n) ? rhs(p, lo + r, col) : make_double2(0.0, 0.0);

    // 2. incoming w state
    double wx0[Q][P], ws0[NR][P], Vn0[NR];
    {
        const bool has = act && seg < K - 1 && (seg + 1) * R < n;
        const double* t = tab + ((long)seg * 2 * ncols + (long)p * ncols + (act ? col : 0)) * WS;
#pragma unroll
        for (int d = 0; d < Q; ++d)
#pragma unroll
            for (int e = 0; e < P; ++e) wx0[d][e] = has ? t[d * P + e] : 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int e = 0; e < P; ++e) ws0[r][e] = has ? t[(Q + r) * P + e] : 0.0;
        double band[2 * P + 1], U[NR], V[NR];
        const int hi = (seg + 1) * R;
        if (S == 2 && hi < n) {
            row_coeffs<KIND>(rows, p, hi, n, mu1, mu2, band, U, V);
#pragma unroll
            for (int r = 0; r < NR; ++r) Vn0[r] = V[r];
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) Vn0[r] = 0.0;
        }
    }

    // 3. symbolic pass over the segment: its map c_out = H + Mat c_in
    Aff<NC> cx[Q], cs[NR];
    {
        double wx[Q][P], ws[NR][P], Vnext[NR];
#pragma unroll
        for (int d = 0; d < Q; ++d) {
            cx[d].h = make_double2(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < NC; ++c) cx[d].m[c] = c == d ? 1.0 : 0.0;
#pragma unroll
            for (int e = 0; e < P; ++e) wx[d][e] = wx0[d][e];
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            cs[r].h = make_double2(0.0, 0.0);
#pragma unroll
            for (int c = 0; c < NC; ++c) cs[r].m[c] = c == Q + r ? 1.0 : 0.0;
#pragma unroll
            for (int e = 0; e < P; ++e) ws[r][e] = ws0[r][e];
            Vnext[r] = Vn0[r];
        }
#pragma unroll
        for (int r = R - 1; r >= 0; --r) {
            const int i = lo + r;
            if (i < n) {
                double band[2 * P + 1], U[NR], V[NR], b[P];
                row_coeffs<KIND>(rows, p, i, n, mu1, mu2, band, U, V);
                Aff<NC> cst;
                cst.h = fr[r];
#pragma unroll
                for (int c = 0; c < NC; ++c) cst.m[c] = 0.0;
                elim_row<KIND>(band, U, V, Vnext, (i - 1 + S) < n, wx, ws, cx, cs, cst, b);
            }
        }
    }

    // 4. scan up the chain: c_in of segment s = map of segment s+1 applied to its c_in
    double2 cin[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) cin[c] = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < K - 1; ++t) {
        double2 cout[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const Aff<NC>& src = j < Q ? cx[j] : cs[j - Q];
            double2 v = src.h;
#pragma unroll
            for (int c = 0; c < NC; ++c) { v.x += src.m[c] * cin[c].x; v.y += src.m[c] * cin[c].y; }
            cout[j] = v;
        }
#pragma unroll
        for (int j = 0; j < NC; ++j) {
            const double2 v = shfl_down2(cout[j], C);
            cin[j] = seg == K - 1 ? make_double2(0.0, 0.0) : v;
        }
    }

    // 5. concrete pass from the exact entering state: a_i (over f_i) and b_i
    double bb[R][P];
    {
        double wx[Q][P], ws[NR][P], Vnext[NR];
        double2 cx2[Q], cs2[NR];
#pragma unroll
        for (int d = 0; d < Q; ++d) {
            cx2[d] = cin[d];
#pragma unroll
            for (int e = 0; e < P; ++e) wx[d][e] = wx0[d][e];
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            cs2[r] = cin[Q + r];
#pragma unroll
            for (int e = 0; e < P; ++e) ws[r][e] = ws0[r][e];
            Vnext[r] = Vn0[r];
        }
#pragma unroll
        for (int r = R - 1; r >= 0; --r) {
            const int i = lo + r;
#pragma unroll
            for (int e = 0; e < P; ++e) bb[r][e] = 0.0;
            if (i < n) {
                double band[2 * P + 1], U[NR], V[NR];
                row_coeffs<KIND>(rows, p, i, n, mu1, mu2, band, U, V);
                elim_row<KIND>(band, U, V, Vnext, (i - 1 + S) < n, wx, ws, cx2, cs2, fr[r], bb[r]);
            }
        }
    }

    // 6. top-down recovery, symbolic in the window entering the segment
    Aff<P> win[P];
#pragma unroll
    for (int e = 0; e < P; ++e) {
        win[e].h = make_double2(0.0, 0.0);
#pragma unroll
        for (int c = 0; c < P; ++c) win[e].m[c] = c == e ? 1.0 : 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        Aff<P> x;
        x.h = fr[r];
#pragma unroll
        for (int c = 0; c < P; ++c) x.m[c] = 0.0;
#pragma unroll
        for (int e = 0; e < P; ++e) aff_axpy(x, bb[r][e], win[e]);
#pragma unroll
        for (int e = P - 1; e > 0; --e) win[e] = win[e - 1];
        win[0] = x;
    }
    double2 zin[P];
#pragma unroll
    for (int e = 0; e < P; ++e) zin[e] = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < K - 1; ++t) {
        double2 zout[P];
#pragma unroll
        for (int e = 0; e < P; ++e) {
            double2 v = win[e].h;
#pragma unroll
            for (int c = 0; c < P; ++c) { v.x += win[e].m[c] * zin[c].x; v.y += win[e].m[c] * zin[c].y; }
            zout[e] = v;
        }
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const double2 v = shfl_up2(zout[e], C);
            zin[e] = seg == 0 ? make_double2(0.0, 0.0) : v;
        }
    }

    // 7. final sweep
    double2 w[P];
#pragma unroll
    for (int e = 0; e < P; ++e) w[e] = zin[e];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = lo + r;
        double2 x = fr[r];
#pragma unroll
        for (int e = 0; e < P; ++e) { x.x += bb[r][e] * w[e].x; x.y += bb[r][e] * w[e].y; }
        if (act && i < n) out(p, i, col, x);
#pragma unroll
        for (int e = P - 1; e > 0; --e) w[e] = w[e - 1];
        w[0] = x;
    }
    // rows beyond the basis of this parity are zero
    if (act)
        for (int l = p + 2 * n + 2 * seg; l < cd.N; l += 2 * K) out.zero(l, col);
}

}  // namespace segdev
}  // namespace sgm
