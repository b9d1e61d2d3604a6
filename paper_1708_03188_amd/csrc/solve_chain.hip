// Per-wavenumber Galerkin solves, one lane per (column, parity) chain.
//
// Lane -> (column c, parity p): a block of 256 threads covers 128 adjacent
// columns for both parities, so each row access of a wave is 64 adjacent
// complex values.  The system of one chain is
//   M x = f,  M = T0 + mu1 T1 + mu2 T2 (band, offsets -P..Q) + sum_r U_r(i) V_r(j) [j >= i + S]
// (Helmholtz, Shen-Dirichlet: P = Q = S = 1, one tail term, coefficients in
// closed form; biharmonic: P = Q = S = 2, two tail terms, plan tables).
// Bottom-up elimination keeps x_{i+1..i+Q} and the tail sums
// sigma_r(i+S) = sum_{j >= i+S} V_r(j) x_j as affine functions of the window
// (x_i .. x_{i-P+1}); row i then gives x_i = a_i + sum_e b_{i,e} x_{i-e}.  a_i
// goes to the output array, b_i to the plan workspace, and a top-down sweep
// recovers x in place.
#include "fft_lds.h"
#include "kernels.h"
#include "solve_chain.h"

namespace sgm {

template <int P>
struct RepC {
    double2 c;
    double w[P];
};

__device__ __forceinline__ int wavenum(int q, int M) { return q < (M + 1) / 2 ? q : q - M; }

template <int KIND>
__global__ void __launch_bounds__(256) k_solve_chain(const double2* in, double2* out, double* scr, ChebDev cd,
                                                     ColGeom g, double alpha) {
    constexpr int P = KIND == SGM_SHEN_DIRICHLET ? 1 : 2;
    constexpr int Q = P, S = P, NR = P;
    const int ncols = g.ncols;
    const int half = blockDim.x / 2;
    const int col = blockIdx.x * half + (threadIdx.x % half);
    const int p = threadIdx.x / half;
    if (col >= ncols) return;
    const int N = cd.N;
    const int n = cd.npar[p];
    const int iy = col / g.nlast, iz = col - iy * g.nlast;
    const double m = g.Mmid > 1 ? (double)wavenum(iy, g.Mmid) : 0.0;
    const double nn = g.last_r2c ? (double)iz : (double)wavenum(iz, g.Mlast);
    const double k2 = g.sy * m * m + g.sz * nn * nn;
    const double mu1 = KIND == SGM_SHEN_DIRICHLET ? k2 + alpha : -2.0 * k2;
    const double mu2 = KIND == SGM_SHEN_DIRICHLET ? 0.0 : k2 * k2;
    const long stride = 2L * ncols;  // between consecutive rows of one parity
    const long base = (long)p * ncols + col;
    const double* tab = cd.solve[p];
    const double hpi = 1.5707963267948966192;

    RepC<P> rx[Q];
    RepC<P> rs[NR];
#pragma unroll
    for (int d = 0; d < Q; ++d) { rx[d].c = make_double2(0.0, 0.0); for (int e = 0; e < P; ++e) rx[d].w[e] = 0.0; }
#pragma unroll
    for (int r = 0; r < NR; ++r) { rs[r].c = make_double2(0.0, 0.0); for (int e = 0; e < P; ++e) rs[r].w[e] = 0.0; }
    double Vnext[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) Vnext[r] = 0.0;

    for (int i = n - 1; i >= 0; --i) {
        const long idx = base + (long)i * stride;
        const double2 f = in[idx];
        double band[P + Q + 1];
        double U[NR], V[NR];
        if constexpr (KIND == SGM_SHEN_DIRICHLET) {
            const double k = (double)(p + 2 * i);
            const double ck = (p + 2 * i) == 0 ? 2.0 : 1.0;
            band[0] = i >= 1 ? -mu1 * hpi : 0.0;
            band[1] = 4.0 * hpi * (k + 1.0) * (k + 2.0) + mu1 * hpi * (ck + 1.0);
            band[2] = i + 1 < n ? -mu1 * hpi : 0.0;
            U[0] = 8.0 * hpi * (k + 1.0);
            V[0] = 1.0;
        } else {
            const double* row = tab + 20 * i;
#pragma unroll
            for (int d = -P; d <= Q; ++d) band[d + P] = row[d + 2] + mu1 * row[5 + d + 2] + mu2 * row[10 + d + 2];
#pragma unroll
            for (int r = 0; r < NR; ++r) { U[r] = row[15 + r]; V[r] = row[17 + r]; }
        }
        double coef[P + 1];
        coef[0] = band[P];
#pragma unroll
        for (int e = 1; e <= P; ++e) coef[e] = band[P - e];
        double2 cst = f;
#pragma unroll
        for (int d = 1; d <= Q; ++d) {
            const double bd = band[P + d];
            cst.x -= bd * rx[d - 1].c.x; cst.y -= bd * rx[d - 1].c.y;
#pragma unroll
            for (int e = 0; e < P; ++e) coef[e] += bd * rx[d - 1].w[e];
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            cst.x -= U[r] * rs[r].c.x; cst.y -= U[r] * rs[r].c.y;
#pragma unroll
            for (int e = 0; e < P; ++e) coef[e] += U[r] * rs[r].w[e];
        }
        const double inv = 1.0 / coef[0];
        const double2 a = make_double2(cst.x * inv, cst.y * inv);
        double b[P];
#pragma unroll
        for (int e = 0; e < P; ++e) b[e] = -coef[e + 1] * inv;
        out[idx] = a;
#pragma unroll
        for (int e = 0; e < P; ++e) scr[2 * idx + e] = b[e];
        auto subst = [&](const RepC<P>& q) {
            RepC<P> o;
            o.c = make_double2(q.c.x + q.w[0] * a.x, q.c.y + q.w[0] * a.y);
#pragma unroll
            for (int e = 0; e < P; ++e) o.w[e] = q.w[0] * b[e] + (e + 1 < P ? q.w[e + 1] : 0.0);
            return o;
        };
        RepC<P> nrx[Q];
        nrx[0].c = a;
#pragma unroll
        for (int e = 0; e < P; ++e) nrx[0].w[e] = b[e];
#pragma unroll
        for (int d = 1; d < Q; ++d) nrx[d] = subst(rx[d - 1]);
        const bool inside = (i - 1 + S) < n;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double Vt = (S == 1) ? V[r] : Vnext[r];
            RepC<P> o = subst(rs[r]);
            if (inside) {
                const RepC<P>& xs = nrx[S - 1];
                o.c.x += Vt * xs.c.x; o.c.y += Vt * xs.c.y;
#pragma unroll
                for (int e = 0; e < P; ++e) o.w[e] += Vt * xs.w[e];
            }
            rs[r] = o;
        }
#pragma unroll
        for (int d = 0; d < Q; ++d) rx[d] = nrx[d];
#pragma unroll
        for (int r = 0; r < NR; ++r) Vnext[r] = V[r];
    }
    double2 hist[P];
#pragma unroll
    for (int e = 0; e < P; ++e) hist[e] = make_double2(0.0, 0.0);
    for (int i = 0; i < n; ++i) {
        const long idx = base + (long)i * stride;
        double2 x = out[idx];
#pragma unroll
        for (int e = 0; e < P; ++e) {
            const double be = scr[2 * idx + e];
            x.x += be * hist[e].x; x.y += be * hist[e].y;
        }
        out[idx] = x;
#pragma unroll
        for (int e = P - 1; e > 0; --e) hist[e] = hist[e - 1];
        hist[0] = x;
    }
    // rows beyond the basis of this parity are zero
    for (int l = p + 2 * n; l < N; l += 2) out[(long)l * ncols + col] = make_double2(0.0, 0.0);
}

hipError_t launch_solve_chain(const double2* in, double2* out, double* scratch, const ChebDev& cd, const ColGeom& g,
                              int kind, double alpha, hipStream_t s) {
    const int threads = 256;
    const int blocks = (g.ncols + threads / 2 - 1) / (threads / 2);
    if (kind == SGM_SHEN_DIRICHLET)
        hipLaunchKernelGGL(k_solve_chain<SGM_SHEN_DIRICHLET>, dim3(blocks), dim3(threads), 0, s, in, out, scratch, cd,
                           g, alpha);
    else
        hipLaunchKernelGGL(k_solve_chain<SGM_SHEN_BIHARMONIC>, dim3(blocks), dim3(threads), 0, s, in, out, scratch,
                           cd, g, alpha);
    return hipGetLastError();
}

}  // namespace sgm
