// Spectral derivative and projection pass (Sec. 5: the Dx operator, nested for
// mixed derivatives, and project onto a regular, Shen-Dirichlet or Shen-Neumann
// space of the Chebyshev or the Legendre family).
//
// One work-group takes 16 adjacent spectral columns; each column is split into
// 16 chunks of E consecutive rows, one thread per chunk, so every row access of a
// wave is a run of 16 columns (256 bytes).  Per column:
//   1. Chebyshev coefficients of the source function (Shen recombination,
//      a_k = u_k + beta_{k-2} u_{k-2} + gamma_{k-4} u_{k-4});
//   2. ox times the coefficient form of d/dx: with u = sum a_k T_k,
//      u' = sum b_k T_k, b_k = (2 / c_k) sum_{p > k, p - k odd} p a_p (c_0 = 2,
//      else 1): a suffix sum per parity class, combined across chunks in LDS;
//   3. the Fourier factors (i k_y)^oy (i k_z)^oz of the column;
//   4. onto the regular Chebyshev space the result is the coefficients b
//      themselves (the derivative is a polynomial of degree < N and Gauss
//      quadrature is exact); onto the Shen-Dirichlet space, the weighted L2
//      projection: with w_0 = 1/2, w_k = 1, subtract lambda_p w_k per parity
//      (lambda_p = sum_{k in p} b_k / sum_{k in p} w_k, which makes the
//      coefficients vanish at x = +-1) and sum the result along each parity
//      (u_l = sum_{k <= l, k = l mod 2} (b_k - lambda_p w_k), the inverse of the
//      recombination T_l - T_{l+2}); onto the Shen-Neumann space
//      (T_l - (l/(l+2))^2 T_{l+2}), the same with the constraint u'(+-1) = 0,
//      sum_{k in p} k^2 a_k = 0: a_k = b_k - mu_p k^2 with
//      mu_p = sum_{k in p} k^2 b_k / sum_{k in p} k^4, then
//      u_l = (1 / l^2) sum_{k <= l, k = l mod 2} k^2 a_k (l >= 1; u_0 = a_0), which
//      inverts a_k = u_k - ((k-2)/k)^2 u_{k-2}.
// The Legendre family (coefficients of L_k, weight 1) takes the same steps with
// its own constants: d/dx gives b_k = (2k + 1) sum_{p > k, p - k odd} a_p; the
// functions orthogonal to the Dirichlet space L_l - L_{l+2} have coefficients
// proportional per parity to h_k = (2k + 1) / 2 (the inverse squared norm of L_k;
// Chebyshev: w_k above), and those orthogonal to the Neumann space
// L_l - (l(l+1) / ((l+2)(l+3))) L_{l+2} to q_k h_k with q_k = k(k+1)
// (L_k'(1) = q_k / 2; Chebyshev: q_k = k^2, h_k = 1).  So the Dirichlet target
// subtracts lambda_p h_k, lambda_p = sum_{k in p} b_k / sum_{k in p} h_k, and the
// Neumann target subtracts mu_p q_k h_k, mu_p = sum_{k in p} q_k b_k /
// sum_{k in p} q_k^2 h_k, then u_l = (1 / q_l) sum_{k <= l, k = l mod 2} q_k a_k.
// The cross-chunk sums go through LDS: one thread per (parity, column) scans the
// 16 chunk partials serially.
#include "derivative.h"

namespace sgm {

namespace {

constexpr int kT = 16;  // chunks (threads) per column
constexpr int kW = 16;  // columns per work-group

__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 cscale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// (i k s)^o for stored index q of an axis of M points (FFT order; R2C keeps
// 0..M/2); odd orders of the Nyquist coefficient (q = M/2, M even) are zero.
__device__ inline double2 axis_factor(int q, int M, int r2c, int o, double s) {
    if (o == 0) return make_double2(1.0, 0.0);
    if ((M & 1) == 0 && 2 * q == M && (o & 1)) return make_double2(0.0, 0.0);
    const int k = (r2c || q < (M + 1) / 2) ? q : q - M;
    const double ks = (double)k * s;
    double mag = 1.0;
    for (int i = 0; i < o; ++i) mag *= ks;
    switch (o & 3) {
        case 0: return make_double2(mag, 0.0);
        case 1: return make_double2(0.0, mag);
        case 2: return make_double2(-mag, 0.0);
        default: return make_double2(0.0, -mag);
    }
}

template <int E>
__global__ __launch_bounds__(256) void k_dx_project(const double2* __restrict__ in, double2* __restrict__ out,
                                                     DxArgs a) {
    __shared__ double2 part[2][kT][kW];
    __shared__ double2 total[2][kW];
    const int c = threadIdx.x % kW, j = threadIdx.x / kW;
    const long col = (long)blockIdx.x * kW + c;
    const bool live = col < a.ncols;
    const long ld = a.ncols;
    const int N = a.N, nb = a.nb_src, r0 = j * E;

    double2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = r0 + e;
        v[e] = (live && k < nb) ? in[k * ld + col] : make_double2(0.0, 0.0);
    }
    const bool leg = a.leg != 0;
    // 1. Chebyshev (Legendre) coefficients (descending, so u_{k-2} and u_{k-4} are
    //    still the inputs)
    if (a.src_basis != SGM_CHEBYSHEV && a.src_basis != SGM_LEGENDRE) {
        double2 h[4];  // u_{r0-4} .. u_{r0-1}
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = r0 - 4 + q;
            h[q] = (live && k >= 0 && k < nb) ? in[k * ld + col] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int e = E - 1; e >= 0; --e) {
            const int k = r0 + e;
            const double2 u2 = e >= 2 ? v[e >= 2 ? e - 2 : 0] : h[e + 2 < 4 ? e + 2 : 3];
            const double2 u4 = e >= 4 ? v[e >= 4 ? e - 4 : 0] : h[e < 4 ? e : 3];
            const double b2 = (k >= 2 && k - 2 < nb) ? a.beta[k - 2] : 0.0;
            const double g4 = (k >= 4 && k - 4 < nb) ? a.gamma[k - 4] : 0.0;
            v[e] = cadd(v[e], cadd(cscale(b2, u2), cscale(g4, u4)));
        }
    }
    // 2. derivatives along x
    for (int d = 0; d < a.ox; ++d) {
        double2 t0 = make_double2(0.0, 0.0), t1 = t0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = r0 + e;
            const double2 w = cscale(leg ? 1.0 : (double)k, v[e]);
            if (k & 1) t1 = cadd(t1, w);
            else t0 = cadd(t0, w);
        }
        part[0][j][c] = t0;
        part[1][j][c] = t1;
        __syncthreads();
        if (j < 2) {  // exclusive suffix sums over the chunks, one thread per (parity, column)
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll 1
            for (int jj = kT - 1; jj >= 0; --jj) {
                const double2 t = part[j][jj][c];
                part[j][jj][c] = acc;
                acc = cadd(acc, t);
            }
        }
        __syncthreads();
        double2 R0 = part[0][j][c], R1 = part[1][j][c];  // sums over later chunks, per parity
        __syncthreads();
#pragma unroll
        for (int e = E - 1; e >= 0; --e) {
            const int k = r0 + e;
            const double2 ak = v[e];
            const double pk = leg ? 1.0 : (double)k;
            v[e] = cscale(leg ? 2.0 * k + 1.0 : (k == 0 ? 1.0 : 2.0), (k & 1) ? R0 : R1);
            if (k & 1) R1 = cadd(R1, cscale(pk, ak));
            else R0 = cadd(R0, cscale(pk, ak));
        }
    }
    // 3. Fourier factors of the column
    if (a.oy | a.oz) {
        double2 f = make_double2(1.0, 0.0);
        if (a.ndim == 3) {
            const int iy = (int)(col / a.nlast), iz = (int)(col % a.nlast);
            f = cmul(axis_factor(iy, a.Mmid, 0, a.oy, a.ky), axis_factor(iz, a.Mlast, a.last_r2c, a.oz, a.kz));
        } else {
            f = axis_factor((int)col, a.Mlast, a.last_r2c, a.oy, a.ky);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) v[e] = cmul(f, v[e]);
    }
    // 4. projection onto the Shen-Dirichlet space
    if (a.dst_basis == SGM_SHEN_DIRICHLET || a.dst_basis == SGM_LEG_DIRICHLET) {
        double2 s0 = make_double2(0.0, 0.0), s1 = s0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = r0 + e;
            if (k < N) {
                if (k & 1) s1 = cadd(s1, v[e]);
                else s0 = cadd(s0, v[e]);
            }
        }
        part[0][j][c] = s0;
        part[1][j][c] = s1;
        __syncthreads();
        if (j < 2) {  // exclusive prefix sums over the chunks and the column total
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll 1
            for (int jj = 0; jj < kT; ++jj) {
                const double2 t = part[j][jj][c];
                part[j][jj][c] = acc;
                acc = cadd(acc, t);
            }
            total[j][c] = acc;
        }
        __syncthreads();
        const double2 P0 = part[0][j][c], P1 = part[1][j][c], T0 = total[0][c], T1 = total[1][c];
        // sums of h_k over the even / odd k < N (W) and k < r0 (pw), in closed form
        const double me = (double)((N + 1) / 2), mo = (double)(N / 2);
        const double pe = (double)((r0 + 1) / 2), po = (double)(r0 / 2);
        const double W0 = leg ? me * (2.0 * me - 1.0) / 2.0 : me - 0.5;
        const double W1 = leg ? mo * (2.0 * mo + 1.0) / 2.0 : mo;
        const double pw0 = leg ? pe * (2.0 * pe - 1.0) / 2.0 : (r0 > 0 ? pe - 0.5 : 0.0);
        const double pw1 = leg ? po * (2.0 * po + 1.0) / 2.0 : po;
        const double2 lam0 = cscale(1.0 / W0, T0), lam1 = cscale(1.0 / W1, T1);
        double2 D0 = cadd(P0, cscale(-pw0, lam0)), D1 = cadd(P1, cscale(-pw1, lam1));
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = r0 + e;
            const double hk = leg ? (2.0 * k + 1.0) / 2.0 : (k == 0 ? 0.5 : 1.0);
            if (k & 1) {
                D1 = cadd(D1, cadd(v[e], cscale(-hk, lam1)));
                v[e] = D1;
            } else {
                D0 = cadd(D0, cadd(v[e], cscale(-hk, lam0)));
                v[e] = D0;
            }
            if (k >= N - 2) v[e] = make_double2(0.0, 0.0);
        }
    }
    // 4'. projection onto the Shen-Neumann space
    if (a.dst_basis == SGM_SHEN_NEUMANN || a.dst_basis == SGM_LEG_NEUMANN) {
        double2 s0 = make_double2(0.0, 0.0), s1 = s0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = r0 + e;
            if (k < N) {
                const double2 w = cscale(leg ? (double)k * (k + 1.0) : (double)k * (double)k, v[e]);
                if (k & 1) s1 = cadd(s1, w);
                else s0 = cadd(s0, w);
            }
        }
        part[0][j][c] = s0;
        part[1][j][c] = s1;
        __syncthreads();
        if (j < 2) {
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll 1
            for (int jj = 0; jj < kT; ++jj) acc = cadd(acc, part[j][jj][c]);
            total[j][c] = acc;
        }
        __syncthreads();
        const double2 mu0 = cscale(1.0 / a.k4[0], total[0][c]), mu1 = cscale(1.0 / a.k4[1], total[1][c]);
        double2 t0 = make_double2(0.0, 0.0), t1 = t0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = r0 + e;
            const double k2 = leg ? (double)k * (k + 1.0) : (double)k * (double)k;
            const double hk = leg ? (2.0 * k + 1.0) / 2.0 : 1.0;
            if (k < N) {
                v[e] = cadd(v[e], cscale(-k2 * hk, (k & 1) ? mu1 : mu0));
                if (k & 1) t1 = cadd(t1, cscale(k2, v[e]));
                else t0 = cadd(t0, cscale(k2, v[e]));
            }
        }
        __syncthreads();  // every thread has read total[] and part[] of the first round
        part[0][j][c] = t0;
        part[1][j][c] = t1;
        __syncthreads();
        if (j < 2) {  // exclusive prefix sums of k^2 a_k over the chunks
            double2 acc = make_double2(0.0, 0.0);
#pragma unroll 1
            for (int jj = 0; jj < kT; ++jj) {
                const double2 t = part[j][jj][c];
                part[j][jj][c] = acc;
                acc = cadd(acc, t);
            }
        }
        __syncthreads();
        double2 P0 = part[0][j][c], P1 = part[1][j][c];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = r0 + e;
            const double k2 = leg ? (double)k * (k + 1.0) : (double)k * (double)k;
            if (k & 1) {
                P1 = cadd(P1, cscale(k2, v[e]));
                v[e] = cscale(1.0 / k2, P1);
            } else if (k > 0) {
                P0 = cadd(P0, cscale(k2, v[e]));
                v[e] = cscale(1.0 / k2, P0);
            }
            if (k >= N - 2) v[e] = make_double2(0.0, 0.0);
        }
    }
    if (live) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = r0 + e;
            if (k < N) out[k * ld + col] = v[e];
        }
    }
}

}  // namespace

hipError_t launch_dx_project(const double2* in, double2* out, const DxArgs& a, hipStream_t s) {
    const long blocks = ((long)a.ncols + kW - 1) / kW;
    if (blocks <= 0) return hipSuccess;
    const int need = (a.N + kT - 1) / kT;  // rows per chunk
    dim3 g((unsigned)blocks), b(kT * kW);
    if (need <= 2) hipLaunchKernelGGL(k_dx_project<2>, g, b, 0, s, in, out, a);
    else if (need <= 4) hipLaunchKernelGGL(k_dx_project<4>, g, b, 0, s, in, out, a);
    else if (need <= 8) hipLaunchKernelGGL(k_dx_project<8>, g, b, 0, s, in, out, a);
    else if (need <= 16) hipLaunchKernelGGL(k_dx_project<16>, g, b, 0, s, in, out, a);
    else if (need <= 32) hipLaunchKernelGGL(k_dx_project<32>, g, b, 0, s, in, out, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace sgm
