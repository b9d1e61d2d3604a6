// Transform-pass and solver kernels for gfx950.
//
// Every kernel stages its tile in LDS: contiguous-line passes read whole rows,
// strided passes (the middle periodic axis and the Chebyshev axis) read
// column tiles of W adjacent columns per row, so each row segment is one
// coalesced W * 16-byte access.  The tile is transformed in LDS and written
// back once.
#include "fft_lds.h"
#include "kernels.h"

namespace sgm {

// ---------------------------------------------------------------------------
// Contiguous lines: R2C by the two-for-one trick.  Block b packs real lines
// 2g and 2g+1 of its 2G-line slab as the real and imaginary part of complex
// line g, transforms, then splits X1 = (Z_k + conj Z_{L-k})/2 and
// X2 = (Z_k - conj Z_{L-k})/(2i) for k = 0..L/2.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_lines_r2c(const double* __restrict__ in, double2* __restrict__ out,
                                                   int L, int nlines, int G, RadixPlan rp, double scale) {
    extern __shared__ double2 lds[];
    double2* A = lds;
    double2* B = lds + (size_t)G * L;
    const long line0 = (long)blockIdx.x * 2 * G;
    const int nreal = 2 * G * L;
    double* Ad = reinterpret_cast<double*>(A);
    for (int f = threadIdx.x; f < nreal; f += blockDim.x) {
        int row = f / L, e = f - row * L;
        long ln = line0 + row;
        double v = ln < nlines ? in[ln * L + e] : 0.0;
        Ad[2 * ((row >> 1) * L + e) + (row & 1)] = v;
    }
    __syncthreads();
    double2* R = lds_fft<-1>(A, B, rp, G, 1, L, false);
    const int Lh = L / 2 + 1;
    for (int t = threadIdx.x; t < G * Lh; t += blockDim.x) {
        int g = t / Lh, k = t - g * Lh;
        double2 z = R[g * L + k];
        double2 zr = cconj(R[g * L + (k == 0 ? 0 : L - k)]);
        double2 x1 = make_double2(0.5 * scale * (z.x + zr.x), 0.5 * scale * (z.y + zr.y));
        double2 d = csub(z, zr);  // X2 = d / (2i) = (d.y, -d.x) / 2
        double2 x2 = make_double2(0.5 * scale * d.y, -0.5 * scale * d.x);
        long l0 = line0 + 2 * g;
        if (l0 < nlines) out[l0 * Lh + k] = x1;
        if (l0 + 1 < nlines) out[(l0 + 1) * Lh + k] = x2;
    }
}

// C2R by the same pairing: Z = X1 + i X2 on the Hermitian-extended spectra.
__global__ void __launch_bounds__(256) k_lines_c2r(const double2* __restrict__ in, double* __restrict__ out,
                                                   int L, int nlines, int G, RadixPlan rp) {
    extern __shared__ double2 lds[];
    double2* A = lds;
    double2* B = lds + (size_t)G * L;
    const long line0 = (long)blockIdx.x * 2 * G;
    const int Lh = L / 2 + 1;
    for (int t = threadIdx.x; t < G * Lh; t += blockDim.x) {
        int g = t / Lh, k = t - g * Lh;
        long l0 = line0 + 2 * g;
        double2 x1 = l0 < nlines ? in[l0 * Lh + k] : make_double2(0.0, 0.0);
        double2 x2 = l0 + 1 < nlines ? in[(l0 + 1) * Lh + k] : make_double2(0.0, 0.0);
        if (k == 0 || 2 * k == L) {
            A[g * L + k] = make_double2(x1.x, x2.x);
        } else {
            A[g * L + k] = make_double2(x1.x - x2.y, x1.y + x2.x);
            A[g * L + L - k] = make_double2(x1.x + x2.y, -x1.y + x2.x);
        }
    }
    __syncthreads();
    double2* R = lds_fft<1>(A, B, rp, G, 1, L, false);
    const int nreal = 2 * G * L;
    const double* Rd = reinterpret_cast<const double*>(R);
    for (int f = threadIdx.x; f < nreal; f += blockDim.x) {
        int row = f / L, e = f - row * L;
        long ln = line0 + row;
        if (ln < nlines) out[ln * L + e] = Rd[2 * ((row >> 1) * L + e) + (row & 1)];
    }
}

template <int SIGN>
__global__ void __launch_bounds__(256) k_lines_c2c(const double2* __restrict__ in, double2* __restrict__ out,
                                                   int L, int nlines, int G, RadixPlan rp, double scale) {
    extern __shared__ double2 lds[];
    double2* A = lds;
    double2* B = lds + (size_t)G * L;
    const long line0 = (long)blockIdx.x * G;
    for (int t = threadIdx.x; t < G * L; t += blockDim.x) {
        int g = t / L;
        long ln = line0 + g;
        A[t] = ln < nlines ? in[line0 * L + t] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double2* R = lds_fft<SIGN>(A, B, rp, G, 1, L, false);
    for (int t = threadIdx.x; t < G * L; t += blockDim.x) {
        int g = t / L;
        if (line0 + g < nlines) out[line0 * L + t] = cscale(R[t], scale);
    }
}

// ---------------------------------------------------------------------------
// Strided C2C: data[o][e][c], e = 0..L-1 the transform index, c = 0..inner-1.
// Block -> (o, column tile of W); LDS tile [e][W].
// ---------------------------------------------------------------------------
template <int SIGN>
__global__ void __launch_bounds__(256) k_strided_c2c(const double2* in, double2* out, int L, int outer,
                                                     int inner, int W, RadixPlan rp, double scale) {
    extern __shared__ double2 lds[];
    double2* A = lds;
    double2* B = lds + (size_t)L * W;
    const int tiles = (inner + W - 1) / W;
    const int o = blockIdx.x / tiles;
    const int c0 = (blockIdx.x - o * tiles) * W;
    const long base = (long)o * L * inner + c0;
    for (int t = threadIdx.x; t < L * W; t += blockDim.x) {
        int e = t / W, c = t - e * W;
        A[t] = (c0 + c < inner) ? in[base + (long)e * inner + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double2* R = lds_fft<SIGN>(A, B, rp, W, W, 1, true);
    for (int t = threadIdx.x; t < L * W; t += blockDim.x) {
        int e = t / W, c = t - e * W;
        if (c0 + c < inner) out[base + (long)e * inner + c] = cscale(R[t], scale);
    }
}

// ---------------------------------------------------------------------------
// Chebyshev axis, forward direction.  Column tile [N][W] of the spectral
// array (row stride ncols).  Steps:
//   1. DCT-II of every column through one complex FFT of the reordered
//      sequence v_j = g_{2j}, v_{N-1-j} = g_{2j+1} (Makhoul 1980):
//      C_k = Re(theta_k A_k) + i Re(theta_k B_k), theta_k = e^{-i pi k/(2N)},
//      A_k = (V_k + conj V_{N-k})/2, B_k = (V_k - conj V_{N-k})/(2i).
//      C_k = sum_j g_j cos(pi k (2j+1)/(2N)) = (N/pi) (g, T_k)^N_w.
//   2a. scalar product: S_l = (pi/N)(C_l + beta_l C_{l+2} + gamma_l C_{l+4}).
//   2b. projection u_hat = B^{-1} S: the equivalent weighted least-squares
//       problem min || D^{1/2} (P u_hat - c) || (c = Chebyshev coefficients,
//       D = diag(c_k pi/2), P the recombination).  Per parity, b = D^{1/2} c is
//       first projected onto range(D^{1/2} P) (the null space of the boundary
//       functionals, exact integers), then the now consistent banded system is
//       solved with the plan's Givens rotations and banded R.  Projecting first
//       keeps the data residual out of the least-squares solve, whose rounding
//       it would otherwise amplify by cond^2.  Regular Chebyshev: u_hat = c.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dct2_post(double2 V, double2 Vr, double2 th, double2* Ck, double2* Cnk,
                                          double2 thn) {
    // A = (V + conj Vr)/2, B = (V - conj Vr)/(2i); C = Re(th A) + i Re(th B)
    double2 cv = cconj(Vr);
    double2 a = make_double2(0.5 * (V.x + cv.x), 0.5 * (V.y + cv.y));
    double2 d = csub(V, cv);
    double2 b = make_double2(0.5 * d.y, -0.5 * d.x);
    *Ck = make_double2(th.x * a.x - th.y * a.y, th.x * b.x - th.y * b.y);
    // For N-k: A' = conj(a), B' = conj(b)
    *Cnk = make_double2(thn.x * a.x + thn.y * a.y, thn.x * b.x + thn.y * b.y);
}

__global__ void __launch_bounds__(256) k_cheb_fwd(const double2* in, double2* out, ChebDev cd, int ncols, int W,
                                                  RadixPlan rp, int mode) {
    extern __shared__ double2 lds[];
    const int N = cd.N;
    double2* A = lds;
    double2* B = lds + (size_t)N * W;
    const int c0 = blockIdx.x * W;
    for (int t = threadIdx.x; t < N * W; t += blockDim.x) {
        int j = t / W, c = t - j * W;
        double2 v = (c0 + c < ncols) ? in[(long)j * ncols + c0 + c] : make_double2(0.0, 0.0);
        int vj = (j & 1) ? (N - 1 - (j >> 1)) : (j >> 1);
        A[vj * W + c] = v;
    }
    __syncthreads();
    double2* R = lds_fft<-1>(A, B, rp, W, W, 1, true);
    double2* C = (R == A) ? B : A;
    const int half = N / 2 + 1;
    for (int t = threadIdx.x; t < half * W; t += blockDim.x) {
        int k = t / W, c = t - k * W;
        int kn = k == 0 ? 0 : N - k;
        if (kn < k) continue;  // pair handled by its lower index
        double2 ck, cnk;
        dct2_post(R[k * W + c], R[kn * W + c], cd.theta[k], &ck, &cnk, cd.theta[kn]);
        C[k * W + c] = ck;
        if (kn != k) C[kn * W + c] = cnk;
    }
    __syncthreads();
    const int nb = cd.nb;
    if (mode == kScalarProduct) {
        const double s = M_PI / N;
        for (int t = threadIdx.x; t < N * W; t += blockDim.x) {
            int l = t / W, c = t - l * W;
            double2 v = make_double2(0.0, 0.0);
            if (l < nb) {
                v = C[l * W + c];
                if (l + 2 < N) { double bb = cd.beta[l]; v.x += bb * C[(l + 2) * W + c].x; v.y += bb * C[(l + 2) * W + c].y; }
                if (l + 4 < N) { double gg = cd.gamma[l]; v.x += gg * C[(l + 4) * W + c].x; v.y += gg * C[(l + 4) * W + c].y; }
                v = cscale(v, s);
            }
            R[t] = v;
        }
        __syncthreads();
    } else if (cd.basis == SGM_CHEBYSHEV) {
        for (int t = threadIdx.x; t < N * W; t += blockDim.x) {
            int k = t / W;
            R[t] = cscale(C[t], cd.fscale[k]);
        }
        __syncthreads();
    } else {
        // scale to b = D^{1/2} c
        for (int t = threadIdx.x; t < N * W; t += blockDim.x) {
            int k = t / W;
            C[t] = cscale(C[t], cd.bscale[k]);
        }
        __syncthreads();
        const int nrot = cd.basis == SGM_SHEN_DIRICHLET ? 1 : 2;
        const int lane = threadIdx.x;
        if (lane < 2 * W) {
            const int p = lane / W, c = lane - p * W;
            const int n = cd.npar[p], m = cd.mpar[p];
            const int es = 2 * W;
            double2* col = C + p * W + c;
            const double* rot = cd.rot[p];
            const double* rt = cd.rtab[p];
            const double* qt = cd.qtab[p];
            // (i) project b onto range(D^{1/2} P): remove the components along the
            //     orthonormalised boundary functionals, b <- b - sum_r q_r (q_r . b)
            double2 s1 = make_double2(0.0, 0.0), s2 = make_double2(0.0, 0.0);
            for (int t = 0; t < m; ++t) {
                double2 v = col[t * es];
                double q1 = qt[2 * t], q2 = qt[2 * t + 1];
                s1.x += q1 * v.x; s1.y += q1 * v.y;
                s2.x += q2 * v.x; s2.y += q2 * v.y;
            }
            auto ld = [&](int t) {
                if (t >= m) return make_double2(0.0, 0.0);
                double2 v = col[t * es];
                double q1 = qt[2 * t], q2 = qt[2 * t + 1];
                return make_double2(v.x - q1 * s1.x - q2 * s2.x, v.y - q1 * s1.y - q2 * s2.y);
            };
            // (ii) Givens sweep: Q^T b, then back substitution with the banded R
            double2 w0 = ld(0), w1 = ld(1);
            double2 w2 = nrot == 2 ? ld(2) : make_double2(0.0, 0.0);
            for (int i = 0; i < n; ++i) {
                double c1 = rot[4 * i], s1r = rot[4 * i + 1];
                double2 a = w0, b = w1;
                w0 = make_double2(c1 * a.x + s1r * b.x, c1 * a.y + s1r * b.y);
                w1 = make_double2(-s1r * a.x + c1 * b.x, -s1r * a.y + c1 * b.y);
                if (nrot == 2) {
                    double c2 = rot[4 * i + 2], s2r = rot[4 * i + 3];
                    a = w0; b = w2;
                    w0 = make_double2(c2 * a.x + s2r * b.x, c2 * a.y + s2r * b.y);
                    w2 = make_double2(-s2r * a.x + c2 * b.x, -s2r * a.y + c2 * b.y);
                    col[i * es] = w0;
                    w0 = w1; w1 = w2;
                    w2 = ld(i + 3);
                } else {
                    col[i * es] = w0;
                    w0 = w1;
                    w1 = ld(i + 2);
                }
            }
            double2 x1 = make_double2(0.0, 0.0), x2 = make_double2(0.0, 0.0);
            for (int i = n - 1; i >= 0; --i) {
                double r0 = rt[3 * i], r1 = rt[3 * i + 1], r2 = rt[3 * i + 2];
                double2 z = col[i * es];
                double2 x = make_double2((z.x - r1 * x1.x - r2 * x2.x) * r0, (z.y - r1 * x1.y - r2 * x2.y) * r0);
                col[i * es] = x;
                x2 = x1; x1 = x;
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < N * W; t += blockDim.x) {
            int l = t / W;
            R[t] = l < nb ? C[t] : make_double2(0.0, 0.0);
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < N * W; t += blockDim.x) {
        int l = t / W, c = t - l * W;
        if (c0 + c < ncols) out[(long)l * ncols + c0 + c] = R[t];
    }
}

// ---------------------------------------------------------------------------
// Chebyshev axis, backward direction: recombination to Chebyshev coefficients
// c_k = u_k + beta_{k-2} u_{k-2} + gamma_{k-4} u_{k-4}, then the DCT-III
// u_j = sum_k c_k cos(pi k (2j+1)/(2N)) through one inverse complex FFT of
// W_0 = 2 c_0, W_k = e^{i pi k/(2N)} (c_k - i c_{N-k}); u_{2n} = w_n / 2,
// u_{2n+1} = w_{N-1-n} / 2.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_cheb_bwd(const double2* in, double2* out, ChebDev cd, int ncols, int W,
                                                  RadixPlan rp) {
    extern __shared__ double2 lds[];
    const int N = cd.N, nb = cd.nb;
    double2* A = lds;
    double2* B = lds + (size_t)N * W;
    const int c0 = blockIdx.x * W;
    for (int t = threadIdx.x; t < N * W; t += blockDim.x) {
        int l = t / W, c = t - l * W;
        B[t] = (l < nb && c0 + c < ncols) ? in[(long)l * ncols + c0 + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    // recombination into A
    for (int t = threadIdx.x; t < N * W; t += blockDim.x) {
        int k = t / W, c = t - k * W;
        double2 v = B[t];
        if (k >= 2 && k - 2 < nb) { double bb = cd.beta[k - 2]; double2 u = B[(k - 2) * W + c]; v.x += bb * u.x; v.y += bb * u.y; }
        if (k >= 4 && k - 4 < nb) { double gg = cd.gamma[k - 4]; double2 u = B[(k - 4) * W + c]; v.x += gg * u.x; v.y += gg * u.y; }
        A[t] = v;
    }
    __syncthreads();
    // DCT-III pre-processing into B
    for (int t = threadIdx.x; t < N * W; t += blockDim.x) {
        int k = t / W, c = t - k * W;
        double2 w;
        if (k == 0) {
            double2 v = A[c];
            w = make_double2(2.0 * v.x, 2.0 * v.y);
        } else {
            double2 ck = A[t], cn = A[(N - k) * W + c];
            // d = c_k - i c_{N-k}
            double2 d = make_double2(ck.x + cn.y, ck.y - cn.x);
            w = cmul(cconj(cd.theta[k]), d);
        }
        B[t] = w;
    }
    __syncthreads();
    double2* R = lds_fft<1>(B, A, rp, W, W, 1, true);
    for (int t = threadIdx.x; t < N * W; t += blockDim.x) {
        int j = t / W, c = t - j * W;
        int vj = (j & 1) ? (N - 1 - (j >> 1)) : (j >> 1);
        if (c0 + c < ncols) out[(long)j * ncols + c0 + c] = cscale(R[vj * W + c], 0.5);
    }
}

// ---------------------------------------------------------------------------
// Per-wavenumber Galerkin solves.  Each (column, parity) lane solves
//   M x = f,  M = T0 + mu1 T1 + mu2 T2 (band, offsets -P..Q) + sum_r U_r(i) V_r(j) [j >= i + S]
// by bottom-up elimination: for i = n-1..0 every unknown above row i and
// the running tail sums sigma_r(i+S) = sum_{j>=i+S} V_r(j) x_j are kept as
// affine functions of the window (x_i .. x_{i-P+1}); row i then gives
// x_i = a_i + sum_e b_{i,e} x_{i-e}, and a top-down sweep recovers x.
// Helmholtz (Shen-Dirichlet): P = Q = S = 1, one tail term; biharmonic:
// P = Q = S = 2, two tail terms.  a_i overwrites f_i in LDS, b_i goes to a
// per-lane LDS scratch.
// ---------------------------------------------------------------------------
template <int P>
struct Rep {
    double2 c;
    double w[P];
};

template <int P, int Q, int S, int NR>
__device__ void ul_solve_lane(double2* col, int es, int n, const double* tab, double mu1, double mu2, double* bs,
                              int bstride) {
    Rep<P> rx[Q];
    Rep<P> rs[NR];
    for (int d = 0; d < Q; ++d) { rx[d].c = make_double2(0.0, 0.0); for (int e = 0; e < P; ++e) rx[d].w[e] = 0.0; }
    for (int r = 0; r < NR; ++r) { rs[r].c = make_double2(0.0, 0.0); for (int e = 0; e < P; ++e) rs[r].w[e] = 0.0; }
    double Vnext[NR];  // V_r(i + S - 1) for the update at row i (needs row i+S-1's V)
    for (int r = 0; r < NR; ++r) Vnext[r] = 0.0;
    for (int i = n - 1; i >= 0; --i) {
        const double* row = tab + 20 * i;
        double band[P + Q + 1];
#pragma unroll
        for (int d = -P; d <= Q; ++d)
            band[d + P] = row[d + 2] + mu1 * row[5 + d + 2] + mu2 * row[10 + d + 2];
        double U[NR], V[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) { U[r] = row[15 + r]; V[r] = row[17 + r]; }
        double2 f = col[i * es];
        double coef[P + 1];
        coef[0] = band[P];
#pragma unroll
        for (int e = 1; e <= P; ++e) coef[e] = band[P - e];
        double2 cst = f;
#pragma unroll
        for (int d = 1; d <= Q; ++d) {
            double bd = band[P + d];
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
        double2 a = make_double2(cst.x * inv, cst.y * inv);
        double b[P];
#pragma unroll
        for (int e = 0; e < P; ++e) b[e] = -coef[e + 1] * inv;
        col[i * es] = a;
#pragma unroll
        for (int e = 0; e < P; ++e) bs[(long)i * bstride + e] = b[e];
        // substitute x_i into a representation over (x_i, x_{i-1}, ..)
        auto subst = [&](const Rep<P>& q) {
            Rep<P> o;
            o.c = make_double2(q.c.x + q.w[0] * a.x, q.c.y + q.w[0] * a.y);
#pragma unroll
            for (int e = 0; e < P; ++e) o.w[e] = q.w[0] * b[e] + (e + 1 < P ? q.w[e + 1] : 0.0);
            return o;
        };
        Rep<P> nrx[Q];
        nrx[0].c = a;
#pragma unroll
        for (int e = 0; e < P; ++e) nrx[0].w[e] = b[e];
#pragma unroll
        for (int d = 1; d < Q; ++d) nrx[d] = subst(rx[d - 1]);
        // sigma_r(i-1+S) = V_r(i-1+S) x_{i-1+S} + sigma_r(i+S)
        double Vt[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) Vt[r] = (S == 1) ? V[r] : Vnext[r];
        const bool inside = (i - 1 + S) < n;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            Rep<P> o = subst(rs[r]);
            if (inside) {
                const Rep<P>& xs = nrx[S - 1];
                o.c.x += Vt[r] * xs.c.x; o.c.y += Vt[r] * xs.c.y;
#pragma unroll
                for (int e = 0; e < P; ++e) o.w[e] += Vt[r] * xs.w[e];
            }
            rs[r] = o;
        }
#pragma unroll
        for (int d = 0; d < Q; ++d) rx[d] = nrx[d];
#pragma unroll
        for (int r = 0; r < NR; ++r) Vnext[r] = V[r];
    }
    // top-down: x_i = a_i + sum_e b_{i,e} x_{i-1-e}
    double2 hist[P];
#pragma unroll
    for (int e = 0; e < P; ++e) hist[e] = make_double2(0.0, 0.0);
    for (int i = 0; i < n; ++i) {
        double2 x = col[i * es];
#pragma unroll
        for (int e = 0; e < P; ++e) {
            double be = bs[(long)i * bstride + e];
            x.x += be * hist[e].x; x.y += be * hist[e].y;
        }
        col[i * es] = x;
#pragma unroll
        for (int e = P - 1; e > 0; --e) hist[e] = hist[e - 1];
        hist[0] = x;
    }
}

__device__ __forceinline__ int wavenumber(int q, int M) { return q < (M + 1) / 2 ? q : q - M; }

__global__ void __launch_bounds__(256) k_solve(const double2* in, double2* out, ChebDev cd, ColGeom g, int W,
                                               int kind, double alpha) {
    extern __shared__ double2 lds[];
    const int N = cd.N, nb = cd.nb;
    double2* D = lds;
    double* bs = reinterpret_cast<double*>(lds + (size_t)N * W);
    const int c0 = blockIdx.x * W;
    const int ncols = g.ncols;
    for (int t = threadIdx.x; t < N * W; t += blockDim.x) {
        int l = t / W, c = t - l * W;
        D[t] = (l < nb && c0 + c < ncols) ? in[(long)l * ncols + c0 + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int lane = threadIdx.x;
    if (lane < 2 * W) {
        const int p = lane / W, c = lane - p * W;
        const int col = c0 + c;
        if (col < ncols) {
            int iy = col / g.nlast, iz = col - iy * g.nlast;
            double m = g.Mmid > 1 ? (double)wavenumber(iy, g.Mmid) : 0.0;
            double nn = g.last_r2c ? (double)iz : (double)wavenumber(iz, g.Mlast);
            double k2 = g.sy * m * m + g.sz * nn * nn;
            const int n = cd.npar[p];
            if (kind == SGM_SHEN_DIRICHLET) {
                ul_solve_lane<1, 1, 1, 1>(D + p * W + c, 2 * W, n, cd.solve[p], k2 + alpha, 0.0,
                                          bs + lane, 2 * W);
            } else {
                ul_solve_lane<2, 2, 2, 2>(D + p * W + c, 2 * W, n, cd.solve[p], -2.0 * k2, k2 * k2,
                                          bs + 2 * lane, 4 * W);
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < N * W; t += blockDim.x) {
        int l = t / W, c = t - l * W;
        if (c0 + c < ncols) out[(long)l * ncols + c0 + c] = l < nb ? D[t] : make_double2(0.0, 0.0);
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t lds_bytes_lines(int L, int G) { return 2 * sizeof(double2) * (size_t)L * G; }
size_t lds_bytes_strided(int L, int W) { return 2 * sizeof(double2) * (size_t)L * W; }
size_t lds_bytes_cheb(int N, int W) { return 2 * sizeof(double2) * (size_t)N * W; }
size_t lds_bytes_solve(int N, int W, int basis) {
    int P = basis == SGM_SHEN_BIHARMONIC ? 2 : 1;
    int half = (N + 1) / 2;
    return sizeof(double2) * (size_t)N * W + sizeof(double) * (size_t)half * 2 * W * P;
}

hipError_t launch_lines_r2c(const double* in, double2* out, int L, int nlines, int G, const RadixPlan& rp,
                            double scale, hipStream_t s) {
    int blocks = (nlines + 2 * G - 1) / (2 * G);
    hipLaunchKernelGGL(k_lines_r2c, dim3(blocks), dim3(256), lds_bytes_lines(L, G), s, in, out, L, nlines, G, rp,
                       scale);
    return hipGetLastError();
}
hipError_t launch_lines_c2r(const double2* in, double* out, int L, int nlines, int G, const RadixPlan& rp,
                            hipStream_t s) {
    int blocks = (nlines + 2 * G - 1) / (2 * G);
    hipLaunchKernelGGL(k_lines_c2r, dim3(blocks), dim3(256), lds_bytes_lines(L, G), s, in, out, L, nlines, G, rp);
    return hipGetLastError();
}
hipError_t launch_lines_c2c(const double2* in, double2* out, int L, int nlines, int G, const RadixPlan& rp,
                            int sign, double scale, hipStream_t s) {
    int blocks = (nlines + G - 1) / G;
    if (sign < 0)
        hipLaunchKernelGGL(k_lines_c2c<-1>, dim3(blocks), dim3(256), lds_bytes_lines(L, G), s, in, out, L, nlines,
                           G, rp, scale);
    else
        hipLaunchKernelGGL(k_lines_c2c<1>, dim3(blocks), dim3(256), lds_bytes_lines(L, G), s, in, out, L, nlines, G,
                           rp, scale);
    return hipGetLastError();
}
hipError_t launch_strided_c2c(const double2* in, double2* out, int L, int outer, int inner, int W,
                              const RadixPlan& rp, int sign, double scale, hipStream_t s) {
    int blocks = outer * ((inner + W - 1) / W);
    if (sign < 0)
        hipLaunchKernelGGL(k_strided_c2c<-1>, dim3(blocks), dim3(256), lds_bytes_strided(L, W), s, in, out, L, outer,
                           inner, W, rp, scale);
    else
        hipLaunchKernelGGL(k_strided_c2c<1>, dim3(blocks), dim3(256), lds_bytes_strided(L, W), s, in, out, L, outer,
                           inner, W, rp, scale);
    return hipGetLastError();
}
hipError_t launch_cheb_fwd(const double2* in, double2* out, const ChebDev& cd, int ncols, int W,
                           const RadixPlan& rp, int mode, hipStream_t s) {
    int blocks = (ncols + W - 1) / W;
    hipLaunchKernelGGL(k_cheb_fwd, dim3(blocks), dim3(256), lds_bytes_cheb(cd.N, W), s, in, out, cd, ncols, W, rp,
                       mode);
    return hipGetLastError();
}
hipError_t launch_cheb_bwd(const double2* in, double2* out, const ChebDev& cd, int ncols, int W,
                           const RadixPlan& rp, hipStream_t s) {
    int blocks = (ncols + W - 1) / W;
    hipLaunchKernelGGL(k_cheb_bwd, dim3(blocks), dim3(256), lds_bytes_cheb(cd.N, W), s, in, out, cd, ncols, W, rp);
    return hipGetLastError();
}
hipError_t launch_solve(const double2* in, double2* out, const ChebDev& cd, const ColGeom& g, int W, int kind,
                        double alpha, hipStream_t s) {
    int blocks = (g.ncols + W - 1) / W;
    hipLaunchKernelGGL(k_solve, dim3(blocks), dim3(256), lds_bytes_solve(cd.N, W, kind), s, in, out, cd, g, W,
                       kind, alpha);
    return hipGetLastError();
}

}  // namespace sgm
