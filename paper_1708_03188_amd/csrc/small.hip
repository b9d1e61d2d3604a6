// One-kernel transforms of small 2D spaces (N, M <= 64): the field in LDS, the
// periodic axis as a DFT product, the x axis as a product with the plan's dense
// projection, scalar-product or synthesis matrix.  One work-group of 256 threads;
// consecutive threads take consecutive outputs of a row, so the table rows and
// the LDS rows they read are contiguous and the input row they share is a
// broadcast.
#include "small.h"

namespace sgm {

namespace {

__global__ void __launch_bounds__(256) k_small(const void* in, void* out, SmallDev sd, int mode) {
    extern __shared__ double2 sm[];
    const int N = sd.N, M = sd.M, Mc = sd.Mc;
    const double* P = sd.P[mode];
    const int tid = threadIdx.x;
    if (mode != kSmallBackward) {
        double2* A = sm;          // [N][M] physical field
        double2* U = sm + N * M;  // [N][Mc] after the periodic axis
        if (sd.r2c) {
            const double* u = static_cast<const double*>(in);
            for (int i = tid; i < N * M; i += 256) A[i] = make_double2(u[i], 0.0);
        } else {
            const double2* u = static_cast<const double2*>(in);
            for (int i = tid; i < N * M; i += 256) A[i] = u[i];
        }
        __syncthreads();
        for (int o = tid; o < N * Mc; o += 256) {
            const int x = o / Mc, n = o - x * Mc;
            double2 acc = make_double2(0.0, 0.0);
            for (int y = 0; y < M; ++y) {
                const double2 a = A[x * M + y], f = sd.F[y * Mc + n];
                acc.x += a.x * f.x - a.y * f.y;
                acc.y += a.x * f.y + a.y * f.x;
            }
            U[o] = acc;
        }
        __syncthreads();
        double2* uh = static_cast<double2*>(out);
        for (int o = tid; o < N * Mc; o += 256) {
            const int l = o / Mc, n = o - l * Mc;
            double2 acc = make_double2(0.0, 0.0);
            for (int x = 0; x < N; ++x) {
                const double p = P[l * N + x];
                const double2 v = U[x * Mc + n];
                acc.x += p * v.x;
                acc.y += p * v.y;
            }
            uh[o] = acc;
        }
    } else {
        double2* V0 = sm;           // [N][Mc] coefficients
        double2* V = sm + N * Mc;   // [N][Mc] after the x axis
        const double2* uh = static_cast<const double2*>(in);
        for (int i = tid; i < N * Mc; i += 256) V0[i] = uh[i];
        __syncthreads();
        for (int o = tid; o < N * Mc; o += 256) {
            const int x = o / Mc, n = o - x * Mc;
            double2 acc = make_double2(0.0, 0.0);
            for (int l = 0; l < N; ++l) {
                const double p = P[x * N + l];
                const double2 v = V0[l * Mc + n];
                acc.x += p * v.x;
                acc.y += p * v.y;
            }
            V[o] = acc;
        }
        __syncthreads();
        if (sd.r2c) {
            double* u = static_cast<double*>(out);
            for (int o = tid; o < N * M; o += 256) {
                const int x = o / M, y = o - x * M;
                double acc = 0.0;
                for (int n = 0; n < Mc; ++n) {
                    const double2 v = V[x * Mc + n], g = sd.G[n * M + y];
                    acc += v.x * g.x - v.y * g.y;
                }
                u[o] = acc;
            }
        } else {
            double2* u = static_cast<double2*>(out);
            for (int o = tid; o < N * M; o += 256) {
                const int x = o / M, y = o - x * M;
                double2 acc = make_double2(0.0, 0.0);
                for (int n = 0; n < Mc; ++n) {
                    const double2 v = V[x * Mc + n], g = sd.G[n * M + y];
                    acc.x += v.x * g.x - v.y * g.y;
                    acc.y += v.x * g.y + v.y * g.x;
                }
                u[o] = acc;
            }
        }
    }
}

}  // namespace

hipError_t launch_small_pass(const void* in, void* out, const SmallDev& sd, int mode, hipStream_t s) {
    if (sd.N < 1 || sd.N > kSmallMaxN || sd.M < 1 || sd.M > kSmallMaxM || mode < 0 || mode > 2)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_small, dim3(1), dim3(256), small_lds_bytes(sd.N, sd.M, sd.r2c != 0), s, in, out, sd, mode);
    return hipGetLastError();
}

}  // namespace sgm
