// Dense x-axis pass of the Legendre-family spaces on the FP64 matrix cores.
//
// The Legendre transforms have no fast algorithm (Sec. 3.4.2): every x pass is
// the product of a plan-constant N x N matrix with the N x C real view of the
// spectral array.  A work-group owns TC adjacent real columns: it stages all N
// rows of them in LDS (coalesced 8 TC-byte rows), then its four waves compute
// the output rows in 16-row blocks with v_mfma_f64_16x16x4 (A fragment: one
// matrix element per lane, fetched from the fragment-ordered matrix in one
// coalesced 512-byte load; B fragment: one staged value per lane), and write
// them back.  All reads of the block's columns precede its writes, so the pass
// may run in place.
#include "legendre.h"

namespace sgm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

template <int TC, int RBW>
__global__ __launch_bounds__(256) void k_leg_pass(const double* __restrict__ Apk, const double* in, double* out, int N,
                                                   long C) {
    extern __shared__ double tile[];  // [Kp][TC]
    constexpr int CB = TC / 16;
    const long c0 = (long)blockIdx.x * TC;
    const int Kp = (N + 3) & ~3;
    for (int idx = threadIdx.x; idx < Kp * TC; idx += 256) {
        const int r = idx / TC, c = idx - r * TC;
        tile[idx] = (r < N && c0 + c < C) ? in[(long)r * C + c0 + c] : 0.0;
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int RB = (N + 15) >> 4;
    d4 acc[RBW][CB];
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = d4{0.0, 0.0, 0.0, 0.0};
    const int kl = lane >> 4, cl = lane & 15;
    for (int g = 0; g < (Kp >> 2); ++g) {
        double b[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) b[cb] = tile[(4 * g + kl) * TC + cb * 16 + cl];
#pragma unroll
        for (int rb = 0; rb < RBW; ++rb) {
            const int r = wave + 4 * rb;
            if (r < RB) {
                const double a = Apk[((long)g * RB + r) * 64 + lane];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[cb], acc[rb][cb], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
        const int r = wave + 4 * rb;
        if (r >= RB) continue;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const long col = c0 + cb * 16 + cl;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * r + 4 * i + kl;  // D element i of lane l: row 4 i + l / 16, column l % 16
                if (row < N && col < C) out[(long)row * C + col] = acc[rb][cb][i];
            }
        }
    }
}

}  // namespace

hipError_t launch_leg_pass(const double* Apk, const double* in, double* out, int N, long C, hipStream_t s) {
    if (C <= 0) return hipSuccess;
    const int Kp = (N + 3) & ~3;
    if (N <= 256) {
        constexpr int TC = 32;
        const long blocks = (C + TC - 1) / TC;
        const size_t lds = (size_t)Kp * TC * sizeof(double);
        if (N <= 64) hipLaunchKernelGGL((k_leg_pass<TC, 1>), dim3((unsigned)blocks), dim3(256), lds, s, Apk, in, out, N, C);
        else if (N <= 128) hipLaunchKernelGGL((k_leg_pass<TC, 2>), dim3((unsigned)blocks), dim3(256), lds, s, Apk, in, out, N, C);
        else hipLaunchKernelGGL((k_leg_pass<TC, 4>), dim3((unsigned)blocks), dim3(256), lds, s, Apk, in, out, N, C);
    } else if (N <= kLegMaxN) {
        constexpr int TC = 16;
        const long blocks = (C + TC - 1) / TC;
        const size_t lds = (size_t)Kp * TC * sizeof(double);
        hipLaunchKernelGGL((k_leg_pass<TC, 8>), dim3((unsigned)blocks), dim3(256), lds, s, Apk, in, out, N, C);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sgm
