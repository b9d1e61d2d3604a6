// Dense x-axis pass of the Legendre-family spaces on the FP64 matrix cores.
//
// The Legendre transforms have no fast algorithm (Sec. 3.4.2): every x pass is
// the product of a plan-constant N x N matrix with the N x C real view of the
// spectral array, out = A in.  A work-group owns 16 adjacent real columns: it
// stages all N rows of them in LDS (16-byte loads, 128-byte rows), then each of
// its four waves computes RBW 16-row blocks of the output with v_mfma_f64_16x16x4
// (lane l: A fragment element A[16 r + l % 16][4 g + l / 16], fetched from the
// fragment-ordered matrix in one coalesced 512-byte load per block two k-groups
// ahead; B fragment element in[4 g + l / 16][c0 + l % 16] from LDS; result
// elements rows 4 i + l / 16 of column l % 16).  16-column work-groups (32 KB of
// LDS at N = 256) keep five per CU resident, which measured faster than wider
// tiles with more reuse of the matrix.  A work-group reads all of its columns
// before writing them, so the pass may run in place.
#include "legendre.h"

namespace sgm {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kLegTC = 16;   // real columns per work-group
constexpr int kLegRing = 2;  // k-groups of matrix fragments fetched ahead

template <int RBW>
__global__ __launch_bounds__(256) void k_leg_pass(const double* __restrict__ Apk, const double* in, double* out, int N,
                                                   long C) {
    extern __shared__ double tile[];  // [Kp][16]
    constexpr int RBP = 4 * RBW;      // row blocks of the packed matrix
    const long c0 = (long)blockIdx.x * kLegTC;
    const int Kp = (N + 3) & ~3, KG = Kp >> 2;
    for (int idx = threadIdx.x; idx < Kp * (kLegTC / 2); idx += 256) {
        const int r = idx / (kLegTC / 2), c = 2 * (idx - r * (kLegTC / 2));
        double2 v = make_double2(0.0, 0.0);
        if (r < N) {
            const double* p = in + (long)r * C + c0 + c;
            if (c0 + c + 1 < C) v = *reinterpret_cast<const double2*>(p);
            else if (c0 + c < C) v.x = p[0];
        }
        reinterpret_cast<double2*>(tile)[idx] = v;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int kl = lane >> 4, cl = lane & 15;
    // row blocks wave, wave + 4, ...; zero rows past N in the packed matrix make
    // every load and product unconditional
    const double* ap = Apk + (long)wave * 64 + lane;
    double a[kLegRing][RBW];
#pragma unroll
    for (int q = 0; q < kLegRing; ++q)
#pragma unroll
        for (int rb = 0; rb < RBW; ++rb) a[q][rb] = ap[(long)(q < KG ? q : KG - 1) * RBP * 64 + rb * 256];
    d4 acc[RBW];
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) acc[rb] = d4{0.0, 0.0, 0.0, 0.0};
    __syncthreads();
    for (int g0 = 0; g0 < KG; g0 += kLegRing) {
#pragma unroll
        for (int q = 0; q < kLegRing; ++q) {
            const int g = g0 + q;
            if (g < KG) {  // uniform: only an odd KG leaves a half ring at the end
                const double b = tile[(4 * g + kl) * kLegTC + cl];
                const long gn = (long)(g + kLegRing < KG ? g + kLegRing : g) * RBP * 64;
                double an[RBW];
#pragma unroll
                for (int rb = 0; rb < RBW; ++rb) an[rb] = ap[gn + rb * 256];
#pragma unroll
                for (int rb = 0; rb < RBW; ++rb) acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q][rb], b, acc[rb], 0, 0, 0);
#pragma unroll
                for (int rb = 0; rb < RBW; ++rb) a[q][rb] = an[rb];
            }
        }
    }
    const long col = c0 + cl;
    if (col >= C) return;
#pragma unroll
    for (int rb = 0; rb < RBW; ++rb) {
        const int r = wave + 4 * rb;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 16 * r + 4 * i + kl;  // D element i of lane l: row 4 i + l / 16, column l % 16
            if (row < N) out[(long)row * C + col] = acc[rb][i];
        }
    }
}

}  // namespace

hipError_t launch_leg_pass(const double* Apk, const double* in, double* out, int N, long C, hipStream_t s) {
    if (C <= 0) return hipSuccess;
    if (N < 1 || N > kLegMaxN) return hipErrorInvalidValue;
    const dim3 g((unsigned)((C + kLegTC - 1) / kLegTC)), b(256);
    const size_t lds = (size_t)((N + 3) & ~3) * kLegTC * sizeof(double);
    switch (leg_row_blocks(N)) {
        case 4: hipLaunchKernelGGL(k_leg_pass<1>, g, b, lds, s, Apk, in, out, N, C); break;
        case 8: hipLaunchKernelGGL(k_leg_pass<2>, g, b, lds, s, Apk, in, out, N, C); break;
        case 16: hipLaunchKernelGGL(k_leg_pass<4>, g, b, lds, s, Apk, in, out, N, C); break;
        default: hipLaunchKernelGGL(k_leg_pass<8>, g, b, lds, s, Apk, in, out, N, C); break;
    }
    return hipGetLastError();
}

}  // namespace sgm
