// Batched bf16 GEMM on the gfx950 matrix cores.
//
// 64 x 64 output tile per 256-thread block, four waves of 32 x 32 each, K in
// steps of 32 staged through LDS (operands converted to bf16 on the way in),
// v_mfma_f32_32x32x16_bf16 with fp32 accumulation.  Operand lane layout of
// that instruction: lane i supplies A[i % 32][8 (i / 32) + v] and
// B[8 (i / 32) + v][i % 32], v = 0..7, and receives
// C[8 r + 4 (i / 32) + v][i % 32] in accumulator 4 r + v, r, v = 0..3.
#include "fno_gemm.h"

namespace sgm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int GBM = 64, GBN = 64, GBK = 32, GPAD = 8;

template <typename T>
__device__ __forceinline__ float ldf(const void* p, long i) {
    return (float)static_cast<const T*>(p)[i];
}

__global__ void __launch_bounds__(256) k_gemm(GemmDesc d) {
    __shared__ __bf16 As[GBM][GBK + GPAD];
    __shared__ __bf16 Bs[GBN][GBK + GPAD];
    const int tilesM = (d.M + GBM - 1) / GBM, tilesN = (d.N + GBN - 1) / GBN;
    long id = blockIdx.x;
    const int tn = (int)(id % tilesN); id /= tilesN;
    const int tm = (int)(id % tilesM); id /= tilesM;
    const int ks = (int)(id % d.splitk); id /= d.splitk;
    const long b = id;
    const int m0 = tm * GBM, n0 = tn * GBN;
    const int kchunk = ((d.K + d.splitk - 1) / d.splitk + GBK - 1) / GBK * GBK;
    const int kbeg = ks * kchunk, kend = min(d.K, kbeg + kchunk);
    const long aoff = b * d.sAb, boff = b * d.sBb;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    floatx16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
    const bool a_kfast = d.sAk == 1;
    const bool b_nfast = d.sBn == 1;
    for (int k0 = kbeg; k0 < kend; k0 += GBK) {
        for (int e = tid; e < GBM * GBK; e += 256) {
            int m, k;
            if (a_kfast) { m = e / GBK; k = e - m * GBK; }
            else { k = e / GBM; m = e - k * GBM; }
            const int gm = m0 + m, gk = k0 + k;
            float v = 0.f;
            if (gm < d.M && gk < kend) {
                const long i = aoff + gm * d.sAm + gk * d.sAk;
                v = d.a_f32 ? ldf<float>(d.A, i) : ldf<__bf16>(d.A, i);
            }
            As[m][k] = (__bf16)v;
        }
        for (int e = tid; e < GBN * GBK; e += 256) {
            int n, k;
            if (b_nfast) { k = e / GBN; n = e - k * GBN; }
            else { n = e / GBK; k = e - n * GBK; }
            const int gn = n0 + n, gk = k0 + k;
            float v = 0.f;
            if (gn < d.N && gk < kend) {
                const long i = boff + gk * d.sBk + gn * d.sBn;
                v = d.b_f32 ? ldf<float>(d.B, i) : ldf<__bf16>(d.B, i);
            }
            Bs[n][k] = (__bf16)v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 16) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wm + (lane & 31)][kk + 8 * (lane >> 5)]);
            const bf16x8 bb = *reinterpret_cast<const bf16x8*>(&Bs[wn + (lane & 31)][kk + 8 * (lane >> 5)]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    const int col = n0 + wn + (lane & 31);
    if (col >= d.N) return;
    const long coff = b * d.sCb + (long)col * d.sCn;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = m0 + wm + 8 * r + 4 * (lane >> 5) + v;
            if (row >= d.M) continue;
            float* cp = d.C + coff + (long)row * d.sCm;
            const float val = d.alpha * acc[4 * r + v];
            if (d.splitk > 1) atomicAdd(cp, val);
            else *cp = d.beta == 0.f ? val : val + d.beta * *cp;
        }
}

hipError_t gemm(const GemmDesc& d, hipStream_t s) {
    if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
    const long tiles = (long)((d.M + GBM - 1) / GBM) * ((d.N + GBN - 1) / GBN) * d.batch * (d.splitk > 1 ? d.splitk : 1);
    GemmDesc e = d;
    if (e.splitk < 1) e.splitk = 1;
    hipLaunchKernelGGL(k_gemm, dim3((unsigned)tiles), dim3(256), 0, s, e);
    return hipGetLastError();
}

}  // namespace sgm
