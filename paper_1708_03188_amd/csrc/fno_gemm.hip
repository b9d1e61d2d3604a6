// Batched bf16 GEMM on the gfx950 matrix cores.
//
// 64 x 64 output tile per 256-thread block, four waves of 32 x 32 each, K in
// steps of 32 staged through LDS (operands converted to bf16 on the way in),
// v_mfma_f32_32x32x16_bf16 with fp32 accumulation.  Operand lane layout of
// that instruction: lane i supplies A[i % 32][8 (i / 32) + v] and
// B[8 (i / 32) + v][i % 32], v = 0..7, and receives
// C[8 r + 4 (i / 32) + v][i % 32] in accumulator 4 r + v, r, v = 0..3.
#include <cstdint>

#include "fno_gemm.h"

namespace sgm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int GBM = 64, GBN = 64, GBK = 32, GPAD = 8;

template <typename T>
__device__ __forceinline__ float ldf(const void* p, long i) {
    return (float)static_cast<const T*>(p)[i];
}

// Eight consecutive operand elements starting at element i (16-byte aligned),
// converted to bf16.
__device__ __forceinline__ bf16x8 ld8_bf16(const void* p, long i, int f32) {
    bf16x8 r;
    if (f32) {
        const float4* q = reinterpret_cast<const float4*>(static_cast<const float*>(p) + i);
        const float4 u = q[0], v = q[1];
        r[0] = (__bf16)u.x; r[1] = (__bf16)u.y; r[2] = (__bf16)u.z; r[3] = (__bf16)u.w;
        r[4] = (__bf16)v.x; r[5] = (__bf16)v.y; r[6] = (__bf16)v.z; r[7] = (__bf16)v.w;
    } else {
        r = *reinterpret_cast<const bf16x8*>(static_cast<const __bf16*>(p) + i);
    }
    return r;
}

// Stage one operand tile (R rows of the output dimension x GBK along K) into
// LDS as S[r][k] bf16.  vec: 0 scalar, 1 K contiguous, 2 R contiguous (both
// with 8-element aligned chunks); one 8-element chunk per thread.
template <int R>
__device__ __forceinline__ void stage(__bf16 (*S)[GBK + GPAD], const void* P, int f32, long off, long sR, long sK,
                                      int r0, int nR, int k0, int kend, int vec, int tid) {
    if (vec == 1) {
        const int r = tid / (GBK / 8), kc = (tid % (GBK / 8)) * 8;
        const int gr = r0 + r, gk = k0 + kc;
        bf16x8 v;
        if (gr < nR && gk + 7 < kend) {
            v = ld8_bf16(P, off + gr * sR + gk, f32);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                float x = 0.f;
                if (gr < nR && gk + j < kend) x = f32 ? ldf<float>(P, off + gr * sR + gk + j) : ldf<__bf16>(P, off + gr * sR + gk + j);
                v[j] = (__bf16)x;
            }
        }
        *reinterpret_cast<bf16x8*>(&S[r][kc]) = v;
        return;
    }
    if (vec == 2) {
        const int k = tid / (R / 8), rc = (tid % (R / 8)) * 8;
        const int gr = r0 + rc, gk = k0 + k;
        bf16x8 v;
        if (gk < kend && gr + 7 < nR) {
            v = ld8_bf16(P, off + gk * sK + gr, f32);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                float x = 0.f;
                if (gk < kend && gr + j < nR) x = f32 ? ldf<float>(P, off + gk * sK + gr + j) : ldf<__bf16>(P, off + gk * sK + gr + j);
                v[j] = (__bf16)x;
            }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) S[rc + j][k] = v[j];
        return;
    }
    for (int e = tid; e < R * GBK; e += 256) {
        int r, k;
        if (sK == 1) { r = e / GBK; k = e - r * GBK; }
        else { k = e / R; r = e - k * R; }
        const int gr = r0 + r, gk = k0 + k;
        float v = 0.f;
        if (gr < nR && gk < kend) {
            const long i = off + gr * sR + gk * sK;
            v = f32 ? ldf<float>(P, i) : ldf<__bf16>(P, i);
        }
        S[r][k] = (__bf16)v;
    }
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
    for (int k0 = kbeg; k0 < kend; k0 += GBK) {
        stage<GBM>(As, d.A, d.a_f32, aoff, d.sAm, d.sAk, m0, d.M, k0, kend, d.a_vec, tid);
        stage<GBN>(Bs, d.B, d.b_f32, boff, d.sBn, d.sBk, n0, d.N, k0, kend, d.b_vec, tid);
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
            const float val = d.alpha * acc[4 * r + v];
            if (d.c_bf16) {
                reinterpret_cast<__bf16*>(d.C)[coff + (long)row * d.sCm] = (__bf16)val;
                continue;
            }
            float* cp = d.C + coff + (long)row * d.sCm;
            if (d.splitk > 1) atomicAdd(cp, val);
            else *cp = d.beta == 0.f ? val : val + d.beta * *cp;
        }
}

hipError_t gemm(const GemmDesc& d, hipStream_t s) {
    if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return hipSuccess;
    if (d.c_bf16 && (d.beta != 0.f || d.splitk > 1)) return hipErrorInvalidValue;
    const long tiles = (long)((d.M + GBM - 1) / GBM) * ((d.N + GBN - 1) / GBN) * d.batch * (d.splitk > 1 ? d.splitk : 1);
    GemmDesc e = d;
    if (e.splitk < 1) e.splitk = 1;
    // 8-element chunks along the contiguous dimension when every other stride
    // and the base keep them 16-byte aligned
    auto vec = [](const void* p, int f32, long sb, long sr, long sk) {
        const size_t align = f32 ? 32 : 16;
        if ((reinterpret_cast<uintptr_t>(p) % align) != 0 || sb % 8 != 0) return 0;
        if (sk == 1 && sr % 8 == 0) return 1;
        if (sr == 1 && sk % 8 == 0) return 2;
        return 0;
    };
    e.a_vec = vec(d.A, d.a_f32, d.sAb, d.sAm, d.sAk);
    e.b_vec = vec(d.B, d.b_f32, d.sBb, d.sBn, d.sBk);
    hipLaunchKernelGGL(k_gemm, dim3((unsigned)tiles), dim3(256), 0, s, e);
    return hipGetLastError();
}

}  // namespace sgm
