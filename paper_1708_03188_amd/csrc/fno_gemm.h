// Strided batched GEMM on MFMA (bf16 inputs, fp32 accumulate) - internal.
#pragma once
#include <hip/hip_runtime.h>

namespace sgm {

struct GemmDesc {
    int M, N, K, batch;
    const void* A;
    long sAb, sAm, sAk;  // element strides of A(b, m, k)
    const void* B;
    long sBb, sBk, sBn;  // element strides of B(b, k, n)
    float* C;
    long sCb, sCm, sCn;  // element strides of C(b, m, n)
    float alpha, beta;
    int a_f32, b_f32;    // operand element type: 1 = float (rounded to bf16 on load), 0 = bf16
    int c_bf16;          // 1: C is bf16 storage, written rounded (needs beta = 0, splitk = 1)
    int splitk;          // > 1: K is split over blocks and the partial sums are added
                         // atomically into C (C must hold beta * C beforehand)
    int a_vec, b_vec;    // set by gemm(): staging along the contiguous dimension
};

// C = alpha op(A) op(B) + beta C for every batch entry.
hipError_t gemm(const GemmDesc& d, hipStream_t s);

}  // namespace sgm
