// Fused FNO row kernels (width 32, 16 x-modes) - internal.
#pragma once
#include <hip/hip_runtime.h>

namespace sgm {

// GELU on erf by Abramowitz & Stegun 7.1.26 (absolute error <= 1.5e-7, far
// below the bf16 rounding every activation goes through), written through erfc:
// with x = z / sqrt 2, 1 - erf|x| = q(t) t exp(-x^2), t = 1 / (1 + p |x|), and,
// for either sign of z,
// z (1 + erf x) / 2 = z / 2 + |z| (1/2 - (1 - erf|x|) / 2).
// The 1/sqrt 2, the -1/2 and log2 e are folded into the constants (10 plain
// operations and two transcendental ones).
__device__ __forceinline__ float fno_gelu(float z) {
    const float az = fabsf(z);
    const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f * 0.70710678118654752f, az, 1.f));
    float q = __builtin_fmaf(-0.5f * 1.061405429f, t, -0.5f * -1.453152027f);
    q = __builtin_fmaf(q, t, -0.5f * 1.421413741f);
    q = __builtin_fmaf(q, t, -0.5f * -0.284496736f);
    q = __builtin_fmaf(q, t, -0.5f * 0.254829592f);
    // exp(-z^2 / 2) = 2^(-z^2 log2(e) / 2)
    const float e = __builtin_amdgcn_exp2f(z * z * (-0.5f * 1.4426950408889634f));
    return __builtin_fmaf(az, __builtin_fmaf(q * t, e, 0.5f), 0.5f * z);
}
// GELU and its derivative from one evaluation of the same approximation: with
// m = erf(|z| / sqrt 2) / 2 (the fma inside fno_gelu) and e = exp(-z^2 / 2),
// gelu = z / 2 + |z| m (bit-identical to fno_gelu) and
// gelu' = Phi(z) + z phi(z) = 1/2 + sign(z) m + z e / sqrt(2 pi).
__device__ __forceinline__ void fno_gelu_fd(float z, float& f, float& d) {
    const float az = fabsf(z);
    const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f * 0.70710678118654752f, az, 1.f));
    float q = __builtin_fmaf(-0.5f * 1.061405429f, t, -0.5f * -1.453152027f);
    q = __builtin_fmaf(q, t, -0.5f * 1.421413741f);
    q = __builtin_fmaf(q, t, -0.5f * -0.284496736f);
    q = __builtin_fmaf(q, t, -0.5f * 0.254829592f);
    const float e = __builtin_amdgcn_exp2f(z * z * (-0.5f * 1.4426950408889634f));
    const float m = __builtin_fmaf(q * t, e, 0.5f);
    f = __builtin_fmaf(az, m, 0.5f * z);
    d = __builtin_fmaf(z * e, 0.39894228040143268f, 0.5f + copysignf(m, z));
}
__device__ __forceinline__ float fno_gelu_d(float z) {
    float f, d;
    fno_gelu_fd(z, f, d);
    return d;
}

struct FnoLayerArgs {
    const __bf16* a;      // layer input [rows][W][32]
    const __bf16* U;      // inverse-y spectral rows [rows][32][32] (may alias Tn)
    __bf16* Tn;           // next layer's x-DFT rows [rows][32][32] (mode 0)
    const __bf16* Gx;     // [W][32] inverse x-DFT
    const __bf16* Fx;     // [32][W] forward x-DFT
    const __bf16* Wp;     // [32][32] pointwise weights
    const float* bp;      // [32]
    __bf16* a_out;        // [rows][W][32] (modes 0, 1, 3)
    __bf16* zsave;        // pre-activation [rows][W][32] or null (modes 0, 1, 3)
    long rows;
    int W;
    int act;              // 1: GELU
    // projection (modes 2, 3)
    const __bf16* W1T;    // [P][32]
    const float* b1;      // [P]
    const __bf16* W2;     // [P][2]
    const __bf16* W2P;    // [P/16][64 lanes][8]: W2 as MFMA A operands (mode 2)
    const float* b2;      // [2]
    const float* x;       // [rows][W][2] network input (residual)
    float* pred;          // [rows][W][2]
    int P;
};

// Work-groups of the fused backward kernels (persistent grids): each writes one
// row of partial parameter gradients, summed afterwards by launch_fno_sum_partials
// (device-scope atomics from every work-group onto the same few cache lines are
// serialised).
constexpr int kFnoBwdMaxGroups = 512;

// Backward of the projection pred = x + gelu(a W1 + b1) W2 + b2 over tiles of
// 32 pixels, with the hidden pre-activation recomputed from a (it is not kept):
// da = dz W1^T (overwritten) and the parameter gradients gW1 = a^T dz ([32][P]),
// gb1 = sum dz, gW2 = h^T dpred ([P][2]) as per-work-group partials, with
// dz = (dpred W2^T) gelu'(z) rounded to bf16 and dpred rounded to bf16 as the
// products' operands.
struct FnoProjBwdArgs {
    const __bf16* a;      // last layer output [pix][32]
    const float* dpred;   // [pix][2]
    const __bf16* W1T;    // [P][32]
    const __bf16* W1;     // [32][P]
    const float* b1;      // [P]
    const __bf16* W2;     // [P][2]
    float* da;            // [pix][32]
    // per-work-group partial sums, one row of 32 P + 3 P values per work-group:
    // gW1 [32][P], gb1 [P], gW2 [P][2] (the grid is at most kFnoBwdMaxGroups)
    float* part;
    long pix;             // multiple of 32
    int P;                // 32, 64 or 128
};

// Backward of one spectral layer a' = act(Gx U + a Wp + bp), one wave per
// activation row (b, y), for the fused shapes.  In: da = gradient of the layer
// output (fp32), completed on the fly by Fx^T gT of the layer above when addT
// (gT: T's rows, fp32).  Out: da = dz Wp^T (the pointwise part of the input
// gradient, overwritten in place), T = Gx^T dz per row (the adjoint of the
// inverse x-DFT, overwriting gT row by row), gWp = a^T dz and gbp = sum dz as
// per-work-group partials, with dz = da gelu'(z) (or da when !act) rounded to bf16.
struct FnoLayerBwdArgs {
    float* da;            // [rows][W][32]
    float* T;             // [rows][32][32]
    const __bf16* z;      // [rows][W][32] pre-activation (read when act)
    const __bf16* aprev;  // [rows][W][32] layer input
    const __bf16* Wp;     // [32][32]
    const __bf16* FxT;    // [W][32] forward x-DFT, transposed
    const __bf16* GxT;    // [32][W] inverse x-DFT, transposed
    float* part;          // per-work-group rows of 32 x 32 + 32 values: gWp [32][32], gbp [32]
    long rows;
    int W;
    int act;
    int addT;
};
hipError_t launch_fno_layer_bwd(const FnoLayerBwdArgs& a, hipStream_t s);
// Backward of the lift a0 = x Wl + bl after the first layer's backward: with
// da0 = da + Fx^T gT (da: the first layer's pointwise input gradient, gT: T's
// rows, both fp32), per-work-group partial rows of gWl = x^T da0 ([2][32]) and
// gbl = sum da0 ([32]); one wave per activation row, da0 is not stored.
hipError_t launch_fno_lift_bwd(const float* da, const float* T, const float* x, const __bf16* FxT, long rows, int W,
                               float* part, hipStream_t s);
// Work-groups (= partial rows) a backward launch over `rows` rows / `pix` pixels uses.
int fno_layer_bwd_groups(long rows);
int fno_proj_bwd_groups(long pix, int P);
// out[v] += sum over r < nrows of part[r nvals + v]
hipError_t launch_fno_sum_partials(const float* part, int nrows, int nvals, float* out, hipStream_t s);

bool fno_fused_ok(int C, int K, int W, int P);
// The fused projection backward handles width 32 with P in {32, 64, 128}.
bool fno_proj_bwd_ok(int C, int P);
hipError_t launch_fno_proj_bwd(const FnoProjBwdArgs& a, hipStream_t s);
// W2 [P][2] (bf16) -> the A operands of the projection's second MFMA (P % 32 == 0).
hipError_t launch_fno_w2_operands(const __bf16* W2, __bf16* W2P, int P, hipStream_t s);
hipError_t launch_fno_lift_dft(const float* x, const float* Wl, const float* bl, const __bf16* Fx, __bf16* a0,
                               __bf16* T, long rows, int W, hipStream_t s);
// mode 0: a_out + next T; 1: a_out (last layer); 2: projection to pred (last
// layer); 3: a_out, z and the projection to pred (last layer, training)
hipError_t launch_fno_layer(const FnoLayerArgs& a, int mode, hipStream_t s);
hipError_t launch_transpose_bf16(const float* in, __bf16* out, int R, int Cc, hipStream_t s);

}  // namespace sgm
