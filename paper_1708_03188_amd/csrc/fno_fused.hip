// Fused FNO row kernels for width 32 and 16 retained x-modes (2K = 32 real
// DFT rows): one wave per activation row (b, y) of W pixels x 32 channels.
//
// MFMA v_mfma_f32_32x32x16_bf16 operand layout: lane i (c = i % 32,
// g = i / 32) supplies A[c][8 g + v] and B[8 g + v][c], v = 0..7, and
// receives C[8 r + 4 g + v][c] in accumulator 4 r + v.
//
//  k_fno_lift_dft : a0 = x Wl + bl (stored), T = Fx a0 (x-DFT of layer 0).
//  k_fno_layer    : z = Gx U + a Wp + bp over the concatenated K = 2K + C,
//                   a' = gelu(z) (not after the last layer), stored with z
//                   when training; the next layer's x-DFT T = Fx a' is taken
//                   from the accumulators directly (no re-read of a'), and
//                   for inference after the last layer the projection
//                   pred = x + gelu(a' W1 + b1) W2 + b2 runs in the same pass.
// The next-layer DFT chains the two MFMAs without data movement: the output
// rows x = 8 r + 4 g + v that lane group g holds are taken as that group's
// eight K entries, and Fx is read in the same permuted order.
#include "fno_fused.h"

namespace sgm {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int FC = 32;   // channels
constexpr int F2K = 32;  // real x-DFT rows (Re, Im of 16 modes)
constexpr int WAVES = 4;

__device__ __forceinline__ float gelu(float z) { return fno_gelu(z); }

__device__ __forceinline__ bf16x8 ld8(const bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }

__device__ __forceinline__ floatx16 zero16() {
    floatx16 a;
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = 0.f;
    return a;
}

__device__ __forceinline__ floatx16 mfma(bf16x8 a, bf16x8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

}  // namespace

__global__ void __launch_bounds__(64 * WAVES) k_fno_lift_dft(const float* __restrict__ x, const float* __restrict__ Wl,
                                                           const float* __restrict__ bl, const bf16* __restrict__ Fx,
                                                           bf16* __restrict__ a0, bf16* __restrict__ T, long rows,
                                                           int W) {
    // the row's input, 256 pixels at a time, staged by coalesced loads: each lane
    // then reads the eight pixels it lifts from LDS instead of eight dependent
    // broadcast loads per 16 pixels; a0 leaves through an LDS tile in 16-byte runs
    constexpr int XCH = 256;
    __shared__ float2 xs[WAVES][XCH];
    __shared__ bf16 tile[WAVES][32][FC + 8];
    const long row = (long)blockIdx.x * WAVES + (threadIdx.x >> 6);
    const bool live = row < rows;  // waves past the end still reach the barriers
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63, c = lane & 31, g = lane >> 5;
    const long rr = live ? row : 0;
    const float w0 = Wl[c], w1 = Wl[FC + c], b = bl[c];
    const float2* xr = reinterpret_cast<const float2*>(x) + rr * W;
    bf16* ar = a0 + rr * W * FC;
    floatx16 acc = zero16();
    for (int ch0 = 0; ch0 < W; ch0 += XCH) {
        const int n = W - ch0 < XCH ? W - ch0 : XCH;  // a multiple of 32
        for (int i = lane; i < n; i += 64) xs[wv][i] = xr[ch0 + i];
        __syncthreads();
        for (int s2 = 0; s2 < n / 32; ++s2) {
            // 32 pixels: each lane lifts channel c of eight pixels per half, feeds them to
            // the x-DFT and parks them in the wave's tile [pixel][channel] ...
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int p0 = 32 * s2 + 16 * h + 8 * g;
                bf16x8 bop;
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    const float2 u = xs[wv][p0 + v];
                    bop[v] = (bf16)(u.x * w0 + u.y * w1 + b);
                    tile[wv][16 * h + 8 * g + v][c] = bop[v];
                }
                acc = mfma(ld8(Fx + (long)c * W + ch0 + p0), bop, acc);
            }
            __syncthreads();
            // ... from which each lane stores 32 bytes: half of one pixel's channels
            const int pl = lane >> 1, cc = 16 * (lane & 1);
            const bf16x8 q0 = *reinterpret_cast<const bf16x8*>(&tile[wv][pl][cc]);
            const bf16x8 q1 = *reinterpret_cast<const bf16x8*>(&tile[wv][pl][cc + 8]);
            if (live) {
                bf16* o = ar + (long)(ch0 + 32 * s2 + pl) * FC + cc;
                *reinterpret_cast<bf16x8*>(o) = q0;
                *reinterpret_cast<bf16x8*>(o + 8) = q1;
            }
            __syncthreads();
        }
    }
    if (live) {
        bf16* tr = T + rr * F2K * FC;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int v = 0; v < 4; ++v) tr[(8 * r + 4 * g + v) * FC + c] = (bf16)acc[4 * r + v];
    }
}

// MODE 0: a_out and the next layer's T; 1: a_out only (last layer, training);
// 2: projection to pred (last layer, inference).  Both products of the
// projection run on MFMA: the GELU'd hidden accumulators of one 32-unit block
// are taken directly as the B operand of two 32x32x16 MFMAs for the P -> 2
// product (lane group g's eight K entries are its own accumulator rows
// 8 kb + v), with W2 read in that permuted order and padded to 32 output rows
// (k_fno_w2_operands); rows 0, 1 of the result are the two outputs.
template <int MODE>
__global__ void __launch_bounds__(64 * WAVES) k_fno_layer(FnoLayerArgs p) {
    __shared__ bf16 tile[WAVES][32][FC + 8];
    const long row = (long)blockIdx.x * WAVES + (threadIdx.x >> 6);
    const bool live = row < p.rows;  // waves past the end still reach the barriers
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63, c = lane & 31, g = lane >> 5;
    const long rr = live ? row : 0;
    const int W = p.W;
    // B operand over the concatenated K: U rows (x-spectral input) then Wp
    bf16x8 bop[4];
    {
        const bf16* u = p.U + rr * F2K * FC;
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int v = 0; v < 8; ++v) bop[s][v] = u[(16 * s + 8 * g + v) * FC + c];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int v = 0; v < 8; ++v) bop[2 + s][v] = p.Wp[(16 * s + 8 * g + v) * FC + c];
    }
    const float bias = p.bp[c];
    const bf16* ar = p.a + rr * W * FC;
    floatx16 tacc = zero16();
    for (int t = 0; t < W / 32; ++t) {
        const int x0 = 32 * t;
        // every accumulator entry of a lane is output channel c: start from its bias
        floatx16 acc;
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[e] = bias;
#pragma unroll
        for (int s = 0; s < 2; ++s) acc = mfma(ld8(p.Gx + (long)(x0 + c) * F2K + 16 * s + 8 * g), bop[s], acc);
#pragma unroll
        for (int s = 0; s < 2; ++s) acc = mfma(ld8(ar + (long)(x0 + c) * FC + 16 * s + 8 * g), bop[2 + s], acc);
        bf16x8 yb[2], zb[2];
        if (p.act) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                zb[e >> 3][e & 7] = (bf16)acc[e];
                yb[e >> 3][e & 7] = (bf16)gelu(acc[e]);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) zb[e >> 3][e & 7] = yb[e >> 3][e & 7] = (bf16)acc[e];
        }
        if constexpr (MODE != 2) {
            // a' (and z) of the 32 pixels through the wave's LDS tile, so that each lane
            // stores 16-byte runs of one pixel's channels instead of single values
            auto store_tile = [&](const bf16x8 (&v)[2], bf16* dst) {
#pragma unroll
                for (int e = 0; e < 16; ++e) tile[wv][8 * (e >> 2) + 4 * g + (e & 3)][c] = v[e >> 3][e & 7];
                __syncthreads();
                const int pl = lane >> 1, ch = 16 * (lane & 1);
                const bf16x8 w0 = *reinterpret_cast<const bf16x8*>(&tile[wv][pl][ch]);
                const bf16x8 w1 = *reinterpret_cast<const bf16x8*>(&tile[wv][pl][ch + 8]);
                if (live) {
                    bf16* o = dst + (rr * W + x0 + pl) * FC + ch;
                    *reinterpret_cast<bf16x8*>(o) = w0;
                    *reinterpret_cast<bf16x8*>(o + 8) = w1;
                }
                __syncthreads();
            };
            if (p.zsave) store_tile(zb, p.zsave);
            store_tile(yb, p.a_out);
        }
        if constexpr (MODE == 0) {
            // next x-DFT: k = 8 g + v <-> pixel x0 + 16 q + 8 (v / 4) + 4 g + v % 4
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const bf16* f = p.Fx + (long)c * W + x0 + 16 * q + 4 * g;
                const bf16x4 lo = *reinterpret_cast<const bf16x4*>(f);
                const bf16x4 hi = *reinterpret_cast<const bf16x4*>(f + 8);
                bf16x8 aop;
#pragma unroll
                for (int v = 0; v < 4; ++v) { aop[v] = lo[v]; aop[4 + v] = hi[v]; }
                tacc = mfma(aop, yb[q], tacc);
            }
        }
        if constexpr (MODE == 2) {
            // a' tile [pixel][channel] through LDS, then h^T = W1T a'^T per 32 hidden units
#pragma unroll
            for (int e = 0; e < 16; ++e) tile[wv][8 * (e >> 2) + 4 * g + (e & 3)][c] = yb[e >> 3][e & 7];
            __syncthreads();
            bf16x8 bt[2];
#pragma unroll
            for (int s = 0; s < 2; ++s) bt[s] = *reinterpret_cast<const bf16x8*>(&tile[wv][c][16 * s + 8 * g]);
            floatx16 o2 = zero16();
            for (int T = 0; T < p.P / 32; ++T) {
                // the accumulator starts from b1: entry e is hidden unit 32 T + 8 (e / 4) + 4 g + e % 4,
                // so each run of four entries is one 16-byte load (b1 is 16-byte aligned)
                floatx16 h;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float4 bb = *reinterpret_cast<const float4*>(p.b1 + 32 * T + 8 * j + 4 * g);
                    h[4 * j] = bb.x;
                    h[4 * j + 1] = bb.y;
                    h[4 * j + 2] = bb.z;
                    h[4 * j + 3] = bb.w;
                }
#pragma unroll
                for (int s = 0; s < 2; ++s) h = mfma(ld8(p.W1T + (long)(32 * T + c) * FC + 16 * s + 8 * g), bt[s], h);
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    bf16x8 hop;
#pragma unroll
                    for (int v = 0; v < 8; ++v) hop[v] = (bf16)gelu(h[8 * kb + v]);
                    o2 = mfma(ld8(p.W2P + ((long)(2 * T + kb) * 64 + lane) * 8), hop, o2);
                }
            }
            // rows 0 and 1 of the padded product, in lane group 0
            const float o0 = o2[0], o1 = o2[1];
            if (live && g == 0) {
                const long pi = rr * W + x0 + c;
                const float2 xin = reinterpret_cast<const float2*>(p.x)[pi];
                reinterpret_cast<float2*>(p.pred)[pi] = make_float2(xin.x + o0 + p.b2[0], xin.y + o1 + p.b2[1]);
            }
            __syncthreads();
        }
    }
    if constexpr (MODE == 0) {
        if (live) {
            bf16* tr = p.Tn + rr * F2K * FC;
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int v = 0; v < 4; ++v) tr[(8 * r + 4 * g + v) * FC + c] = (bf16)tacc[4 * r + v];
        }
    }
}

__global__ void k_transpose_bf16(const float* in, bf16* out, int R, int Cc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= R * Cc) return;
    const int r = i / Cc, c = i - r * Cc;
    out[(long)c * R + r] = (bf16)in[i];
}

// A operand of k-block kg (= 2 T + kb) for lane l (output row o = l % 32, lane
// group g = l / 32), entry v: W2[h][o] with h = 32 T + 16 kb + 8 (v / 4) + 4 g + v % 4
// for o < 2, zero for the padding rows.
__global__ void k_fno_w2_operands(const bf16* W2, bf16* W2P, int P) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (P / 16) * 512) return;
    const int kg = i / 512, l = (i / 8) % 64, v = i % 8;
    const int o = l % 32, g = l / 32, T = kg / 2, kb = kg % 2;
    const int h = 32 * T + 16 * kb + 8 * (v / 4) + 4 * g + (v % 4);
    W2P[i] = o < 2 ? W2[2 * h + o] : (bf16)0.f;
}

hipError_t launch_fno_w2_operands(const bf16* W2, bf16* W2P, int P, hipStream_t s) {
    const int n = (P / 16) * 512;
    hipLaunchKernelGGL(k_fno_w2_operands, dim3((n + 255) / 256), dim3(256), 0, s, W2, W2P, P);
    return hipGetLastError();
}

bool fno_fused_ok(int C, int K, int W, int P) { return C == FC && 2 * K == F2K && W % 32 == 0 && P % 32 == 0; }

hipError_t launch_fno_lift_dft(const float* x, const float* Wl, const float* bl, const bf16* Fx, bf16* a0, bf16* T,
                               long rows, int W, hipStream_t s) {
    hipLaunchKernelGGL(k_fno_lift_dft, dim3((unsigned)((rows + WAVES - 1) / WAVES)), dim3(64 * WAVES), 0, s, x, Wl, bl,
                       Fx, a0, T, rows, W);
    return hipGetLastError();
}

hipError_t launch_fno_layer(const FnoLayerArgs& a, int mode, hipStream_t s) {
    if (mode == 2 && (reinterpret_cast<uintptr_t>(a.b1) & 15) != 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.rows + WAVES - 1) / WAVES)), block(64 * WAVES);
    if (mode == 0) hipLaunchKernelGGL(k_fno_layer<0>, grid, block, 0, s, a);
    else if (mode == 1) hipLaunchKernelGGL(k_fno_layer<1>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(k_fno_layer<2>, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_transpose_bf16(const float* in, bf16* out, int R, int Cc, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose_bf16, dim3((R * Cc + 255) / 256), dim3(256), 0, s, in, out, R, Cc);
    return hipGetLastError();
}

}  // namespace sgm
