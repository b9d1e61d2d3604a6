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

#include <algorithm>

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
        // U may alias Tn, which row 0's wave rewrites: a wave past the end reads no U
        const bf16* u = p.U + rr * F2K * FC;
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int v = 0; v < 8; ++v) bop[s][v] = live ? u[(16 * s + 8 * g + v) * FC + c] : (bf16)0.f;
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
        if constexpr (MODE >= 2) {
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
    if (mode >= 2 && (reinterpret_cast<uintptr_t>(a.b1) & 15) != 0) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((a.rows + WAVES - 1) / WAVES)), block(64 * WAVES);
    if (mode == 0) hipLaunchKernelGGL(k_fno_layer<0>, grid, block, 0, s, a);
    else if (mode == 1) hipLaunchKernelGGL(k_fno_layer<1>, grid, block, 0, s, a);
    else if (mode == 2) hipLaunchKernelGGL(k_fno_layer<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(k_fno_layer<3>, grid, block, 0, s, a);
    return hipGetLastError();
}

// Projection backward, one wave per tile of 32 pixels (persistent work-groups,
// uniform trip count so the barriers are reached by every wave).  Per hidden
// block of 32 units T:
//   z  = a W1 + b1      rows = pixels (A = a), cols = hidden units (B = W1T rows)
//   dz = (dpred W2^T) gelu'(z), h = gelu(z)   per accumulator entry
//   gW1^T += dz^T a     A = dz straight from the accumulators (K = the lane's
//                       16 pixels in accumulator order), B = a^T from LDS in
//                       the same pixel order
//   da  += dz W1^T      A = dz rows through LDS, B = W1 rows
// gW2 and gb1 are per-lane sums over the lane's pixels of one hidden unit.
template <int NT>
__global__ void __launch_bounds__(64 * WAVES) k_fno_proj_bwd(FnoProjBwdArgs p) {
    constexpr int LD = FC + 8;
    __shared__ bf16 sm[WAVES][1 + NT][32][LD];  // [0]: a tile [pixel][channel]; [1 + T]: dz [pixel][unit]
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63, c = lane & 31, g = lane >> 5;
    const int P = p.P;
    const long ntiles = p.pix / 32, nbt = (ntiles + WAVES - 1) / WAVES;
    floatx16 gw1[NT];
    float gw2a[NT], gw2b[NT], gb[NT];
#pragma unroll
    for (int T = 0; T < NT; ++T) { gw1[T] = zero16(); gw2a[T] = gw2b[T] = gb[T] = 0.f; }
    float w2a[NT], w2b[NT], bb[NT];
#pragma unroll
    for (int T = 0; T < NT; ++T) {
        w2a[T] = (float)p.W2[2 * (32 * T + c)];
        w2b[T] = (float)p.W2[2 * (32 * T + c) + 1];
        bb[T] = p.b1[32 * T + c];
    }
    for (long bt = blockIdx.x; bt < nbt; bt += gridDim.x) {
        const long tile = bt * WAVES + wv;
        const bool live = tile < ntiles;
        const long p0 = live ? tile * 32 : 0;
        const bf16* ar = p.a + p0 * FC;
        bf16x8 aop[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) aop[s] = ld8(ar + (long)c * FC + 16 * s + 8 * g);
        // dpred of the lane's 16 pixels (entry e <-> pixel 8 (e / 4) + 4 g + e % 4), zero on a dead tile
        float d0[16], d1[16];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const float2 d = live ? reinterpret_cast<const float2*>(p.dpred)[p0 + 8 * (e >> 2) + 4 * g + (e & 3)]
                                  : make_float2(0.f, 0.f);
            d0[e] = (float)(bf16)d.x;
            d1[e] = (float)(bf16)d.y;
        }
        __syncthreads();  // the previous tile's LDS reads are done
#pragma unroll
        for (int s = 0; s < 2; ++s) *reinterpret_cast<bf16x8*>(&sm[wv][0][c][16 * s + 8 * g]) = aop[s];
        __syncthreads();
        // a^T in accumulator pixel order: K entry 8 g + v of step q <-> pixel 16 q + 8 (v / 4) + 4 g + v % 4
        bf16x8 at[2];
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int v = 0; v < 8; ++v) at[q][v] = sm[wv][0][16 * q + 8 * (v >> 2) + 4 * g + (v & 3)][c];
#pragma unroll
        for (int T = 0; T < NT; ++T) {
            floatx16 h;
#pragma unroll
            for (int e = 0; e < 16; ++e) h[e] = bb[T];
#pragma unroll
            for (int s = 0; s < 2; ++s) h = mfma(aop[s], ld8(p.W1T + (long)(32 * T + c) * FC + 16 * s + 8 * g), h);
            bf16x8 dz[2];
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                float gf, gd;
                fno_gelu_fd(h[e], gf, gd);
                const float hv = (float)(bf16)gf;
                const bf16 dzv = (bf16)((d0[e] * w2a[T] + d1[e] * w2b[T]) * gd);
                dz[e >> 3][e & 7] = dzv;
                gw2a[T] += hv * d0[e];
                gw2b[T] += hv * d1[e];
                gb[T] += (float)dzv;
                sm[wv][1 + T][8 * (e >> 2) + 4 * g + (e & 3)][c] = dzv;
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) gw1[T] = mfma(dz[q], at[q], gw1[T]);
        }
        __syncthreads();
        floatx16 da = zero16();
#pragma unroll
        for (int T = 0; T < NT; ++T)
#pragma unroll
            for (int s = 0; s < 2; ++s)
                da = mfma(*reinterpret_cast<const bf16x8*>(&sm[wv][1 + T][c][16 * s + 8 * g]),
                          ld8(p.W1 + (long)c * P + 32 * T + 16 * s + 8 * g), da);
        if (live) {
#pragma unroll
            for (int e = 0; e < 16; ++e) p.da[(p0 + 8 * (e >> 2) + 4 * g + (e & 3)) * FC + c] = da[e];
        }
    }
    // block reduction of the parameter gradients through LDS into this work-group's partial row
    __syncthreads();
    float* prow = p.part + (long)blockIdx.x * 35 * P;
    float* red = reinterpret_cast<float*>(&sm[0][0][0][0]);  // >= WAVES * 64 * 16 floats
    static_assert(sizeof(sm) >= sizeof(float) * WAVES * 64 * 16, "reduction buffer");
#pragma unroll
    for (int T = 0; T < NT; ++T) {
#pragma unroll
        for (int e = 0; e < 16; ++e) red[(wv * 64 + lane) * 16 + e] = gw1[T][e];
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * 16; i += 64 * WAVES) {
            float sum = 0.f;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) sum += red[w * 64 * 16 + i];
            const int ln = i >> 4, e = i & 15;
            // entry e of lane (channel ln % 32, group ln / 32): unit 32 T + 8 (e / 4) + 4 g + e % 4
            const int unit = 32 * T + 8 * (e >> 2) + 4 * (ln >> 5) + (e & 3);
            prow[(long)(ln & 31) * P + unit] = sum;
        }
        __syncthreads();
    }
#pragma unroll
    for (int T = 0; T < NT; ++T) {
        red[(wv * 64 + lane) * 3 * NT + 3 * T] = gw2a[T];
        red[(wv * 64 + lane) * 3 * NT + 3 * T + 1] = gw2b[T];
        red[(wv * 64 + lane) * 3 * NT + 3 * T + 2] = gb[T];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 32 * 3 * NT; i += 64 * WAVES) {
        // unit 32 T + cc: lanes cc and cc + 32 of every wave
        const int cc = i / (3 * NT), k = i % (3 * NT), T = k / 3, which = k % 3;
        float sum = 0.f;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) sum += red[(w * 64 + cc) * 3 * NT + k] + red[(w * 64 + cc + 32) * 3 * NT + k];
        const int unit = 32 * T + cc;
        if (which == 2) prow[32 * P + unit] = sum;
        else prow[33 * P + 2 * unit + which] = sum;
    }
}

// Layer backward, one wave per row.  Accumulator ("pixel") layout of a 32-pixel
// tile: lane (channel c, group g) entry e holds pixel 8 (e / 4) + 4 g + e % 4.
//   da  = da_in + Fx^T gT        A = FxT rows (pixels), B = gT (bf16)
//   dz  = da gelu'(z)            per entry
//   gWp += a^T dz                A = a in the accumulator pixel order (K = the
//                                lane group's pixels), B = dz from the accumulators
//   gU  += Gx^T dz               A = GxT in the same pixel order, B = dz
//   da' = dz Wp^T                A = dz rows through LDS, B = Wp rows
__global__ void __launch_bounds__(64 * WAVES) k_fno_layer_bwd(FnoLayerBwdArgs p) {
    // per-wave tiles: da [pixel][channel] fp32, z, a and dz [pixel][channel] bf16
    __shared__ float sda[WAVES][32][FC + 4];
    __shared__ bf16 sz[WAVES][32][FC + 8], sap[WAVES][32][FC + 8], sdz[WAVES][32][FC + 8];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: row tests branch per wave
    const int lane = threadIdx.x & 63, c = lane & 31, g = lane >> 5;
    const int W = p.W, nt = W / 32;
    bf16x8 wb[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) wb[s] = ld8(p.Wp + c * FC + 16 * s + 8 * g);
    floatx16 gw = zero16(), gwr = zero16(), uacc = zero16();
    float gb = 0.f, gbr = 0.f;
    bf16x8 tb[2];
    // a tile is 32 consecutive pixels of one row: contiguous 4 KB of da, 2 KB of z and of a.
    // Lane loads: da float4 i = j * 64 + lane (pixel i / 8, channels 4 (i % 8)..), z and a 16-byte
    // chunk i = j * 64 + lane (pixel i / 4, channels 8 (i % 4)..), j = 0..3 and 0..1.
    // the next step's tile, in flight during this step (named registers, not arrays)
    float4 nd0, nd1, nd2, nd3;
    uint4 nz0, nz1, na0, na1;
    // rows past the end get zeros (their addresses are clamped to row 0, which another
    // wave may be updating in place; whatever such a load returns is discarded)
    auto fetch = [&](long row, int tile) __attribute__((always_inline)) {
        const bool ok = row < p.rows;
        const long pb = (ok ? row : 0) * W + 32 * tile;
        const float4* d4 = reinterpret_cast<const float4*>(p.da + pb * FC);
        const uint4* z4 = reinterpret_cast<const uint4*>(p.z + pb * FC);
        const uint4* a4 = reinterpret_cast<const uint4*>(p.aprev + pb * FC);
        const float4 f0 = make_float4(0.f, 0.f, 0.f, 0.f);
        const uint4 u0 = make_uint4(0, 0, 0, 0);
        nd0 = ok ? d4[lane] : f0;
        nd1 = ok ? d4[64 + lane] : f0;
        nd2 = ok ? d4[128 + lane] : f0;
        nd3 = ok ? d4[192 + lane] : f0;
        nz0 = ok ? z4[lane] : u0;
        nz1 = ok ? z4[64 + lane] : u0;
        na0 = ok ? a4[lane] : u0;
        na1 = ok ? a4[64 + lane] : u0;
    };
    // (row group, tile) steps, the same sequence for every wave of the block; rows past
    // the end compute on zeros and discard
    const long ngr = (p.rows + WAVES - 1) / WAVES;
    long gr = blockIdx.x;
    int t = 0;
    if (gr < ngr) fetch(gr * WAVES + wv, 0);
    while (gr < ngr) {
        const long row = gr * WAVES + wv;
        const bool live = row < p.rows;
        const long rr = live ? row : 0;
        const int x0 = 32 * t;
        const long pb = rr * W + x0;
        if (t == 0) {
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int v = 0; v < 8; ++v)
                    tb[s][v] = (p.addT && live) ? (bf16)p.T[rr * F2K * FC + (16 * s + 8 * g + v) * FC + c] : (bf16)0.f;
            uacc = zero16();
            gwr = zero16();
            gbr = 0.f;
        }
        __syncthreads();  // the previous step's LDS reads are done
        // float4 i of the tile: pixel i / 8, channels 4 (i % 8)..; 16-byte chunk i: pixel i / 4, channels 8 (i % 4)..
        *reinterpret_cast<float4*>(&sda[wv][lane >> 3][4 * (lane & 7)]) = nd0;
        *reinterpret_cast<float4*>(&sda[wv][8 + (lane >> 3)][4 * (lane & 7)]) = nd1;
        *reinterpret_cast<float4*>(&sda[wv][16 + (lane >> 3)][4 * (lane & 7)]) = nd2;
        *reinterpret_cast<float4*>(&sda[wv][24 + (lane >> 3)][4 * (lane & 7)]) = nd3;
        *reinterpret_cast<uint4*>(&sz[wv][lane >> 2][8 * (lane & 3)]) = nz0;
        *reinterpret_cast<uint4*>(&sz[wv][16 + (lane >> 2)][8 * (lane & 3)]) = nz1;
        *reinterpret_cast<uint4*>(&sap[wv][lane >> 2][8 * (lane & 3)]) = na0;
        *reinterpret_cast<uint4*>(&sap[wv][16 + (lane >> 2)][8 * (lane & 3)]) = na1;
        // next step's tile, in flight during this step
        int tn = t + 1;
        long grn = gr;
        if (tn == nt) { tn = 0; grn += gridDim.x; }
        if (grn < ngr) fetch(grn * WAVES + wv, tn);
        __syncthreads();
        floatx16 acc;
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[e] = sda[wv][8 * (e >> 2) + 4 * g + (e & 3)][c];
        if (p.addT) {
#pragma unroll
            for (int s = 0; s < 2; ++s) acc = mfma(ld8(p.FxT + (long)(x0 + c) * F2K + 16 * s + 8 * g), tb[s], acc);
        }
        bf16x8 dz[2];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int pe = 8 * (e >> 2) + 4 * g + (e & 3);
            float v = acc[e];
            if (p.act) v *= fno_gelu_d((float)sz[wv][pe][c]);
            const bf16 d = (bf16)v;
            dz[e >> 3][e & 7] = d;
            gbr += (float)d;
            sdz[wv][pe][c] = d;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            // K entry 8 g + v <-> pixel 16 q + 8 (v / 4) + 4 g + v % 4 (accumulator entries 8 q + v)
            bf16x8 ap;
#pragma unroll
            for (int v = 0; v < 8; ++v) ap[v] = sap[wv][16 * q + 8 * (v >> 2) + 4 * g + (v & 3)][c];
            gwr = mfma(ap, dz[q], gwr);
            const bf16* gx = p.GxT + (long)c * W + x0 + 16 * q + 4 * g;
            const bf16x4 lo = *reinterpret_cast<const bf16x4*>(gx);
            const bf16x4 hi = *reinterpret_cast<const bf16x4*>(gx + 8);
            bf16x8 gop;
#pragma unroll
            for (int v = 0; v < 4; ++v) { gop[v] = lo[v]; gop[4 + v] = hi[v]; }
            uacc = mfma(gop, dz[q], uacc);
        }
        __syncthreads();
        floatx16 dout = zero16();
#pragma unroll
        for (int s = 0; s < 2; ++s) dout = mfma(*reinterpret_cast<const bf16x8*>(&sdz[wv][c][16 * s + 8 * g]), wb[s], dout);
        if (live) {
#pragma unroll
            for (int e = 0; e < 16; ++e) p.da[(pb + 8 * (e >> 2) + 4 * g + (e & 3)) * FC + c] = dout[e];
        }
        if (t == nt - 1 && live) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int v = 0; v < 4; ++v) p.T[rr * F2K * FC + (8 * r + 4 * g + v) * FC + c] = uacc[4 * r + v];
            // only live rows count towards the parameter gradients
#pragma unroll
            for (int e = 0; e < 16; ++e) gw[e] += gwr[e];
            gb += gbr;
        }
        t = tn;
        gr = grn;
    }
    // block reduction of gWp (entry e of lane (c, g): input channel 8 (e / 4) + 4 g + e % 4,
    // output channel c) and gbp into this work-group's partial row, through the da tiles' LDS
    __syncthreads();
    float* red = &sda[0][0][0];
    static_assert(sizeof(sda) >= sizeof(float) * WAVES * 64 * 16, "reduction buffer");
    float* prow = p.part + (long)blockIdx.x * (FC * FC + FC);
#pragma unroll
    for (int e = 0; e < 16; ++e) red[(wv * 64 + lane) * 16 + e] = gw[e];
    __syncthreads();
    for (int i = threadIdx.x; i < 64 * 16; i += 64 * WAVES) {
        float sum = 0.f;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) sum += red[w * 64 * 16 + i];
        const int ln = i >> 4, e = i & 15;
        prow[(8 * (e >> 2) + 4 * (ln >> 5) + (e & 3)) * FC + (ln & 31)] = sum;
    }
    __syncthreads();
    red[wv * 64 + lane] = gb;
    __syncthreads();
    if (threadIdx.x < 32) {
        float sum = 0.f;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) sum += red[w * 64 + threadIdx.x] + red[w * 64 + 32 + threadIdx.x];
        prow[FC * FC + threadIdx.x] = sum;
    }
}

// Lift backward, one wave per row: da0 = da + Fx^T gT in the accumulator pixel
// layout (lane (channel c, group g), entry e: pixel 8 (e / 4) + 4 g + e % 4), then
// per-lane sums x_0 da0, x_1 da0 and da0 over the lane's pixels.
__global__ void __launch_bounds__(64 * WAVES) k_fno_lift_bwd(const float* __restrict__ da, const float* __restrict__ T,
                                                         const float* __restrict__ x, const bf16* __restrict__ FxT,
                                                         long rows, int W, float* __restrict__ part) {
    __shared__ float red[WAVES * 64 * 3];
    const int wv = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63, c = lane & 31, g = lane >> 5;
    float s0 = 0.f, s1 = 0.f, sb = 0.f;
    const long ngr = (rows + WAVES - 1) / WAVES;
    for (long gr = blockIdx.x; gr < ngr; gr += gridDim.x) {
        const long row = gr * WAVES + wv;
        if (row >= rows) continue;  // no barrier inside the loop
        bf16x8 tb[2];
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int v = 0; v < 8; ++v) tb[s][v] = (bf16)T[row * F2K * FC + (16 * s + 8 * g + v) * FC + c];
        for (int x0 = 0; x0 < W; x0 += 32) {
            const long pb = row * W + x0;
            floatx16 acc;
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[e] = da[(pb + 8 * (e >> 2) + 4 * g + (e & 3)) * FC + c];
#pragma unroll
            for (int s = 0; s < 2; ++s) acc = mfma(ld8(FxT + (long)(x0 + c) * F2K + 16 * s + 8 * g), tb[s], acc);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const float2 xi = reinterpret_cast<const float2*>(x)[pb + 8 * (e >> 2) + 4 * g + (e & 3)];
                s0 = __builtin_fmaf(xi.x, acc[e], s0);
                s1 = __builtin_fmaf(xi.y, acc[e], s1);
                sb += acc[e];
            }
        }
    }
    red[(wv * 64 + lane) * 3] = s0;
    red[(wv * 64 + lane) * 3 + 1] = s1;
    red[(wv * 64 + lane) * 3 + 2] = sb;
    __syncthreads();
    if (threadIdx.x < 3 * FC) {
        const int k = threadIdx.x / FC, ch = threadIdx.x % FC;  // k: 0, 1 -> gWl row k; 2 -> gbl
        float sum = 0.f;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) sum += red[(w * 64 + ch) * 3 + k] + red[(w * 64 + 32 + ch) * 3 + k];
        part[(long)blockIdx.x * 3 * FC + k * FC + ch] = sum;
    }
}

hipError_t launch_fno_lift_bwd(const float* da, const float* T, const float* x, const bf16* FxT, long rows, int W,
                               float* part, hipStream_t s) {
    if (W % 32 != 0 || rows <= 0 || (reinterpret_cast<uintptr_t>(FxT) & 15) || (reinterpret_cast<uintptr_t>(x) & 7))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fno_lift_bwd, dim3((unsigned)fno_layer_bwd_groups(rows)), dim3(64 * WAVES), 0, s, da, T, x, FxT,
                       rows, W, part);
    return hipGetLastError();
}

// out[v] += sum_r part[r nvals + v]: blockIdx.y takes every gridDim.y-th row
__global__ void k_sum_partials(const float* part, int nrows, int nvals, float* out) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvals) return;
    float sum = 0.f;
    for (int r = blockIdx.y; r < nrows; r += gridDim.y) sum += part[(long)r * nvals + v];
    atomicAdd(&out[v], sum);
}

int fno_layer_bwd_groups(long rows) {
    return (int)std::max(1L, std::min((rows + WAVES - 1) / WAVES, (long)kFnoBwdMaxGroups));
}
int fno_proj_bwd_groups(long pix, int P) {
    // P = 128: a tile per work-group (four waves on one tile); else a tile per wave
    const long per = P == 128 ? 1 : WAVES;
    return (int)std::max(1L, std::min((pix / 32 + per - 1) / per, (long)kFnoBwdMaxGroups));
}

hipError_t launch_fno_sum_partials(const float* part, int nrows, int nvals, float* out, hipStream_t s) {
    const int ys = std::min(nrows, 64);
    hipLaunchKernelGGL(k_sum_partials, dim3((unsigned)((nvals + 255) / 256), (unsigned)ys), dim3(256), 0, s, part, nrows,
                       nvals, out);
    return hipGetLastError();
}

hipError_t launch_fno_layer_bwd(const FnoLayerBwdArgs& a, hipStream_t s) {
    if (a.W % 32 != 0 || a.rows <= 0 || (reinterpret_cast<uintptr_t>(a.Wp) & 15) ||
        (reinterpret_cast<uintptr_t>(a.da) & 15) || (reinterpret_cast<uintptr_t>(a.z) & 15) ||
        (reinterpret_cast<uintptr_t>(a.aprev) & 15) ||
        (reinterpret_cast<uintptr_t>(a.FxT) & 15) || (reinterpret_cast<uintptr_t>(a.GxT) & 7))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fno_layer_bwd, dim3((unsigned)fno_layer_bwd_groups(a.rows)), dim3(64 * WAVES), 0, s, a);
    return hipGetLastError();
}

// Projection backward for P = 128 = 4 x 32 hidden units: the four waves of a
// work-group share each 32-pixel tile (a and dpred staged once in LDS) and wave w
// takes hidden block w, so a wave holds one block's accumulators (against four in
// k_fno_proj_bwd<4>, which runs at one wave per SIMD).  Per tile:
//   z  = a W1 + b1 (block w)          A = a rows from LDS, B = W1T rows (fixed per wave)
//   dz = (dpred W2^T) gelu'(z)        per accumulator entry; h = gelu(z)
//   gW1^T(block w) += dz^T a          A = dz from the accumulators, B = a^T from LDS
//   da_w = dz W1(block w)^T           A = dz rows through LDS, B = W1 rows (fixed)
//   da = sum over the four waves      through LDS, stored by the whole work-group
// gW1's block w, gb1 and gW2 of units 32 w + c are this wave's alone, so the
// partial row needs no reduction across waves.
__global__ void __launch_bounds__(64 * WAVES) k_fno_proj_bwd_split(FnoProjBwdArgs p) {
    static_assert(WAVES == 4, "one hidden block of 32 units per wave");
    constexpr int LD = FC + 8;
    __shared__ bf16 sa[32][LD];            // a tile [pixel][channel]
    __shared__ float sd[32][2];            // dpred tile, rounded to bf16
    __shared__ bf16 sdz[WAVES][32][LD];    // dz [pixel][unit] per wave
    __shared__ float sdp[WAVES][32][FC + 1];  // per-wave da partials [pixel][channel]
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, c = lane & 31, g = lane >> 5;
    const int P = p.P;  // 128
    const int T = wv;
    // per-wave constants: W1T rows of the block (B of z), W1 rows (B of da), b1, W2
    bf16x8 w1b[2], wb[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        w1b[s] = ld8(p.W1T + (long)(32 * T + c) * FC + 16 * s + 8 * g);
        wb[s] = ld8(p.W1 + (long)c * P + 32 * T + 16 * s + 8 * g);
    }
    const float bb = p.b1[32 * T + c];
    const float w2a = (float)p.W2[2 * (32 * T + c)], w2b = (float)p.W2[2 * (32 * T + c) + 1];
    floatx16 gw1 = zero16();
    float gw2a = 0.f, gw2b = 0.f, gb = 0.f;
    const long ntiles = p.pix / 32;
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long p0 = tile * 32;
        // stage a (2 KB: 128 threads x 16 B) and dpred (64 floats)
        if (threadIdx.x < 128) {
            const int px = threadIdx.x >> 2, ch = 8 * (threadIdx.x & 3);
            *reinterpret_cast<bf16x8*>(&sa[px][ch]) = ld8(p.a + (p0 + px) * FC + ch);
        } else if (threadIdx.x < 192) {
            const int i = threadIdx.x - 128;
            sd[i >> 1][i & 1] = (float)(bf16)p.dpred[2 * p0 + i];
        }
        __syncthreads();
        bf16x8 aop[2], at[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) aop[s] = *reinterpret_cast<const bf16x8*>(&sa[c][16 * s + 8 * g]);
        // a^T in accumulator pixel order: K entry 8 g + v of step q <-> pixel 16 q + 8 (v / 4) + 4 g + v % 4
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int v = 0; v < 8; ++v) at[q][v] = sa[16 * q + 8 * (v >> 2) + 4 * g + (v & 3)][c];
        floatx16 h;
#pragma unroll
        for (int e = 0; e < 16; ++e) h[e] = bb;
#pragma unroll
        for (int s = 0; s < 2; ++s) h = mfma(aop[s], w1b[s], h);
        bf16x8 dz[2];
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int pe = 8 * (e >> 2) + 4 * g + (e & 3);
            const float d0 = sd[pe][0], d1 = sd[pe][1];
            float gf, gd;
            fno_gelu_fd(h[e], gf, gd);
            const float hv = (float)(bf16)gf;
            const bf16 dzv = (bf16)((d0 * w2a + d1 * w2b) * gd);
            dz[e >> 3][e & 7] = dzv;
            gw2a += hv * d0;
            gw2b += hv * d1;
            gb += (float)dzv;
            sdz[wv][pe][c] = dzv;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) gw1 = mfma(dz[q], at[q], gw1);
        __syncthreads();
        floatx16 dp = zero16();
#pragma unroll
        for (int s = 0; s < 2; ++s) dp = mfma(*reinterpret_cast<const bf16x8*>(&sdz[wv][c][16 * s + 8 * g]), wb[s], dp);
#pragma unroll
        for (int e = 0; e < 16; ++e) sdp[wv][8 * (e >> 2) + 4 * g + (e & 3)][c] = dp[e];
        __syncthreads();
        // da = sum of the four partials: 1024 values, four per thread, stored as float4 runs
        {
            const int px = threadIdx.x >> 3, ch = 4 * (threadIdx.x & 7);
            float4 o;
            o.x = sdp[0][px][ch] + sdp[1][px][ch] + sdp[2][px][ch] + sdp[3][px][ch];
            o.y = sdp[0][px][ch + 1] + sdp[1][px][ch + 1] + sdp[2][px][ch + 1] + sdp[3][px][ch + 1];
            o.z = sdp[0][px][ch + 2] + sdp[1][px][ch + 2] + sdp[2][px][ch + 2] + sdp[3][px][ch + 2];
            o.w = sdp[0][px][ch + 3] + sdp[1][px][ch + 3] + sdp[2][px][ch + 3] + sdp[3][px][ch + 3];
            *reinterpret_cast<float4*>(p.da + (p0 + px) * FC + ch) = o;
        }
        __syncthreads();  // LDS reused by the next tile
    }
    // partial row [gW1 (32 x P) | gb1 (P) | gW2 (P x 2)]: block T of gW1 and units 32 T + c are this wave's
    float* prow = p.part + (long)blockIdx.x * (FC + 3) * P;
#pragma unroll
    for (int e = 0; e < 16; ++e) prow[(long)c * P + 32 * T + 8 * (e >> 2) + 4 * g + (e & 3)] = gw1[e];
    gw2a += __shfl_xor(gw2a, 32);
    gw2b += __shfl_xor(gw2b, 32);
    gb += __shfl_xor(gb, 32);
    if (g == 0) {
        prow[32 * P + 32 * T + c] = gb;
        prow[33 * P + 2 * (32 * T + c)] = gw2a;
        prow[33 * P + 2 * (32 * T + c) + 1] = gw2b;
    }
}

bool fno_proj_bwd_ok(int C, int P) { return C == FC && (P == 32 || P == 64 || P == 128); }

hipError_t launch_fno_proj_bwd(const FnoProjBwdArgs& a, hipStream_t s) {
    if (!fno_proj_bwd_ok(FC, a.P) || a.pix % 32 != 0 || a.pix <= 0) return hipErrorInvalidValue;
    if ((reinterpret_cast<uintptr_t>(a.a) & 15) || (reinterpret_cast<uintptr_t>(a.W1T) & 15) ||
        (reinterpret_cast<uintptr_t>(a.W1) & 15) || (reinterpret_cast<uintptr_t>(a.dpred) & 7) ||
        (reinterpret_cast<uintptr_t>(a.da) & 15))
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)fno_proj_bwd_groups(a.pix, a.P)), block(64 * WAVES);
    if (a.P == 32) hipLaunchKernelGGL(k_fno_proj_bwd<1>, grid, block, 0, s, a);
    else if (a.P == 64) hipLaunchKernelGGL(k_fno_proj_bwd<2>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(k_fno_proj_bwd_split, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_transpose_bf16(const float* in, bf16* out, int R, int Cc, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose_bf16, dim3((R * Cc + 255) / 256), dim3(256), 0, s, in, out, R, Cc);
    return hipGetLastError();
}

}  // namespace sgm
