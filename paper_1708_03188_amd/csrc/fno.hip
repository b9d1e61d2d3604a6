// FNO-style surrogate for Ginzburg-Landau states: inference, training
// (forward, backward, Adam) and the checked advance with FP64 fallback.
//
// Activations are channels-last [B][H][W][C] bfloat16; every contraction
// (truncated DFTs along x and y, per-mode complex channel mixing, pointwise
// channel layers) is a strided batched GEMM on the bf16 matrix cores with fp32
// accumulation; GELU, biases, the loss and the optimizer are elementwise
// kernels.  Parameters are kept in fp32 (master copy and Adam moments) and
// mirrored to bf16 for the GEMMs after every update.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "common.h"
#include "fno_fused.h"
#include "fno_gemm.h"

namespace sgm {

typedef __bf16 bf16;

__device__ __forceinline__ float gelu_f(float z) { return fno_gelu(z); }
__device__ __forceinline__ float gelu_df(float z) { return fno_gelu_d(z); }

// a[p, c] = x[p, 0] Wl[0, c] + x[p, 1] Wl[1, c] + bl[c]
__global__ void k_lift(const float* x, const float* Wl, const float* bl, bf16* a, long P, int C) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= P * C) return;
    long p = i / C;
    int c = (int)(i - p * C);
    a[i] = (bf16)(x[2 * p] * Wl[c] + x[2 * p + 1] * Wl[C + c] + bl[c]);
}

// z = s + bias; out = act ? gelu(z) : z; zsave (bf16) keeps z for the backward pass
__global__ void k_bias_act(const float* s, const float* bias, bf16* out, bf16* zsave, long n, int C, int act) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float z = s[i] + bias[i % C];
    if (zsave) zsave[i] = (bf16)z;
    out[i] = (bf16)(act ? gelu_f(z) : z);
}

// pred = x + out + b2
__global__ void k_residual(const float* x, const float* out, const float* b2, float* pred, long P) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= 2 * P) return;
    pred[i] = x[i] + out[i] + b2[i & 1];
}

// per-sample squared norms of (pred - tgt) and tgt
__global__ void k_loss_norms(const float* pred, const float* tgt, long per, double* nd, double* nt) {
    const int b = blockIdx.y;
    __shared__ double sd[256], st[256];
    double a = 0, c = 0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < per; i += (long)gridDim.x * blockDim.x) {
        double d = (double)pred[b * per + i] - (double)tgt[b * per + i];
        double t = tgt[b * per + i];
        a += d * d;
        c += t * t;
    }
    sd[threadIdx.x] = a;
    st[threadIdx.x] = c;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) { sd[threadIdx.x] += sd[threadIdx.x + s]; st[threadIdx.x] += st[threadIdx.x + s]; }
        __syncthreads();
    }
    if (threadIdx.x == 0) { atomicAdd(&nd[b], sd[0]); atomicAdd(&nt[b], st[0]); }
}

// dpred = (pred - tgt) / (|pred - tgt| |tgt|) / B ; per-sample relative L2 out
__global__ void k_loss_grad(const float* pred, const float* tgt, const double* nd, const double* nt, float* dpred,
                            long per, int B, float* rel) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < (long)B && rel) rel[i] = (float)(sqrt(nd[i]) / sqrt(nt[i]));
    if (i >= per * B || !dpred) return;
    int b = (int)(i / per);
    double f = 1.0 / (sqrt(nd[b]) * sqrt(nt[b]) * B);
    dpred[i] = (float)(((double)pred[i] - (double)tgt[i]) * f);
}

// dz = da * gelu'(z) (act) or da, as bf16 for the GEMMs and fp32 for bias gradients
__global__ void k_act_bwd(const float* da, const bf16* z, bf16* dz, long n, int act) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float g = da[i];
    if (act) g *= gelu_df((float)z[i]);
    dz[i] = (bf16)g;
}

// dz = da gelu'(z) (act) or da, four elements per thread (n a multiple of 4)
__global__ void k_act_bwd4(const float* da, const bf16* z, bf16* dz, long n4, int act) {
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n4) return;
    const float4 g4 = reinterpret_cast<const float4*>(da)[i];
    float g[4] = {g4.x, g4.y, g4.z, g4.w};
    typedef __bf16 bf16x4v __attribute__((ext_vector_type(4)));
    if (act) {
        const bf16x4v zz = reinterpret_cast<const bf16x4v*>(z)[i];
#pragma unroll
        for (int j = 0; j < 4; ++j) g[j] *= gelu_df((float)zz[j]);
    }
    bf16x4v o;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = (bf16)g[j];
    reinterpret_cast<bf16x4v*>(dz)[i] = o;
}

// The projection's hidden-layer gradient in one pass: dh = dpred W2^T (the two
// dpred channels rounded to bf16, as the product's operands are), then
// dhp = dh gelu'(hp) to bf16; eight hidden units per thread.
__global__ void k_proj_act_bwd(const float* dpred, const bf16* W2, const bf16* hpz, bf16* dhp, long pix, int P) {
    const int G8 = P / 8;
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= pix * G8) return;
    const long p = i / G8;
    const int j0 = (int)(i - p * G8) * 8;
    const float d0 = (float)(bf16)dpred[2 * p], d1 = (float)(bf16)dpred[2 * p + 1];
    typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
    const bf16x8v z = *reinterpret_cast<const bf16x8v*>(hpz + p * P + j0);
    bf16x8v o;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float w0 = (float)W2[2 * (j0 + j)], w1 = (float)W2[2 * (j0 + j) + 1];
        o[j] = (bf16)((d0 * w0 + d1 * w1) * gelu_df((float)z[j]));
    }
    *reinterpret_cast<bf16x8v*>(dhp + p * P + j0) = o;
}

// db[c] += sum_p g[p, c] with 8 consecutive columns per thread (C a multiple of
// 8): one 16-byte (bf16) or two (fp32) loads per row, so a wave reads whole
// rows; per-block partials reduced in LDS, one atomic add per column and block.
template <typename T>
__global__ void __launch_bounds__(256) k_colsum8(const T* g, float* db, long P, int C) {
    extern __shared__ float sh[];
    const int G8 = C / 8;                     // threads per row
    const int c8 = threadIdx.x % G8, r = threadIdx.x / G8, R = blockDim.x / G8;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (long p = blockIdx.x * (long)R + r; p < P; p += (long)gridDim.x * R) {
        const T* q = g + p * C + 8 * c8;
        if constexpr (sizeof(T) == 2) {
            typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
            const bf16x8v v = *reinterpret_cast<const bf16x8v*>(q);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] += (float)v[j];
        } else {
            const float4 u = reinterpret_cast<const float4*>(q)[0], w = reinterpret_cast<const float4*>(q)[1];
            acc[0] += u.x; acc[1] += u.y; acc[2] += u.z; acc[3] += u.w;
            acc[4] += w.x; acc[5] += w.y; acc[6] += w.z; acc[7] += w.w;
        }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) sh[threadIdx.x * 8 + j] = acc[j];
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        const int cg = c / 8, j = c % 8;
        float sum = 0.f;
        for (int q = 0; q < R; ++q) sum += sh[(q * G8 + cg) * 8 + j];
        atomicAdd(&db[c], sum);
    }
}

// db[c] += sum_p g[p, c]  (g bf16 or fp32), any C
template <typename T>
__global__ void k_colsum(const T* g, float* db, long P, int C) {
    extern __shared__ float sh[];
    const int c = threadIdx.x % C, r = threadIdx.x / C, R = blockDim.x / C;
    float acc = 0.f;
    for (long p = blockIdx.x * (long)R + r; p < P; p += (long)gridDim.x * R) acc += (float)g[p * C + c];
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (r == 0) {
        float s = 0.f;
        for (int q = 0; q < R; ++q) s += sh[q * C + c];
        atomicAdd(&db[c], s);
    }
}

// X[b][part][j][kx][c] -> Xm[(j, kx)][b][part][c]   (and back when inv)
// One thread per V consecutive channels (V = 16 bytes of elements when C is a
// multiple of that: 16-byte moves, else 1), index arithmetic in 32 bits (the
// host keeps the element count below 2^31).
template <typename T>
__global__ void k_perm_modes(const T* in, T* out, int B, int KY, int KX, int C, int inv) {
    constexpr unsigned VMAX = 16 / sizeof(T);
    const unsigned V = (unsigned)C % VMAX == 0 ? VMAX : 1u;
    const unsigned CV = (unsigned)C / V;
    const unsigned n = (unsigned)B * 2u * (unsigned)KY * (unsigned)KX * CV;
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // element index in the [b][part][j][kx][c] layout
    unsigned t = i;
    const unsigned cv = t % CV; t /= CV;
    const unsigned kx = t % (unsigned)KX; t /= (unsigned)KX;
    const unsigned j = t % (unsigned)KY; t /= (unsigned)KY;
    const unsigned part = t & 1u, b = t >> 1;
    const long a = (long)i * V;
    const long o = ((long)((j * (unsigned)KX + kx) * (unsigned)B + b) * 2 + part) * C + cv * V;
    if (V == VMAX) {
        if (inv) *reinterpret_cast<uint4*>(out + a) = *reinterpret_cast<const uint4*>(in + o);
        else *reinterpret_cast<uint4*>(out + o) = *reinterpret_cast<const uint4*>(in + a);
    } else {
        if (inv) out[a] = in[o];
        else out[o] = in[a];
    }
}

// Rreal[m] (2C x 2C) = [[Rr, Ri], [-Ri, Rr]] as bf16, m = (j, kx)
__global__ void k_build_rreal(const float* Rr, const float* Ri, bf16* Rreal, int nm, int C) {
    long n = (long)nm * 4 * C * C;
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int C2 = 2 * C;
    int col = (int)(i % C2);
    int row = (int)((i / C2) % C2);
    long m = i / (C2 * C2);
    int pi = row / C, c = row % C, po = col / C, o = col % C;
    long src = (m * C + c) * C + o;
    float v;
    if (pi == po) v = Rr[src];
    else v = pi == 0 ? Ri[src] : -Ri[src];
    Rreal[i] = (bf16)v;
}

// The same for every layer in one launch (blockIdx.y = layer; layer l's Rr at
// Rr0 + l lstride, its Ri right after it), eight consecutive outputs of one row per
// thread: two 16-byte loads and one 16-byte store (C a multiple of 8).
__global__ void k_build_rreal8(const float* Rr0, long lstride, bf16* Rreal0, int nm, int C) {
    const int C2 = 2 * C;
    const long n8 = (long)nm * C2 * C2 / 8;
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n8) return;
    const float* Rr = Rr0 + blockIdx.y * lstride;
    const float* Ri = Rr + (long)nm * C * C;
    const long e0 = 8 * i;
    const int col0 = (int)(e0 % C2);
    const int row = (int)((e0 / C2) % C2);
    const long m = e0 / ((long)C2 * C2);
    const int pi = row / C, c = row % C, po = col0 / C, o0 = col0 % C;
    const float* srcp = (pi == po ? Rr : Ri) + (m * C + c) * C + o0;
    const float sg = (pi == po || pi == 0) ? 1.f : -1.f;
    const float4 u = reinterpret_cast<const float4*>(srcp)[0], w = reinterpret_cast<const float4*>(srcp)[1];
    typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
    bf16x8v o;
    o[0] = (bf16)(sg * u.x); o[1] = (bf16)(sg * u.y); o[2] = (bf16)(sg * u.z); o[3] = (bf16)(sg * u.w);
    o[4] = (bf16)(sg * w.x); o[5] = (bf16)(sg * w.y); o[6] = (bf16)(sg * w.z); o[7] = (bf16)(sg * w.w);
    reinterpret_cast<bf16x8v*>(Rreal0 + (long)blockIdx.y * nm * C2 * C2)[i] = o;
}

// dRr = G[(re,c),(re,o)] + G[(im,c),(im,o)], dRi = G[(re,c),(im,o)] - G[(im,c),(re,o)]
__global__ void k_fold_rgrad(const float* G, float* dRr, float* dRi, int nm, int C) {
    long n = (long)nm * C * C;
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int o = (int)(i % C);
    int c = (int)((i / C) % C);
    long m = i / ((long)C * C);
    int C2 = 2 * C;
    const float* g = G + m * C2 * C2;
    dRr[i] += g[c * C2 + o] + g[(C + c) * C2 + C + o];
    dRi[i] += g[c * C2 + C + o] - g[(C + c) * C2 + o];
}

__global__ void k_f32_to_bf16(const float* in, bf16* out, long n) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) out[i] = (bf16)in[i];
}

__global__ void k_fill(float* p, float v, long n) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_d(double* p, long n) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void k_adam(float* w, const float* g, float* m, float* v, long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// complex128 packed N x N states [x][y] -> fp32 [b][y?]... channels-last [b][x][y][2]
// Reflections of the square grid: pixel (i, j) of the reflected field takes
// pixel s(i, j) of the field, s = (transpose?) o (flip rows?, flip columns?):
// (i1, j1) = (fx ? H-1-i : i, fy ? W-1-j : j), s = t ? (j1, i1) : (i1, j1)
// (t needs H = W).  bits of op: 1 flip rows, 2 flip columns, 4 transpose.
__device__ __forceinline__ long refl_src(long p, int H, int W, int op) {
    const long HW = (long)H * W;
    const long b = p / HW;
    const int r = (int)(p - b * HW);
    const int i = r / W, j = r - i * W;
    const int i1 = (op & 1) ? H - 1 - i : i, j1 = (op & 2) ? W - 1 - j : j;
    return b * HW + ((op & 4) ? (long)j1 * W + i1 : (long)i1 * W + j1);
}

// out = R in (gather), over npix pixels of 2 channels
__global__ void k_reflect(const float2* in, float2* out, long npix, int H, int W, int op) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < npix) out[p] = in[refl_src(p, H, W, op)];
}

// acc (=|+=) w R^{-1} p: the reflected-frame pixel p goes back to s(p)
__global__ void k_unreflect_acc(const float2* pr, float2* acc, long npix, int H, int W, int op, float w, int first) {
    const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    const long q = refl_src(p, H, W, op);
    const float2 v = pr[p];
    float2 a = first ? make_float2(0.f, 0.f) : acc[q];
    a.x += w * v.x;
    a.y += w * v.y;
    acc[q] = a;
}

__global__ void k_c128_to_x(const double2* u, float* x, long n) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2 v = u[i];
    x[2 * i] = (float)v.x;
    x[2 * i + 1] = (float)v.y;
}
__global__ void k_x_to_c128(const float* x, double2* u, long n) {
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    u[i] = make_double2((double)x[2 * i], (double)x[2 * i + 1]);
}

static inline unsigned nblk(long n, int t = 256) { return (unsigned)((n + t - 1) / t); }
// threads of k_perm_modes<T> over B x 2 x 2K x K x C values
template <typename T>
static inline long perm_threads(long B, long K, long C) {
    const long v = 16 / (long)sizeof(T);
    return B * 4 * K * K * C / (C % v == 0 ? v : 1);
}

}  // namespace sgm

using namespace sgm;

// host bf16 (round to nearest even)
static uint16_t to_bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

struct sgm_fno_s {
    sgm_fno_desc d;
    int C, K, P, nl, H, W, Bmax, KY, KX, NM;
    long npar = 0;
    // parameter offsets (floats) in the flat vector
    long oWl, obl, oW1, ob1, oW2, ob2;
    std::vector<long> oRr, oRi, oWp, obp;
    float* par = nullptr;   // fp32 master
    float* grad = nullptr;
    float* mom1 = nullptr;
    float* mom2 = nullptr;
    long step = 0;
    bool mirrors_ok = false;
    // bf16 mirrors
    bf16 *Wp16 = nullptr, *W1_16 = nullptr, *W2_16 = nullptr, *Rreal = nullptr, *W1T16 = nullptr;
    bf16* W2P = nullptr;  // W2 as MFMA A operands of the fused projection (P % 32 == 0)
    // DFT matrices (bf16)
    bf16 *Fx = nullptr, *Fy = nullptr, *Gy = nullptr, *Gx = nullptr;
    bf16 *FxT = nullptr, *GxT = nullptr;  // transposes of Fx and Gx (fused layer backward)
    float* part = nullptr;  // per-work-group partial parameter gradients of the fused backward kernels
    // activations / scratch (sized for Bmax)
    bf16* acts = nullptr;   // (nl + 1) x [B H W C]
    bf16* zsv = nullptr;    // nl x [B H W C]
    bf16* hbuf = nullptr;   // [B H W P] gelu output
    bf16* hpz = nullptr;    // [B H W P] pre-activation
    float* s32 = nullptr;   // [B H W max(C, P)] fp32 GEMM output / gradient accumulator
    float* da32 = nullptr;  // [B H W C]
    bf16* d16 = nullptr;    // [B H W max(C, P)] bf16 gradient
    float* T = nullptr;     // [B H 2K C]
    float* X = nullptr;     // [B 4K K C]
    float* Xm = nullptr;    // spectral, mode-major, per layer saved: nl x [NM B 2C]
    float* Ym = nullptr;    // [NM B 2C]
    float* Yt = nullptr;    // [B 4K K C]
    float* Rg = nullptr;    // [NM 2C 2C] gradient of Rreal
    float* outb = nullptr;  // [B H W 2]
    float* predb = nullptr; // [B H W 2]
    double* norms = nullptr;// 2 x Bmax
    float* rel = nullptr;   // Bmax
    void* all = nullptr;
    // advance_checked workspace (grown on demand)
    size_t adv_bytes = 0;   // bytes allocated at adv
    void* adv = nullptr;
    // second stream for the FP64 check path, overlapped with inference
    hipStream_t adv_stream = nullptr;
    hipEvent_t adv_ev[2] = {nullptr, nullptr};
    // inference averaged over ens reflections of the periodic square (1 = the plain
    // network); ens_x / ens_p hold one member's input and prediction (Bmax x H x W x 2)
    int ens = 1;
    float* ens_x = nullptr;
    float* ens_p = nullptr;
};

static long fno_act_elems(const sgm_fno_s* f) { return (long)f->Bmax * f->H * f->W * f->C; }

extern "C" sgm_status sgm_fno_destroy(sgm_fno f) {
    clear_error();
    if (!f) return SGM_OK;
    hipFree(f->all);
    hipFree(f->adv);
    hipFree(f->ens_x);
    hipFree(f->ens_p);
    for (hipEvent_t e : f->adv_ev)
        if (e) hipEventDestroy(e);
    if (f->adv_stream) hipStreamDestroy(f->adv_stream);
    delete f;
    return SGM_OK;
}

extern "C" sgm_status sgm_fno_create(const sgm_fno_desc* desc, uint64_t seed, sgm_fno* out) {
    clear_error();
    TraceRange trace_range("sgm_fno_create");
    SGM_CHECK_ARG(desc && out, "null argument");
    *out = nullptr;
    const sgm_fno_desc& d = *desc;
    SGM_CHECK_ARG(d.H >= 4 && d.W >= 4 && d.width >= 1 && d.modes >= 1 && d.layers >= 1 && d.hidden >= 1 &&
                      d.max_batch >= 1,
                  "invalid FNO sizes");
    SGM_CHECK_ARG(2 * d.modes <= d.H && 2 * d.modes <= d.W, "modes must satisfy 2*modes <= H and 2*modes <= W");
    SGM_CHECK_ARG((long)d.max_batch * 4 * d.modes * d.modes * d.width < (1L << 31),
                  "max_batch * 4 * modes^2 * width must stay below 2^31");
    sgm_fno_s* f = new (std::nothrow) sgm_fno_s();
    if (!f) return SGM_ERR_OOM;
    f->d = d;
    f->C = d.width; f->K = d.modes; f->P = d.hidden; f->nl = d.layers; f->H = d.H; f->W = d.W; f->Bmax = d.max_batch;
    f->KY = 2 * d.modes; f->KX = d.modes; f->NM = f->KY * f->KX;
    const int C = f->C, P = f->P, nl = f->nl, NM = f->NM;
    long o = 0;
    f->oWl = o; o += 2L * C;
    f->obl = o; o += C;
    for (int l = 0; l < nl; ++l) {
        f->oRr.push_back(o); o += (long)NM * C * C;
        f->oRi.push_back(o); o += (long)NM * C * C;
        f->oWp.push_back(o); o += (long)C * C;
        f->obp.push_back(o); o += C;
    }
    f->oW1 = o; o += (long)C * P;
    f->ob1 = o; o += P;
    f->oW2 = o; o += 2L * P;
    f->ob2 = o; o += 2;
    f->npar = o;
    // device allocation plan
    const long HW = (long)d.H * d.W, B = d.max_batch;
    const long act = B * HW * C;
    // the hidden projection layer and the wide GEMM scratch are only used outside the
    // fused row kernels (other widths, mode counts or hidden sizes)
    const bool all_fused = fno_fused_ok(C, f->K, d.W, P) && fno_proj_bwd_ok(C, P);
    const long wide = all_fused ? 0 : B * HW * std::max(C, P), hid = all_fused ? 0 : B * HW * P;
    struct Slot { void** p; size_t bytes; };
    std::vector<Slot> slots = {
        {(void**)&f->par, 4 * (size_t)f->npar}, {(void**)&f->grad, 4 * (size_t)f->npar},
        {(void**)&f->mom1, 4 * (size_t)f->npar}, {(void**)&f->mom2, 4 * (size_t)f->npar},
        {(void**)&f->Wp16, 2 * (size_t)nl * C * C}, {(void**)&f->W1_16, 2 * (size_t)C * P},
        {(void**)&f->W2_16, 2 * (size_t)2 * P}, {(void**)&f->Rreal, 2 * (size_t)nl * NM * 4 * C * C},
        {(void**)&f->W1T16, 2 * (size_t)C * P}, {(void**)&f->W2P, 2 * (size_t)(P / 16 + 1) * 512},
        {(void**)&f->Fx, 2 * (size_t)2 * f->K * d.W}, {(void**)&f->Fy, 2 * (size_t)4 * f->K * 2 * d.H},
        {(void**)&f->Gy, 2 * (size_t)2 * d.H * 4 * f->K}, {(void**)&f->Gx, 2 * (size_t)d.W * 2 * f->K},
        {(void**)&f->FxT, 2 * (size_t)2 * f->K * d.W}, {(void**)&f->GxT, 2 * (size_t)d.W * 2 * f->K},
        {(void**)&f->part, 4 * (size_t)kFnoBwdMaxGroups * std::max((long)C * C + C, (long)(C + 3) * P)},
        {(void**)&f->acts, 2 * (size_t)(nl + 1) * act}, {(void**)&f->zsv, 2 * (size_t)nl * act},
        {(void**)&f->hbuf, 2 * (size_t)hid}, {(void**)&f->hpz, 2 * (size_t)hid},
        {(void**)&f->s32, 4 * (size_t)wide}, {(void**)&f->da32, 4 * (size_t)act}, {(void**)&f->d16, 2 * (size_t)wide},
        {(void**)&f->T, 4 * (size_t)B * d.H * 2 * f->K * C}, {(void**)&f->X, 4 * (size_t)B * 4 * f->K * f->K * C},
        {(void**)&f->Xm, 4 * (size_t)nl * NM * B * 2 * C}, {(void**)&f->Ym, 4 * (size_t)NM * B * 2 * C},
        {(void**)&f->Yt, 4 * (size_t)B * 4 * f->K * f->K * C}, {(void**)&f->Rg, 4 * (size_t)NM * 4 * C * C},
        {(void**)&f->outb, 4 * (size_t)B * HW * 2}, {(void**)&f->predb, 4 * (size_t)B * HW * 2},
        {(void**)&f->norms, 8 * (size_t)2 * B}, {(void**)&f->rel, 4 * (size_t)B},
    };
    size_t total = 0;
    for (auto& s : slots) total += (s.bytes + 255) & ~size_t(255);
    if (hipMalloc(&f->all, total) != hipSuccess) {
        set_error("hipMalloc of %zu bytes for the FNO failed", total);
        delete f;
        return SGM_ERR_OOM;
    }
    char* base = static_cast<char*>(f->all);
    size_t off = 0;
    for (auto& s : slots) { *s.p = base + off; off += (s.bytes + 255) & ~size_t(255); }
    // DFT matrices on the host (long double phases, exact index reduction)
    const long double twopi = 6.283185307179586476925286766559L;
    const int K = f->K, H = d.H, W = d.W;
    std::vector<uint16_t> Fx(2 * K * W), Fy(4 * K * 2 * H), Gy(2 * H * 4 * K), Gx(W * 2 * K);
    auto kyv = [&](int j) { return j < K ? j : H - 2 * K + j; };
    for (int kx = 0; kx < K; ++kx)
        for (int x = 0; x < W; ++x) {
            long double a = twopi * (long double)((long)kx * x % W) / W;
            Fx[kx * W + x] = to_bf16_bits((float)(cosl(a) / W));
            Fx[(K + kx) * W + x] = to_bf16_bits((float)(-sinl(a) / W));
            const float w = kx == 0 ? 1.f : 2.f;
            Gx[x * 2 * K + kx] = to_bf16_bits((float)(w * cosl(a)));
            Gx[x * 2 * K + K + kx] = to_bf16_bits((float)(-w * sinl(a)));
        }
    for (int j = 0; j < 2 * K; ++j)
        for (int y = 0; y < H; ++y) {
            long double a = twopi * (long double)((long)kyv(j) * y % H) / H;
            const float fr = (float)(cosl(a) / H), fi = (float)(-sinl(a) / H);  // exp(-i a) / H
            // Fy_real[(part_out, j)][(y, part_in)]
            const int ncol = 2 * H;
            Fy[(0 * 2 * K + j) * ncol + 2 * y + 0] = to_bf16_bits(fr);
            Fy[(0 * 2 * K + j) * ncol + 2 * y + 1] = to_bf16_bits(-fi);
            Fy[(1 * 2 * K + j) * ncol + 2 * y + 0] = to_bf16_bits(fi);
            Fy[(1 * 2 * K + j) * ncol + 2 * y + 1] = to_bf16_bits(fr);
            // Gy_real[(y, part_out)][(part_in, j)] with exp(+i a)
            const float gr = (float)cosl(a), gi = (float)sinl(a);
            const int gcol = 4 * K;
            Gy[(2 * y + 0) * gcol + 0 * 2 * K + j] = to_bf16_bits(gr);
            Gy[(2 * y + 0) * gcol + 1 * 2 * K + j] = to_bf16_bits(-gi);
            Gy[(2 * y + 1) * gcol + 0 * 2 * K + j] = to_bf16_bits(gi);
            Gy[(2 * y + 1) * gcol + 1 * 2 * K + j] = to_bf16_bits(gr);
        }
    hipMemcpy(f->Fx, Fx.data(), Fx.size() * 2, hipMemcpyHostToDevice);
    hipMemcpy(f->Fy, Fy.data(), Fy.size() * 2, hipMemcpyHostToDevice);
    hipMemcpy(f->Gy, Gy.data(), Gy.size() * 2, hipMemcpyHostToDevice);
    hipMemcpy(f->Gx, Gx.data(), Gx.size() * 2, hipMemcpyHostToDevice);
    {
        std::vector<uint16_t> FxT(Fx.size()), GxT(Gx.size());
        for (int k = 0; k < 2 * K; ++k)
            for (int x = 0; x < W; ++x) {
                FxT[(long)x * 2 * K + k] = Fx[(long)k * W + x];
                GxT[(long)k * W + x] = Gx[(long)x * 2 * K + k];
            }
        hipMemcpy(f->FxT, FxT.data(), FxT.size() * 2, hipMemcpyHostToDevice);
        hipMemcpy(f->GxT, GxT.data(), GxT.size() * 2, hipMemcpyHostToDevice);
    }
    // seeded initial parameters (normal / uniform scales as in common FNO practice)
    std::vector<float> hp(f->npar, 0.f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> nd(0.f, 1.f);
    std::uniform_real_distribution<float> ud(0.f, 1.f);
    for (long i = 0; i < 2L * C; ++i) hp[f->oWl + i] = nd(rng) / std::sqrt(2.f);
    for (int l = 0; l < nl; ++l) {
        const float sc = 1.f / (float)(C * C);
        for (long i = 0; i < (long)NM * C * C; ++i) { hp[f->oRr[l] + i] = sc * ud(rng); hp[f->oRi[l] + i] = sc * ud(rng); }
        for (long i = 0; i < (long)C * C; ++i) hp[f->oWp[l] + i] = nd(rng) / std::sqrt((float)C);
    }
    for (long i = 0; i < (long)C * P; ++i) hp[f->oW1 + i] = nd(rng) / std::sqrt((float)C);
    for (long i = 0; i < 2L * P; ++i) hp[f->oW2 + i] = 0.1f * nd(rng) / std::sqrt((float)P);
    hipMemcpy(f->par, hp.data(), 4 * f->npar, hipMemcpyHostToDevice);
    hipMemset(f->mom1, 0, 4 * f->npar);
    hipMemset(f->mom2, 0, 4 * f->npar);
    *out = f;
    return SGM_OK;
}

static sgm_status refresh_mirrors(sgm_fno f, hipStream_t s) {
    if (f->mirrors_ok) return SGM_OK;
    const int C = f->C, P = f->P;
    // every layer's parameters sit at a fixed stride: Rr, Ri, Wp, bp
    const long lstride = f->nl > 1 ? f->oRr[1] - f->oRr[0] : 0;
    const bool vec = C % 8 == 0 && f->oRi[0] == f->oRr[0] + (long)f->NM * C * C && (f->oRr[0] & 3) == 0 &&
                     (lstride & 3) == 0;
    if (vec) {
        hipLaunchKernelGGL(k_build_rreal8, dim3(nblk((long)f->NM * 4 * C * C / 8), f->nl), dim3(256), 0, s,
                           (const float*)(f->par + f->oRr[0]), lstride, f->Rreal, f->NM, C);
    }
    for (int l = 0; l < f->nl; ++l) {
        hipLaunchKernelGGL(k_f32_to_bf16, dim3(nblk((long)C * C)), dim3(256), 0, s, f->par + f->oWp[l],
                           f->Wp16 + (long)l * C * C, (long)C * C);
        if (!vec)
            hipLaunchKernelGGL(k_build_rreal, dim3(nblk((long)f->NM * 4 * C * C)), dim3(256), 0, s,
                               (const float*)(f->par + f->oRr[l]), (const float*)(f->par + f->oRi[l]),
                               f->Rreal + (long)l * f->NM * 4 * C * C, f->NM, C);
    }
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(nblk((long)C * P)), dim3(256), 0, s, f->par + f->oW1, f->W1_16, (long)C * P);
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(nblk(2L * P)), dim3(256), 0, s, f->par + f->oW2, f->W2_16, 2L * P);
    SGM_HIP_TRY(hipGetLastError());
    SGM_HIP_TRY(launch_transpose_bf16(f->par + f->oW1, f->W1T16, C, P, s));
    if (P % 32 == 0) SGM_HIP_TRY(launch_fno_w2_operands(f->W2_16, f->W2P, P, s));
    f->mirrors_ok = true;
    return SGM_OK;
}

extern "C" sgm_status sgm_fno_num_params(sgm_fno f, int64_t* n) {
    clear_error();
    SGM_CHECK_ARG(f && n, "null argument");
    *n = f->npar;
    return SGM_OK;
}

extern "C" sgm_status sgm_fno_set_params(sgm_fno f, const float* host) {
    clear_error();
    SGM_CHECK_ARG(f && host, "null argument");
    SGM_HIP_TRY(hipMemcpy(f->par, host, 4 * f->npar, hipMemcpyHostToDevice));
    SGM_HIP_TRY(hipMemset(f->mom1, 0, 4 * f->npar));
    SGM_HIP_TRY(hipMemset(f->mom2, 0, 4 * f->npar));
    f->step = 0;
    f->mirrors_ok = false;
    return SGM_OK;
}

extern "C" sgm_status sgm_fno_get_params(sgm_fno f, float* host) {
    clear_error();
    SGM_CHECK_ARG(f && host, "null argument");
    SGM_HIP_TRY(hipMemcpy(host, f->par, 4 * f->npar, hipMemcpyDeviceToHost));
    return SGM_OK;
}

// row-major helper: GEMM with A (M x K, lda), B (K x N, ldb), C (M x N, ldc)
static GemmDesc G(int batch, int M, int N, int K, const void* A, long sAb, long sAm, long sAk, int af32, const void* B,
                  long sBb, long sBk, long sBn, int bf32, float* Cp, long sCb, long sCm, long sCn, float beta = 0.f,
                  int splitk = 1) {
    GemmDesc g{};
    g.M = M; g.N = N; g.K = K; g.batch = batch;
    g.A = A; g.sAb = sAb; g.sAm = sAm; g.sAk = sAk; g.a_f32 = af32;
    g.B = B; g.sBb = sBb; g.sBk = sBk; g.sBn = sBn; g.b_f32 = bf32;
    g.C = Cp; g.sCb = sCb; g.sCm = sCm; g.sCn = sCn;
    g.alpha = 1.f; g.beta = beta; g.splitk = splitk;
    return g;
}

static int splits_for(long K) {
    // one split per 1024 rows of the reduction: enough work-groups to cover the
    // device when the output is one 64 x 64 tile
    long s = K / 1024;
    if (s < 1) s = 1;
    if (s > 1024) s = 1024;
    return (int)s;
}

// Forward pass for `batch` samples.  Training (pred_out null) keeps the
// activations for backward and leaves the prediction in predb; inference
// writes pred_out.  Width 32 with 16 x-modes runs the fused row kernels
// (lift + x-DFT; inverse x-DFT + pointwise + bias + GELU + next x-DFT;
// projection), other shapes the GEMM sequence.
// Training with the fused row kernels keeps no hidden projection layer: the last
// layer kernel also projects to the prediction, and the backward recomputes the
// hidden pre-activation from the last layer's output.
static bool proj_fused(sgm_fno f) { return fno_fused_ok(f->C, f->K, f->W, f->P) && fno_proj_bwd_ok(f->C, f->P); }

static sgm_status fno_forward(sgm_fno f, const float* x, int B, hipStream_t s, float* pred_out = nullptr) {
    const int C = f->C, P = f->P, H = f->H, W = f->W, K = f->K, NM = f->NM;
    const long HW = (long)H * W, pix = (long)B * HW, act = (long)f->Bmax * HW * C;
    const bool fused = fno_fused_ok(C, K, W, P);
    const bool projf = proj_fused(f);
    if (fused) {
        SGM_HIP_TRY(launch_fno_lift_dft(x, f->par + f->oWl, f->par + f->obl, f->Fx, f->acts, reinterpret_cast<bf16*>(f->T),
                                        (long)B * H, W, s));
    } else {
        hipLaunchKernelGGL(k_lift, dim3(nblk(pix * C)), dim3(256), 0, s, x, f->par + f->oWl, f->par + f->obl, f->acts,
                           pix, C);
        SGM_HIP_TRY(hipGetLastError());
    }
    for (int l = 0; l < f->nl; ++l) {
        const bf16* a = f->acts + l * act;
        bf16* an = f->acts + (l + 1) * act;
        // G1: T[(b,y)] (2K x C) = Fx (2K x W) a[(b,y)] (W x C)
        if (!fused)
            SGM_HIP_TRY(gemm(G(B * H, 2 * K, C, W, f->Fx, 0, W, 1, 0, a, (long)W * C, C, 1, 0, f->T, 2L * K * C, C, 1), s));
        // G2: X[b] (4K x K C) = Fy_real (4K x 2H) T[b] (2H x K C).  The fused kernels keep T and U
        // in bf16: both consumers round them to bf16 anyway, so the values are the same.
        // X, Xm, Ym and Yt are bf16 too: each is only a GEMM operand downstream (or moved by the
        // permutation), and the GEMM rounds its operands to bf16.
        {
            GemmDesc g2 = G(B, 4 * K, K * C, 2 * H, f->Fy, 0, 2L * H, 1, 0, f->T, 2L * H * K * C, (long)K * C, 1,
                            fused ? 0 : 1, f->X, 4L * K * K * C, (long)K * C, 1);
            g2.c_bf16 = 1;
            SGM_HIP_TRY(gemm(g2, s));
        }
        bf16* Xm = reinterpret_cast<bf16*>(f->Xm) + (long)l * NM * f->Bmax * 2 * C;
        hipLaunchKernelGGL(k_perm_modes<bf16>, dim3(nblk(perm_threads<bf16>(B, K, C))), dim3(256), 0, s,
                           reinterpret_cast<const bf16*>(f->X), Xm, B, 2 * K, K, C, 0);
        // G3: Ym[m] (B x 2C) = Xm[m] (B x 2C) Rreal[m] (2C x 2C)
        {
            GemmDesc g3 = G(NM, B, 2 * C, 2 * C, Xm, (long)B * 2 * C, 2 * C, 1, 0, f->Rreal + (long)l * NM * 4 * C * C,
                            4L * C * C, 2 * C, 1, 0, f->Ym, (long)B * 2 * C, 2 * C, 1);
            g3.c_bf16 = 1;
            SGM_HIP_TRY(gemm(g3, s));
        }
        hipLaunchKernelGGL(k_perm_modes<bf16>, dim3(nblk(perm_threads<bf16>(B, K, C))), dim3(256), 0, s,
                           reinterpret_cast<const bf16*>(f->Ym), reinterpret_cast<bf16*>(f->Yt), B, 2 * K, K, C, 1);
        // G4: U[b] (2H x K C) = Gy_real (2H x 4K) Yt[b] (4K x K C)   (U reuses T)
        {
            GemmDesc g4 = G(B, 2 * H, K * C, 4 * K, f->Gy, 0, 4L * K, 1, 0, f->Yt, 4L * K * K * C, (long)K * C, 1, 0, f->T,
                            2L * H * K * C, (long)K * C, 1);
            g4.c_bf16 = fused ? 1 : 0;
            SGM_HIP_TRY(gemm(g4, s));
        }
        if (fused) {
            FnoLayerArgs la{};
            la.a = a; la.U = reinterpret_cast<const bf16*>(f->T); la.Tn = reinterpret_cast<bf16*>(f->T);
            la.Gx = f->Gx; la.Fx = f->Fx;
            la.Wp = f->Wp16 + (long)l * C * C; la.bp = f->par + f->obp[l];
            la.a_out = an; la.zsave = pred_out ? nullptr : f->zsv + l * act;
            la.rows = (long)B * H; la.W = W; la.act = l < f->nl - 1 ? 1 : 0;
            la.W1T = f->W1T16; la.b1 = f->par + f->ob1; la.W2 = f->W2_16; la.W2P = f->W2P; la.b2 = f->par + f->ob2;
            la.x = x; la.pred = pred_out ? pred_out : f->predb; la.P = P;
            const int mode = l < f->nl - 1 ? 0 : (pred_out ? 2 : (projf ? 3 : 1));
            SGM_HIP_TRY(launch_fno_layer(la, mode, s));
            continue;
        }
        // G5: s[(b,y)] (W x C) = Gx (W x 2K) U[(b,y)] (2K x C)
        SGM_HIP_TRY(gemm(G(B * H, W, C, 2 * K, f->Gx, 0, 2L * K, 1, 0, f->T, 2L * K * C, C, 1, 1, f->s32, (long)W * C, C, 1),
                         s));
        // G6: s += a Wp
        SGM_HIP_TRY(gemm(G(1, (int)pix, C, C, a, 0, C, 1, 0, f->Wp16 + (long)l * C * C, 0, C, 1, 0, f->s32, 0, C, 1, 1.f),
                         s));
        hipLaunchKernelGGL(k_bias_act, dim3(nblk(pix * C)), dim3(256), 0, s, (const float*)f->s32,
                           (const float*)(f->par + f->obp[l]), an, f->zsv + l * act, pix * C, C, l < f->nl - 1 ? 1 : 0);
        SGM_HIP_TRY(hipGetLastError());
    }
    if (fused && (pred_out || projf)) return SGM_OK;  // projection done in the last layer kernel
    // projection
    const bf16* a = f->acts + f->nl * act;
    SGM_HIP_TRY(gemm(G(1, (int)pix, P, C, a, 0, C, 1, 0, f->W1_16, 0, P, 1, 0, f->s32, 0, P, 1), s));
    hipLaunchKernelGGL(k_bias_act, dim3(nblk(pix * P)), dim3(256), 0, s, (const float*)f->s32,
                       (const float*)(f->par + f->ob1), f->hbuf, f->hpz, pix * P, P, 1);
    SGM_HIP_TRY(gemm(G(1, (int)pix, 2, P, f->hbuf, 0, P, 1, 0, f->W2_16, 0, 2, 1, 0, f->outb, 0, 2, 1), s));
    hipLaunchKernelGGL(k_residual, dim3(nblk(2 * pix)), dim3(256), 0, s, x, (const float*)f->outb,
                       (const float*)(f->par + f->ob2), f->predb, pix);
    SGM_HIP_TRY(hipGetLastError());
    return SGM_OK;
}

static sgm_status fno_loss(sgm_fno f, const float* tgt, int B, bool grad, hipStream_t s) {
    const long per = (long)f->H * f->W * 2;
    hipLaunchKernelGGL(k_fill_d, dim3(nblk(2L * B)), dim3(256), 0, s, f->norms, 2L * B);
    hipLaunchKernelGGL(k_loss_norms, dim3(64, B), dim3(256), 0, s, (const float*)f->predb, tgt, per, f->norms,
                       f->norms + B);
    hipLaunchKernelGGL(k_loss_grad, dim3(nblk(std::max(per * B, (long)B))), dim3(256), 0, s, (const float*)f->predb, tgt,
                       (const double*)f->norms, (const double*)(f->norms + B), grad ? f->outb : nullptr, per, B, f->rel);
    SGM_HIP_TRY(hipGetLastError());
    return SGM_OK;
}

static hipError_t colsum_bf16(const bf16* g, float* db, long P, int C, hipStream_t s) {
    if (C % 8 == 0 && C <= 256 * 8 && (reinterpret_cast<uintptr_t>(g) & 15) == 0) {
        const int G8 = C / 8, R = std::max(1, 256 / G8);
        const long blocks = std::min(2048L, std::max(1L, (P + R - 1) / R));
        hipLaunchKernelGGL(k_colsum8<bf16>, dim3((unsigned)blocks), dim3(R * G8), (size_t)R * G8 * 8 * 4, s, g, db, P,
                           C);
        return hipGetLastError();
    }
    int R = std::max(1, 256 / C);
    hipLaunchKernelGGL(k_colsum<bf16>, dim3(512), dim3(R * C), (size_t)R * C * 4, s, g, db, P, C);
    return hipGetLastError();
}
static hipError_t colsum_f32(const float* g, float* db, long P, int C, hipStream_t s) {
    if (C % 8 == 0 && C <= 256 * 8 && (reinterpret_cast<uintptr_t>(g) & 31) == 0) {
        const int G8 = C / 8, R = std::max(1, 256 / G8);
        const long blocks = std::min(2048L, std::max(1L, (P + R - 1) / R));
        hipLaunchKernelGGL(k_colsum8<float>, dim3((unsigned)blocks), dim3(R * G8), (size_t)R * G8 * 8 * 4, s, g, db, P,
                           C);
        return hipGetLastError();
    }
    int R = std::max(1, 256 / C);
    hipLaunchKernelGGL(k_colsum<float>, dim3(512), dim3(R * C), (size_t)R * C * 4, s, g, db, P, C);
    return hipGetLastError();
}

// Backward pass; dpred (fp32 [B H W 2]) is in f->outb.  Gradients -> f->grad.
static sgm_status fno_backward_layers(sgm_fno f, const float* x, int B, hipStream_t s);

// Adjoint of the y-DFT, the per-mode mixing and the inverse y-DFT of layer l:
// gU (T, fp32 rows) -> gT (T), with the mixing weights' gradient folded into
// the grad buffer.
static sgm_status spectral_adjoint(sgm_fno f, int l, int B, hipStream_t s) {
    const int C = f->C, H = f->H, K = f->K, NM = f->NM;
    // gYt[b] (4K x K C) = Gy_real^T (4K x 2H) gU[b] (2H x K C); the reduction (2H) split four
    // ways into the zeroed output: at small batches the product alone is too few work-groups
    const int skY = (B * ((4 * K + 63) / 64) * ((K * C + 63) / 64) < 512 && 2 * H >= 128) ? 4 : 1;
    if (skY > 1) {
        hipLaunchKernelGGL(k_fill, dim3(nblk((long)B * 4 * K * K * C)), dim3(256), 0, s, f->Yt, 0.f,
                           (long)B * 4 * K * K * C);
        SGM_HIP_TRY(hipGetLastError());
    }
    SGM_HIP_TRY(gemm(G(B, 4 * K, K * C, 2 * H, f->Gy, 0, 1, 4L * K, 0, f->T, 2L * H * K * C, (long)K * C, 1, 1, f->Yt,
                       4L * K * K * C, (long)K * C, 1, 0.f, skY), s));
    hipLaunchKernelGGL(k_perm_modes<float>, dim3(nblk(perm_threads<float>(B, K, C))), dim3(256), 0, s,
                       (const float*)f->Yt, f->Ym, B, 2 * K, K, C, 0);
    // dRreal[m] (2C x 2C) = Xm[m]^T (2C x B) gYm[m] (B x 2C)   (Xm saved in bf16 by the forward pass)
    const bf16* Xm = reinterpret_cast<const bf16*>(f->Xm) + (long)l * NM * f->Bmax * 2 * C;
    SGM_HIP_TRY(gemm(G(NM, 2 * C, 2 * C, B, Xm, (long)B * 2 * C, 1, 2 * C, 0, f->Ym, (long)B * 2 * C, 2 * C, 1, 1, f->Rg,
                       4L * C * C, 2 * C, 1), s));
    hipLaunchKernelGGL(k_fold_rgrad, dim3(nblk((long)NM * C * C)), dim3(256), 0, s, (const float*)f->Rg,
                       f->grad + f->oRr[l], f->grad + f->oRi[l], NM, C);
    // gXm[m] (B x 2C) = gYm[m] (B x 2C) Rreal[m]^T   (into the X buffer, mode-major)
    SGM_HIP_TRY(gemm(G(NM, B, 2 * C, 2 * C, f->Ym, (long)B * 2 * C, 2 * C, 1, 1, f->Rreal + (long)l * NM * 4 * C * C,
                       4L * C * C, 1, 2 * C, 0, f->X, (long)B * 2 * C, 2 * C, 1), s));
    hipLaunchKernelGGL(k_perm_modes<float>, dim3(nblk(perm_threads<float>(B, K, C))), dim3(256), 0, s,
                       (const float*)f->X, f->Yt, B, 2 * K, K, C, 1);
    // gT[b] (2H x K C) = Fy_real^T (2H x 4K) gX[b] (4K x K C)
    SGM_HIP_TRY(gemm(G(B, 2 * H, K * C, 4 * K, f->Fy, 0, 1, 2L * H, 0, f->Yt, 4L * K * K * C, (long)K * C, 1, 1, f->T,
                       2L * H * K * C, (long)K * C, 1), s));
    return SGM_OK;
}


static sgm_status fno_backward(sgm_fno f, const float* x, int B, hipStream_t s) {
    const int C = f->C, P = f->P, H = f->H, W = f->W, K = f->K, NM = f->NM;
    const long HW = (long)H * W, pix = (long)B * HW, act = (long)f->Bmax * HW * C;
    hipLaunchKernelGGL(k_fill, dim3(nblk(f->npar)), dim3(256), 0, s, f->grad, 0.f, f->npar);
    const float* dpred = f->outb;
    const int sk = splits_for(pix);
    if (proj_fused(f)) {
        FnoProjBwdArgs pa{};
        pa.a = f->acts + f->nl * act; pa.dpred = dpred;
        pa.W1T = f->W1T16; pa.W1 = f->W1_16; pa.b1 = f->par + f->ob1; pa.W2 = f->W2_16;
        pa.da = f->da32; pa.part = f->part;
        pa.pix = pix; pa.P = P;
        SGM_HIP_TRY(launch_fno_proj_bwd(pa, s));
        // the partial rows are [gW1 | gb1 | gW2], the parameters' order in the gradient buffer
        SGM_HIP_TRY(launch_fno_sum_partials(f->part, fno_proj_bwd_groups(pix, P), (C + 3) * P, f->grad + f->oW1, s));
        SGM_HIP_TRY(colsum_f32(dpred, f->grad + f->ob2, pix, 2, s));
        return fno_backward_layers(f, x, B, s);
    }
    // W2, b2
    SGM_HIP_TRY(gemm(G(1, P, 2, (int)pix, f->hbuf, 0, 1, P, 0, dpred, 0, 2, 1, 1, f->grad + f->oW2, 0, 2, 1, 0.f, sk), s));
    SGM_HIP_TRY(colsum_f32(dpred, f->grad + f->ob2, pix, 2, s));
    // dh = dpred W2^T ; dhp = dh gelu'(hp)
    if (P % 8 == 0) {
        hipLaunchKernelGGL(k_proj_act_bwd, dim3(nblk(pix * (P / 8))), dim3(256), 0, s, dpred, (const bf16*)f->W2_16,
                           (const bf16*)f->hpz, f->d16, pix, P);
    } else {
        SGM_HIP_TRY(gemm(G(1, (int)pix, P, 2, dpred, 0, 2, 1, 1, f->W2_16, 0, 1, 2, 0, f->s32, 0, P, 1), s));
        hipLaunchKernelGGL(k_act_bwd, dim3(nblk(pix * P)), dim3(256), 0, s, (const float*)f->s32, (const bf16*)f->hpz,
                           f->d16, pix * P, 1);
    }
    SGM_HIP_TRY(hipGetLastError());
    const bf16* alast = f->acts + f->nl * act;
    SGM_HIP_TRY(gemm(G(1, C, P, (int)pix, alast, 0, 1, C, 0, f->d16, 0, P, 1, 0, f->grad + f->oW1, 0, P, 1, 0.f, sk), s));
    SGM_HIP_TRY(colsum_bf16(f->d16, f->grad + f->ob1, pix, P, s));
    // da = dhp W1^T
    SGM_HIP_TRY(gemm(G(1, (int)pix, C, P, f->d16, 0, P, 1, 0, f->W1_16, 0, 1, P, 0, f->da32, 0, C, 1), s));
    return fno_backward_layers(f, x, B, s);
}

// Backward through the layers and the lift, from da (fp32, last layer's output
// gradient) in f->da32.
static sgm_status fno_backward_layers(sgm_fno f, const float* x, int B, hipStream_t s) {
    const int C = f->C, H = f->H, W = f->W, K = f->K, NM = f->NM;
    const long HW = (long)H * W, pix = (long)B * HW, act = (long)f->Bmax * HW * C;
    const int sk = splits_for(pix);
    const bool fused = fno_fused_ok(C, K, W, f->P);
    for (int l = f->nl - 1; l >= 0; --l) {
        const bf16* aprev = f->acts + l * act;
        if (fused) {
            // dz, gWp, gbp, da = dz Wp^T and gU = Gx^T dz in one pass over the rows; the
            // layer above's Fx^T gT is added to da on the way in
            FnoLayerBwdArgs lb{};
            lb.da = f->da32; lb.T = f->T; lb.z = f->zsv + l * act; lb.aprev = aprev;
            lb.Wp = f->Wp16 + (long)l * C * C; lb.FxT = f->FxT; lb.GxT = f->GxT;
            lb.part = f->part;
            lb.rows = (long)B * H; lb.W = W; lb.act = l < f->nl - 1 ? 1 : 0; lb.addT = l < f->nl - 1 ? 1 : 0;
            SGM_HIP_TRY(launch_fno_layer_bwd(lb, s));
            // partial rows [gWp | gbp], the parameters' order in the gradient buffer
            SGM_HIP_TRY(launch_fno_sum_partials(f->part, fno_layer_bwd_groups(lb.rows), C * C + C, f->grad + f->oWp[l], s));
            if (const sgm_status st = spectral_adjoint(f, l, B, s)) return st;
            continue;
        }
        // dz = da gelu'(z)
        if ((pix * C) % 4 == 0 && act % 4 == 0)  // whole 4-element groups, 8-byte aligned z rows
            hipLaunchKernelGGL(k_act_bwd4, dim3(nblk(pix * C / 4)), dim3(256), 0, s, (const float*)f->da32,
                               (const bf16*)(f->zsv + l * act), f->d16, pix * C / 4, l < f->nl - 1 ? 1 : 0);
        else
            hipLaunchKernelGGL(k_act_bwd, dim3(nblk(pix * C)), dim3(256), 0, s, (const float*)f->da32,
                               (const bf16*)(f->zsv + l * act), f->d16, pix * C, l < f->nl - 1 ? 1 : 0);
        const bf16* dz = f->d16;
        SGM_HIP_TRY(gemm(G(1, C, C, (int)pix, aprev, 0, 1, C, 0, dz, 0, C, 1, 0, f->grad + f->oWp[l], 0, C, 1, 0.f, sk),
                         s));
        SGM_HIP_TRY(colsum_bf16(dz, f->grad + f->obp[l], pix, C, s));
        // da_new = dz Wp^T  (into da32, overwriting: dz already holds the old da)
        SGM_HIP_TRY(gemm(G(1, (int)pix, C, C, dz, 0, C, 1, 0, f->Wp16 + (long)l * C * C, 0, 1, C, 0, f->da32, 0, C, 1), s));
        // spectral adjoint: gU[(b,y)] (2K x C) = Gx^T (2K x W) dz[(b,y)] (W x C)
        SGM_HIP_TRY(gemm(G(B * H, 2 * K, C, W, f->Gx, 0, 1, 2L * K, 0, dz, (long)W * C, C, 1, 0, f->T, 2L * K * C, C, 1), s));
        if (const sgm_status st = spectral_adjoint(f, l, B, s)) return st;
        // da += Fx^T (W x 2K) gT[(b,y)] (2K x C)
        SGM_HIP_TRY(gemm(G(B * H, W, C, 2 * K, f->Fx, 0, 1, W, 0, f->T, 2L * K * C, C, 1, 1, f->da32, (long)W * C, C, 1,
                           1.f), s));
    }
    if (fused) {
        // layer 0's Fx^T gT is added on the fly; partial rows [gWl | gbl] in the parameters' order
        SGM_HIP_TRY(launch_fno_lift_bwd(f->da32, f->T, x, f->FxT, (long)B * H, W, f->part, s));
        SGM_HIP_TRY(launch_fno_sum_partials(f->part, fno_layer_bwd_groups((long)B * H), 3 * C, f->grad + f->oWl, s));
        return SGM_OK;
    }
    // lift: Wl = x^T da (2 x C), bl = sum da
    SGM_HIP_TRY(gemm(G(1, 2, C, (int)pix, x, 0, 1, 2, 1, f->da32, 0, C, 1, 1, f->grad + f->oWl, 0, C, 1, 0.f, sk), s));
    SGM_HIP_TRY(colsum_f32(f->da32, f->grad + f->obl, pix, C, s));
    return SGM_OK;
}

// One pass of the network over batch states (mirrors current).
static sgm_status infer_once(sgm_fno f, const float* x, float* pred, int batch, hipStream_t s) {
    if (fno_fused_ok(f->C, f->K, f->W, f->P)) return fno_forward(f, x, batch, s, pred);
    sgm_status r = fno_forward(f, x, batch, s);
    if (r != SGM_OK) return r;
    SGM_HIP_TRY(hipMemcpyAsync(pred, f->predb, 4L * batch * f->H * f->W * 2, hipMemcpyDeviceToDevice, s));
    return SGM_OK;
}

// Reflections averaged by an ensemble of 2 (identity, transpose), 4 (the row and
// column flips) or 8 (all of them) members.
static int ens_op(int ens, int m) {
    if (ens == 2) return m ? 4 : 0;
    return m;  // 4: ops 0..3 (flips), 8: ops 0..7
}

extern "C" sgm_status sgm_fno_infer(sgm_fno f, const float* x, float* pred, int batch, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_fno_infer");
    SGM_CHECK_ARG(f && x && pred, "null argument");
    SGM_CHECK_ARG(batch >= 1 && batch <= f->Bmax, "batch must be in 1..%d", f->Bmax);
    hipStream_t s = static_cast<hipStream_t>(stream);
    sgm_status r = refresh_mirrors(f, s);
    if (r != SGM_OK) return r;
    if (f->ens == 1) return infer_once(f, x, pred, batch, s);
    SGM_CHECK_ARG(x != pred, "pred must not alias x for an ensemble of %d members", f->ens);
    const long npix = (long)batch * f->H * f->W;
    for (int m = 0; m < f->ens; ++m) {
        const int op = ens_op(f->ens, m);
        const float* xin = x;
        if (op) {
            hipLaunchKernelGGL(k_reflect, dim3(nblk(npix)), dim3(256), 0, s, reinterpret_cast<const float2*>(x),
                               reinterpret_cast<float2*>(f->ens_x), npix, f->H, f->W, op);
            SGM_HIP_TRY(hipGetLastError());
            xin = f->ens_x;
        }
        if ((r = infer_once(f, xin, f->ens_p, batch, s)) != SGM_OK) return r;
        hipLaunchKernelGGL(k_unreflect_acc, dim3(nblk(npix)), dim3(256), 0, s, reinterpret_cast<const float2*>(f->ens_p),
                           reinterpret_cast<float2*>(pred), npix, f->H, f->W, op, 1.0f / (float)f->ens, m == 0 ? 1 : 0);
        SGM_HIP_TRY(hipGetLastError());
    }
    return SGM_OK;
}

extern "C" sgm_status sgm_fno_set_ensemble(sgm_fno f, int members) {
    clear_error();
    SGM_CHECK_ARG(f, "null network");
    SGM_CHECK_ARG(members == 1 || members == 2 || members == 4 || members == 8,
                  "members must be 1, 2, 4 or 8 (got %d)", members);
    SGM_CHECK_ARG(members == 1 || members == 4 || f->H == f->W,
                  "an ensemble with transposes (2 or 8 members) needs a square grid (H = %d, W = %d)", f->H, f->W);
    if (members > 1 && !f->ens_x) {
        const size_t bytes = (size_t)f->Bmax * f->H * f->W * 2 * sizeof(float);
        if (hipMalloc(&f->ens_x, bytes) != hipSuccess || hipMalloc(&f->ens_p, bytes) != hipSuccess) {
            hipFree(f->ens_x);
            f->ens_x = nullptr;
            f->ens_p = nullptr;
            set_error("hipMalloc ensemble buffers (%zu bytes each) failed", bytes);
            return SGM_ERR_OOM;
        }
    }
    f->ens = members;
    return SGM_OK;
}

extern "C" sgm_status sgm_fno_grads(sgm_fno f, const float* x, const float* target, int batch, float* grads_host,
                                    float* loss_host, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_fno_grads");
    SGM_CHECK_ARG(f && x && target, "null argument");
    SGM_CHECK_ARG(batch >= 1 && batch <= f->Bmax, "batch must be in 1..%d", f->Bmax);
    hipStream_t s = static_cast<hipStream_t>(stream);
    sgm_status r;
    if ((r = refresh_mirrors(f, s)) != SGM_OK) return r;
    if ((r = fno_forward(f, x, batch, s)) != SGM_OK) return r;
    if ((r = fno_loss(f, target, batch, true, s)) != SGM_OK) return r;
    if ((r = fno_backward(f, x, batch, s)) != SGM_OK) return r;
    if (grads_host) SGM_HIP_TRY(hipMemcpyAsync(grads_host, f->grad, 4 * f->npar, hipMemcpyDeviceToHost, s));
    if (loss_host) {
        std::vector<float> rel(batch);
        SGM_HIP_TRY(hipMemcpyAsync(rel.data(), f->rel, 4L * batch, hipMemcpyDeviceToHost, s));
        SGM_HIP_TRY(hipStreamSynchronize(s));
        double m = 0;
        for (float v : rel) m += v;
        *loss_host = (float)(m / batch);
    } else {
        SGM_HIP_TRY(hipStreamSynchronize(s));
    }
    return SGM_OK;
}

extern "C" sgm_status sgm_fno_train_step(sgm_fno f, const float* x, const float* target, int batch, float lr,
                                         float* loss_host, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_fno_train_step");
    SGM_CHECK_ARG(f && x && target, "null argument");
    SGM_CHECK_ARG(batch >= 1 && batch <= f->Bmax, "batch must be in 1..%d", f->Bmax);
    SGM_CHECK_ARG(lr > 0 && std::isfinite(lr), "lr must be positive");
    hipStream_t s = static_cast<hipStream_t>(stream);
    sgm_status r;
    if ((r = refresh_mirrors(f, s)) != SGM_OK) return r;
    if ((r = fno_forward(f, x, batch, s)) != SGM_OK) return r;
    if ((r = fno_loss(f, target, batch, true, s)) != SGM_OK) return r;
    if ((r = fno_backward(f, x, batch, s)) != SGM_OK) return r;
    ++f->step;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)f->step), c2 = 1.f - std::pow(b2, (float)f->step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(f->npar)), dim3(256), 0, s, f->par, (const float*)f->grad, f->mom1, f->mom2,
                       f->npar, lr, b1, b2, 1e-8f, c1, c2);
    SGM_HIP_TRY(hipGetLastError());
    f->mirrors_ok = false;
    if (loss_host) {
        std::vector<float> rel(batch);
        SGM_HIP_TRY(hipMemcpyAsync(rel.data(), f->rel, 4L * batch, hipMemcpyDeviceToHost, s));
        SGM_HIP_TRY(hipStreamSynchronize(s));
        double m = 0;
        for (float v : rel) m += v;
        *loss_host = (float)(m / batch);
    }
    return SGM_OK;
}

extern "C" sgm_status sgm_fno_rel_l2(sgm_fno f, const float* pred, const float* target, int batch, float* rel_dev,
                                     void* stream) {
    clear_error();
    SGM_CHECK_ARG(f && pred && target && rel_dev, "null argument");
    SGM_CHECK_ARG(batch >= 1 && batch <= f->Bmax, "batch must be in 1..%d", f->Bmax);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long per = (long)f->H * f->W * 2;
    hipLaunchKernelGGL(k_fill_d, dim3(nblk(2L * batch)), dim3(256), 0, s, f->norms, 2L * batch);
    hipLaunchKernelGGL(k_loss_norms, dim3(64, batch), dim3(256), 0, s, pred, target, per, f->norms, f->norms + batch);
    hipLaunchKernelGGL(k_loss_grad, dim3(nblk(batch)), dim3(256), 0, s, pred, target, (const double*)f->norms,
                       (const double*)(f->norms + batch), (float*)nullptr, per, batch, rel_dev);
    SGM_HIP_TRY(hipGetLastError());
    return SGM_OK;
}

extern "C" sgm_status sgm_fno_save(sgm_fno f, const char* path) {
    clear_error();
    SGM_CHECK_ARG(f && path, "null argument");
    std::vector<float> buf(3 * f->npar);
    SGM_HIP_TRY(hipMemcpy(buf.data(), f->par, 4 * f->npar, hipMemcpyDeviceToHost));
    SGM_HIP_TRY(hipMemcpy(buf.data() + f->npar, f->mom1, 4 * f->npar, hipMemcpyDeviceToHost));
    SGM_HIP_TRY(hipMemcpy(buf.data() + 2 * f->npar, f->mom2, 4 * f->npar, hipMemcpyDeviceToHost));
    FILE* fp = std::fopen(path, "wb");
    SGM_CHECK_ARG(fp, "cannot open %s", path);
    const char magic[8] = {'S', 'G', 'M', 'F', 'N', 'O', '1', 0};
    int64_t hdr[9] = {f->H, f->W, f->C, f->K, f->nl, f->P, f->npar, f->step, 0};
    bool ok = std::fwrite(magic, 1, 8, fp) == 8 && std::fwrite(hdr, 8, 9, fp) == 9 &&
              std::fwrite(buf.data(), 4, buf.size(), fp) == buf.size();
    std::fclose(fp);
    SGM_CHECK_ARG(ok, "short write to %s", path);
    return SGM_OK;
}

extern "C" sgm_status sgm_fno_load(sgm_fno f, const char* path) {
    clear_error();
    SGM_CHECK_ARG(f && path, "null argument");
    FILE* fp = std::fopen(path, "rb");
    SGM_CHECK_ARG(fp, "cannot open %s", path);
    char magic[8];
    int64_t hdr[9];
    bool ok = std::fread(magic, 1, 8, fp) == 8 && std::memcmp(magic, "SGMFNO1", 7) == 0 && std::fread(hdr, 8, 9, fp) == 9;
    ok = ok && hdr[0] == f->H && hdr[1] == f->W && hdr[2] == f->C && hdr[3] == f->K && hdr[4] == f->nl &&
         hdr[5] == f->P && hdr[6] == f->npar;
    std::vector<float> buf(3 * f->npar);
    ok = ok && std::fread(buf.data(), 4, buf.size(), fp) == buf.size();
    std::fclose(fp);
    SGM_CHECK_ARG(ok, "%s is not a checkpoint of this architecture", path);
    SGM_HIP_TRY(hipMemcpy(f->par, buf.data(), 4 * f->npar, hipMemcpyHostToDevice));
    SGM_HIP_TRY(hipMemcpy(f->mom1, buf.data() + f->npar, 4 * f->npar, hipMemcpyHostToDevice));
    SGM_HIP_TRY(hipMemcpy(f->mom2, buf.data() + 2 * f->npar, 4 * f->npar, hipMemcpyHostToDevice));
    f->step = hdr[7];
    f->mirrors_ok = false;
    return SGM_OK;
}

// packed complex128 GL states <-> fp32 channels-last input
extern "C" sgm_status sgm_fno_pack(const void* u_c128, float* x, int64_t n, void* stream) {
    clear_error();
    SGM_CHECK_ARG(u_c128 && x && n >= 0, "invalid argument");
    hipLaunchKernelGGL(k_c128_to_x, dim3(nblk(n)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       static_cast<const double2*>(u_c128), x, (long)n);
    SGM_HIP_TRY(hipGetLastError());
    return SGM_OK;
}

extern "C" sgm_status sgm_fno_unpack(const float* x, void* u_c128, int64_t n, void* stream) {
    clear_error();
    SGM_CHECK_ARG(u_c128 && x && n >= 0, "invalid argument");
    hipLaunchKernelGGL(k_x_to_c128, dim3(nblk(n)), dim3(256), 0, static_cast<hipStream_t>(stream), x,
                       static_cast<double2*>(u_c128), (long)n);
    SGM_HIP_TRY(hipGetLastError());
    return SGM_OK;
}

// Bytes of the advance_checked workspace for B states and NC checked states of HW
// points: phys c128 [B HW], x and pred fp32 [B HW 2]; chk and chkp c128 [NC HW],
// xs and ps fp32 [NC HW 2]; rel fp32 [NC] (each part a multiple of 256 bytes).
static size_t adv_workspace_bytes(long B, long NC, long HW) {
    auto up = [](size_t n) { return (n + 255) & ~(size_t)255; };
    return up((size_t)B * HW * 16) + 2 * up((size_t)B * HW * 8) + 2 * up((size_t)NC * HW * 16) +
           2 * up((size_t)NC * HW * 8) + up((size_t)NC * 4);
}

extern "C" sgm_status sgm_fno_advance_checked(sgm_fno f, sgm_gl gl, sgm_gl gl_check, void* u_hat, int nsur,
                                              int steps_per, double tol, double max_fail_frac, uint64_t seed,
                                              sgm_fno_stats* stats, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_fno_advance_checked");
    SGM_CHECK_ARG(f && gl && gl_check && u_hat, "null argument");
    SGM_CHECK_ARG(nsur >= 0 && steps_per >= 1 && tol > 0, "invalid nsur / steps_per / tol");
    SGM_CHECK_ARG(max_fail_frac >= 0.0 && max_fail_frac <= 1.0, "max_fail_frac must be in [0, 1] (got %g)",
                  max_fail_frac);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long HW = (long)f->H * f->W;
    // query the packed layout of both batches
    auto layout = [&](sgm_gl g, std::vector<int64_t>& o) -> sgm_status {
        int n = 0;
        sgm_status r = sgm_gl_count(g, &n);
        if (r != SGM_OK) return r;
        o.assign((size_t)n + 1, 0);
        return sgm_gl_offsets(g, o.data());
    };
    std::vector<int64_t> om, oc;
    sgm_status r;
    if ((r = layout(gl, om)) != SGM_OK) return r;
    if ((r = layout(gl_check, oc)) != SGM_OK) return r;
    const int B = (int)om.size() - 1, NC = (int)oc.size() - 1;
    for (int i = 0; i < B; ++i)
        SGM_CHECK_ARG(om[i + 1] - om[i] == HW, "problem %d of gl is not %d x %d", i, f->H, f->W);
    for (int i = 0; i < NC; ++i)
        SGM_CHECK_ARG(oc[i + 1] - oc[i] == HW, "problem %d of gl_check is not %d x %d", i, f->H, f->W);
    SGM_CHECK_ARG(NC >= 1 && NC <= B, "gl_check must hold between 1 and B problems");
    const size_t need = adv_workspace_bytes(B, NC, HW);
    if (f->adv_bytes < need) {
        // the previous workspace may still be in use by queued work of an earlier call
        if (f->adv) SGM_HIP_TRY(hipDeviceSynchronize());
        hipFree(f->adv);
        f->adv = nullptr;
        f->adv_bytes = 0;
        SGM_HIP_TRY(hipMalloc(&f->adv, need));
        f->adv_bytes = need;
    }
    if (!f->adv_stream) {
        SGM_HIP_TRY(hipStreamCreateWithFlags(&f->adv_stream, hipStreamNonBlocking));
        SGM_HIP_TRY(hipEventCreateWithFlags(&f->adv_ev[0], hipEventDisableTiming));
        SGM_HIP_TRY(hipEventCreateWithFlags(&f->adv_ev[1], hipEventDisableTiming));
    }
    hipStream_t s2 = f->adv_stream;
    char* w = static_cast<char*>(f->adv);
    auto take = [&w](size_t n) {
        char* p = w;
        w += (n + 255) & ~(size_t)255;
        return p;
    };
    double2* phys = reinterpret_cast<double2*>(take((size_t)B * HW * 16));
    float* x = reinterpret_cast<float*>(take((size_t)B * HW * 8));
    float* pred = reinterpret_cast<float*>(take((size_t)B * HW * 8));
    double2* chk = reinterpret_cast<double2*>(take((size_t)NC * HW * 16));
    double2* chkp = reinterpret_cast<double2*>(take((size_t)NC * HW * 16));
    float* xs = reinterpret_cast<float*>(take((size_t)NC * HW * 8));
    float* ps = reinterpret_cast<float*>(take((size_t)NC * HW * 8));
    float* reld = reinterpret_cast<float*>(take((size_t)NC * 4));
    double2* uh = static_cast<double2*>(u_hat);
    std::mt19937_64 rng(seed);
    double sum_rel = 0;
    int nchk_total = 0, nfb_total = 0, nbatch_total = 0;
    long nrep_total = 0;
    float maxrel = 0.f;
    const int stride = B / NC;
    for (int it = 0; it < nsur; ++it) {
        const int offs = (int)(rng() % (uint64_t)stride);
        std::vector<int> idx(NC);
        for (int k = 0; k < NC; ++k) idx[k] = offs + k * stride;
        // FP64 solver on the checked subset, on the second stream once the state is ready
        SGM_HIP_TRY(hipEventRecord(f->adv_ev[0], s));
        SGM_HIP_TRY(hipStreamWaitEvent(s2, f->adv_ev[0], 0));
        for (int k = 0; k < NC; ++k)
            SGM_HIP_TRY(hipMemcpyAsync(chk + (long)k * HW, uh + (long)idx[k] * HW, HW * 16, hipMemcpyDeviceToDevice, s2));
        if ((r = sgm_gl_step(gl_check, chk, steps_per, s2)) != SGM_OK) return r;
        if ((r = sgm_gl_backward(gl_check, chk, chkp, s2)) != SGM_OK) return r;
        if ((r = sgm_fno_pack(chkp, xs, (int64_t)NC * HW, s2)) != SGM_OK) return r;
        SGM_HIP_TRY(hipEventRecord(f->adv_ev[1], s2));
        // surrogate prediction for every sample, meanwhile on the caller's stream
        if ((r = sgm_gl_backward(gl, uh, phys, s)) != SGM_OK) return r;
        if ((r = sgm_fno_pack(phys, x, (int64_t)B * HW, s)) != SGM_OK) return r;
        for (int b0 = 0; b0 < B; b0 += f->Bmax) {
            const int nb = std::min(f->Bmax, B - b0);
            if ((r = sgm_fno_infer(f, x + (long)b0 * HW * 2, pred + (long)b0 * HW * 2, nb, s)) != SGM_OK) return r;
        }
        SGM_HIP_TRY(hipStreamWaitEvent(s, f->adv_ev[1], 0));
        for (int k = 0; k < NC; ++k)
            SGM_HIP_TRY(hipMemcpyAsync(ps + (long)k * HW * 2, pred + (long)idx[k] * HW * 2, HW * 8,
                                       hipMemcpyDeviceToDevice, s));
        for (int b0 = 0; b0 < NC; b0 += f->Bmax) {
            const int nb = std::min(f->Bmax, NC - b0);
            if ((r = sgm_fno_rel_l2(f, ps + (long)b0 * HW * 2, xs + (long)b0 * HW * 2, nb, reld + b0, s)) != SGM_OK)
                return r;
        }
        std::vector<float> rel(NC);
        SGM_HIP_TRY(hipMemcpyAsync(rel.data(), reld, 4L * NC, hipMemcpyDeviceToHost, s));
        SGM_HIP_TRY(hipStreamSynchronize(s));
        int nfail = 0;
        for (int k = 0; k < NC; ++k) {
            sum_rel += rel[k];
            maxrel = std::max(maxrel, rel[k]);
            if (!(rel[k] <= tol)) ++nfail;
        }
        nfb_total += nfail;
        nchk_total += NC;
        if ((double)nfail > max_fail_frac * NC) {
            // too many checked states failed to trust the unchecked ones: u_hat still
            // holds the macro-step's starting state, so the FP64 solver advances all of it
            if ((r = sgm_gl_step(gl, uh, steps_per, s)) != SGM_OK) return r;
            ++nbatch_total;
            nrep_total += B;
            continue;
        }
        // new state: transform the surrogate's fields, then overwrite failed checks with the solver
        if ((r = sgm_fno_unpack(pred, phys, (int64_t)B * HW, s)) != SGM_OK) return r;
        if ((r = sgm_gl_forward(gl, phys, uh, s)) != SGM_OK) return r;
        for (int k = 0; k < NC; ++k) {
            if (!(rel[k] <= tol)) {
                ++nrep_total;
                SGM_HIP_TRY(hipMemcpyAsync(uh + (long)idx[k] * HW, chk + (long)k * HW, HW * 16, hipMemcpyDeviceToDevice,
                                           s));
            }
        }
    }
    if (stats) {
        const int prev = stats->n_checked;
        stats->n_checked += nchk_total;
        stats->n_fallback += nfb_total;
        stats->n_batch_fallback += nbatch_total;
        stats->n_replaced += nrep_total;
        stats->max_rel_l2 = std::max(stats->max_rel_l2, maxrel);
        stats->mean_rel_l2 = stats->n_checked ? (float)((stats->mean_rel_l2 * (double)prev + sum_rel) / stats->n_checked)
                                              : 0.f;
    }
    return SGM_OK;
}
