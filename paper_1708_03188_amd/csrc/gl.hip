// Complex Ginzburg-Landau: ragged batches of doubly periodic problems.
//
// A right-hand-side evaluation is a pass over rows and a pass over columns of
// the zero-padded M = floor(3N/2) grid of every problem of the batch:
//   A  rows    : zero-pad each spectral row (ky) to M, inverse FFT
//   B  columns : zero-pad each column (kx) to M, inverse FFT, form
//                (1 + i c)|u|^2 u on the fine grid, forward FFT (1/M), truncate
//   C  rows    : forward FFT (1/M), truncate to the N retained ky, and apply the
//                Runge-Kutta stage update (or write the right-hand side).
// Within a time step pass C of stage s also performs pass A of stage s+1: the
// new stage input of a row is already in the thread's registers at exactly the
// padded positions the inverse transform needs.  Each launch covers every
// problem through a work list of (problem, first line) items and dispatches on
// the problem's padded length: a register-FFT specialisation for the compiled
// lengths, the generic LDS FFT otherwise.  Launch geometry (radix schedule,
// lines per block, exchange buffers) and grid mode (persistent grid-stride or
// one block per item) are chosen by measurement at batch creation.
#include <algorithm>
#include <map>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "fft_reg.h"
#include "kernels.h"
#include "kernels_reg.h"
#include "tables.h"
#include "tune_cache.h"

namespace sgm {

constexpr int kGlThreads = 256;
// Minimum waves per SIMD the pass kernels are compiled for: caps the registers
// so three 256-thread work-groups fit a CU (measured faster than the
// unconstrained two, despite a small call-frame spill).
constexpr int kGlWavesPerSimd = 3;

constexpr int gmin(int a, int b) { return a < b ? a : b; }

// Launch configurations: threads-per-line bound, largest radix, exchange
// buffers, LDS budget per block.
template <int NTMAX_, int MAXR_, int NB_, int LDSB_>
struct GLCfg {
    static constexpr int NTMAX = NTMAX_, MAXR = MAXR_, NB = NB_, LDSB = LDSB_;
};
using GLCfgA = GLCfg<64, 4, 1, 65536>;   // 12 points per thread, small tiles
using GLCfgB = GLCfg<32, 8, 1, 98304>;   // 24 points per thread, wider column tiles
using GLCfgC = GLCfg<64, 4, 2, 131072>;  // two exchange buffers
constexpr int kGlCfgs = 3;

// Padded lengths with register-FFT specialisations (kind k <-> kGlRegLen[k]).
constexpr int kGlRegLen[7] = {48, 96, 192, 288, 384, 576, 768};

template <int M, class CF>
struct GGeo {
    static constexpr Sched sd = make_sched(M, CF::NTMAX, CF::MAXR);
    static constexpr int NT = sd.NT;
    static constexpr int E = sd.E;
    static constexpr int W0 = gmin(kGlThreads / NT, CF::LDSB / (16 * CF::NB * M));
    static constexpr int W = W0 > 0 ? W0 : 1;
    static constexpr int THREADS = W * NT;
    static constexpr int B1OFF = CF::NB == 2 ? W * M : 0;
};

struct GLProb {
    int N, M;
    int kind;       // index into the compiled padded lengths, -1 = generic
    int wrows;      // lines per block, rows passes
    int wcols;      // lines per block, column pass
    long off_s;     // complex offset of the N x N arrays
    long off_w;     // complex offset of the N x M workspace
    long off_e;     // complex offset of the 1D integrating-factor table
    RadixPlan rp;   // FFT of length M (tw valid for both paths)
};

struct GLItem {
    int prob;
    int line0;
};

enum GLMode { kGlRhs = 0, kGlRk4 = 1, kGlIfRk4 = 2 };

struct GLStage {
    const double2* vin;  // stage input (state for stage 0)
    double2* state;
    double2* v;
    double2* acc;
    double2* rhs;        // kGlRhs output
    const double2* etab; // exp(-(1 + i b) k^2 dt / 2) per problem and 1D wavenumber
    double ks;           // 2 pi / L
    double b, c, dt;
    double edt;          // exp(dt / 2)
    int mode, stage;
};

__device__ __forceinline__ int gwn(int q, int M) { return q < (M + 1) / 2 ? q : q - M; }
__device__ __forceinline__ bool kept(int l, int N) { return l >= -(N / 2) && l <= (N - 1) / 2; }
__device__ __forceinline__ int nidx(int l, int N) { return l >= 0 ? l : l + N; }

// Stage operands touched once per stage (state, accumulator, stage input):
// non-temporal, so the padded workspace, which every pass reads back, keeps the MALL.
// One 16-byte access per element (two 8-byte halves would be two partial-line
// requests for the same line).
typedef double nt_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ntld(const double2* p) {
    const nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void ntst(double2* p, double2 v) {
    nt_d2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<nt_d2*>(p));
}

// Operands of one retained mode's stage update (the stage input for the explicit
// schemes, state, accumulator, the integrating factor's y part).
struct StageIn {
    double2 vv, u0, a, ey;
};

typedef __attribute__((address_space(1))) const nt_d2 g_nt_d2;
__device__ __forceinline__ double2 ntld_g(const double2* p) {
    const nt_d2 v = __builtin_nontemporal_load((g_nt_d2*)(const void*)p);
    return make_double2(v.x, v.y);
}

__device__ __forceinline__ StageIn stage_load(const GLStage& s, const GLProb& pr, long idx, int kyi) {
    StageIn in;
    in.vv = in.u0 = in.a = in.ey = make_double2(0.0, 0.0);
    if (s.mode == kGlRhs || s.mode == kGlRk4) {
        in.vv = ntld_g(s.vin + idx);
        if (s.mode == kGlRhs) return in;
    } else {
        const __attribute__((address_space(1))) double* pe =
            (const __attribute__((address_space(1))) double*)(const void*)(s.etab + pr.off_e + kyi);
        in.ey = make_double2(pe[0], pe[1]);
    }
    in.u0 = ntld_g(s.state + idx);
    if (s.stage > 0) in.a = ntld_g(s.acc + idx);
    return in;
}

// Stage update of one retained mode from its loaded operands, ex = the
// integrating factor's x part (IF-RK4).  k = N(v) = -F_trunc[(1 + i c)|u_p|^2 u_p].
// Returns the input of the next stage (stages 0..2); stores it in s.v when
// store_v (the explicit scheme needs it again for L v).
__device__ __forceinline__ double2 stage_apply(const GLStage& s, const GLProb& pr, long idx, int kxi, int kyi,
                                               double2 k, const StageIn& in, double2 ex, bool store_v) {
    double2 vn = make_double2(0.0, 0.0);
    if (s.mode == kGlRhs || s.mode == kGlRk4) {
        const double kx = gwn(kxi, pr.N) * s.ks, ky = gwn(kyi, pr.N) * s.ks;
        const double k2 = kx * kx + ky * ky;
        const double2 vv = in.vv;
        // dU = (1 - (1 + i b) k^2) v + k
        const double2 du = make_double2((1.0 - k2) * vv.x + s.b * k2 * vv.y + k.x,
                                        (1.0 - k2) * vv.y - s.b * k2 * vv.x + k.y);
        if (s.mode == kGlRhs) { s.rhs[idx] = du; return vn; }
        const double2 u0 = in.u0;
        const double dt = s.dt;
        if (s.stage == 0) {
            ntst(s.acc + idx, make_double2(u0.x + dt / 6 * du.x, u0.y + dt / 6 * du.y));
            vn = make_double2(u0.x + dt / 2 * du.x, u0.y + dt / 2 * du.y);
        } else if (s.stage < 3) {
            const double2 a = in.a;
            ntst(s.acc + idx, make_double2(a.x + dt / 3 * du.x, a.y + dt / 3 * du.y));
            const double bb = s.stage == 1 ? dt / 2 : dt;
            vn = make_double2(u0.x + bb * du.x, u0.y + bb * du.y);
        } else {
            const double2 a = in.a;
            ntst(s.state + idx, make_double2(a.x + dt / 6 * du.x, a.y + dt / 6 * du.y));
            return vn;
        }
        if (store_v) s.v[idx] = vn;
        return vn;
    }
    // integrating-factor RK4; E = exp(Lhat dt/2) = e^{dt/2} ex(kx) ex(ky)
    const double2 E = cscale(cmul(ex, in.ey), s.edt);
    const double2 u0 = in.u0;
    const double dt = s.dt;
    if (s.stage == 0) {
        const double2 E2 = cmul(E, E);
        const double2 a = make_double2(u0.x + dt / 6 * k.x, u0.y + dt / 6 * k.y);
        ntst(s.acc + idx, cmul(E2, a));
        vn = cmul(E, make_double2(u0.x + dt / 2 * k.x, u0.y + dt / 2 * k.y));
    } else if (s.stage == 1) {
        const double2 Ek = cmul(E, k);
        const double2 a = in.a;
        ntst(s.acc + idx, make_double2(a.x + dt / 3 * Ek.x, a.y + dt / 3 * Ek.y));
        const double2 Eu = cmul(E, u0);
        vn = make_double2(Eu.x + dt / 2 * k.x, Eu.y + dt / 2 * k.y);
    } else if (s.stage == 2) {
        const double2 Ek = cmul(E, k);
        const double2 a = in.a;
        ntst(s.acc + idx, make_double2(a.x + dt / 3 * Ek.x, a.y + dt / 3 * Ek.y));
        const double2 E2u = cmul(E, cmul(E, u0));
        vn = make_double2(E2u.x + dt * Ek.x, E2u.y + dt * Ek.y);
    } else {
        const double2 a = in.a;
        ntst(s.state + idx, make_double2(a.x + dt / 6 * k.x, a.y + dt / 6 * k.y));
        return vn;
    }
    if (store_v) s.v[idx] = vn;
    return vn;
}

__device__ __forceinline__ double2 stage_update(const GLStage& s, const GLProb& pr, long idx, int kxi, int kyi,
                                                double2 k, bool store_v) {
    const double2 ex = s.mode == kGlIfRk4 ? s.etab[pr.off_e + kxi] : make_double2(0.0, 0.0);
    return stage_apply(s, pr, idx, kxi, kyi, k, stage_load(s, pr, idx, kyi), ex, store_v);
}

// The stage updates of a thread's retained modes in one scope whose operand
// arrays are restrict parameters: the state, accumulator, stage output, stage
// input, right-hand side and integrating-factor table never overlap, so a mode's
// loads may be issued before the previous mode's stores.
template <int M, int NT, int E>
__device__ __forceinline__ void stage_row(double2 (&x)[E], double2* __restrict__ state, double2* __restrict__ acc,
                                          double2* __restrict__ v, const double2* __restrict__ etab,
                                          const double2* __restrict__ vin, double2* __restrict__ rhs,
                                          const GLStage& st0, const GLProb& pr, int row, int t, bool act, bool store_v) {
    GLStage st = st0;
    st.state = state;
    st.acc = acc;
    st.v = v;
    st.etab = etab;
    st.vin = vin;
    st.rhs = rhs;
    const int N = pr.N;
    const double s = -1.0 / M;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int l = gwn(t + NT * e, M);
        double2 vn = make_double2(0.0, 0.0);
        if (act && kept(l, N)) {
            const int ky = nidx(l, N);
            vn = stage_update(st, pr, pr.off_s + (long)row * N + ky, row, ky, cscale(x[e], s), store_v);
        }
        x[e] = vn;
    }
}

// A value every lane of the wave holds, moved to scalar registers.
template <class T>
__device__ __forceinline__ T wave_uniform(const T& v) {
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    int w[sizeof(T) / 4];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
    T r;
    __builtin_memcpy(&r, w, sizeof(T));
    return r;
}

// ---------------- register-FFT specialisations -----------------------------
// Twiddles of a work item's length M from a two-level table in LDS: w^i =
// A[i / 16] B[i % 16] with A[h] = w^(16 h), B[l] = w^l (M / 16 + 16 entries per
// compiled length, 259 for all seven, built on the host in extended precision;
// the product is within a few ulp of w^i).  The register FFT of the transforms
// reads each stage's twiddles from global memory, a dependent load right after
// every exchange barrier; the GL passes wait on it at three waves per SIMD, so
// they run their own copy of the stage loop with this table, which each
// work-group loads into LDS once per launch.
constexpr int kGlTwSize[7] = {48 / 16 + 16, 96 / 16 + 16, 192 / 16 + 16, 288 / 16 + 16,
                              384 / 16 + 16, 576 / 16 + 16, 768 / 16 + 16};
constexpr int gl_tw_base(int M) {
    int off = 0;
    for (int k = 0; k < 7 && kGlRegLen[k] != M; ++k) off += kGlTwSize[k];
    return off;
}
constexpr int kGlTwTotal = gl_tw_base(0);
static_assert(kGlTwTotal == 259, "sum of M / 16 + 16 over the compiled lengths");

__device__ __forceinline__ void gl_load_tw_all(const double2* twtab, double2* lds) {
    for (int i = threadIdx.x; i < kGlTwTotal; i += blockDim.x) lds[i] = twtab[i];
    __syncthreads();
}

template <int M, int SIGN>
__device__ __forceinline__ double2 gl_twiddle(const double2* twl, int i) {
    const double2 w = cmul(twl[i >> 4], twl[M / 16 + (i & 15)]);
    return SIGN < 0 ? w : cconj(w);
}

// The stage loop of reg_fft (same schedule, exchanges and barriers) with the
// twiddles from gl_twiddle.
template <int L, int NTMAX, int SIGN, int S, int NBUF, int MAXR>
__device__ __forceinline__ void gl_stages(double2* x, double2* b0, double2* b1, int ps, int t, const double2* twl,
                                          bool act) {
    constexpr Sched sd = make_sched(L, NTMAX, MAXR);
    if constexpr (S < sd.nst) {
        constexpr int p = sd.rad[S];
        constexpr int m = sched_m(sd, S);
        constexpr int E = sd.E;
        constexpr int NT = sd.NT;
        constexpr int Q = E / p;
        constexpr bool last = (S == sd.nst - 1);
        double2* buf = (NBUF == 2 && (S & 1)) ? b1 : b0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = t + NT * q;
            const int k = i % m;
            double2 y[p];
#pragma unroll
            for (int r = 0; r < p; ++r) y[r] = x[q + r * Q];
            if constexpr (m > 1) {
                const int step = k * (L / (p * m));
#pragma unroll
                for (int r = 1; r < p; ++r) y[r] = cmul(y[r], gl_twiddle<L, SIGN>(twl, r * step));
            }
            Dft<p, SIGN>::run(y);
            if constexpr (last) {
#pragma unroll
                for (int r = 0; r < p; ++r) x[q + r * Q] = y[r];
            } else {
                const int j = (i - k) * p + k;
                if (act) {
#pragma unroll
                    for (int r = 0; r < p; ++r) buf[(j + r * m) * ps] = y[r];
                }
            }
        }
        if constexpr (!last) {
            __syncthreads();
            if (act) {
#pragma unroll
                for (int e = 0; e < E; ++e) x[e] = buf[(t + NT * e) * ps];
            }
            if constexpr (NBUF == 1 && S + 1 < sd.nst - 1) __syncthreads();
            gl_stages<L, NTMAX, SIGN, S + 1, NBUF, MAXR>(x, b0, b1, ps, t, twl, act);
        }
    }
}

template <int M, class CF, int SIGN>
__device__ __forceinline__ void gl_fft(double2* x, double2* b0, double2* b1, int ps, int t, const double2* twl, bool act) {
    gl_stages<M, CF::NTMAX, SIGN, 0, CF::NB, CF::MAXR>(x, b0, b1, ps, t, twl, act);
}

template <int M, class CF>
__device__ __attribute__((noinline)) void rows_inv_reg(const GLProb& prr, int line0, const double2* src, double2* work, double2* lds,
                                                       const double2* twall) {
    using G = GGeo<M, CF>;
    // the descriptor's fields in scalar registers (see rows_fwd_reg)
    GLProb pr;
    pr.N = __builtin_amdgcn_readfirstlane(prr.N);
    pr.off_s = wave_uniform(prr.off_s);
    pr.off_w = wave_uniform(prr.off_w);
    const int t = threadIdx.x % G::NT, g = threadIdx.x / G::NT;
    const int row = line0 + g;
    const bool act = threadIdx.x < G::THREADS && row < pr.N;
    const int N = pr.N;
    double2 x[G::E];
#pragma unroll
    for (int e = 0; e < G::E; ++e) {
        const int q = t + G::NT * e;
        const int l = gwn(q, M);
        x[e] = (act && kept(l, N)) ? src[pr.off_s + (long)row * N + nidx(l, N)] : make_double2(0.0, 0.0);
    }
    const double2* twl = twall + gl_tw_base(M);
    gl_fft<M, CF, 1>(x, lds + g * M, lds + G::B1OFF + g * M, 1, t, twl, act);
    if (act) {
#pragma unroll
        for (int e = 0; e < G::E; ++e) work[pr.off_w + (long)row * M + t + G::NT * e] = x[e];
    }
}

template <int M, class CF>
__device__ __attribute__((noinline)) void cols_reg(const GLProb& prr, int line0, double2* work, double2* lds, double cnl,
                                                   const double2* twall) {
    using G = GGeo<M, CF>;
    // the descriptor's fields in scalar registers (see rows_fwd_reg)
    GLProb pr;
    pr.N = __builtin_amdgcn_readfirstlane(prr.N);
    pr.off_w = wave_uniform(prr.off_w);
    const int c = threadIdx.x % G::W, t = threadIdx.x / G::W;
    const int y = line0 + c;
    const bool act = threadIdx.x < G::THREADS && y < M;
    const int N = pr.N;
    double2 x[G::E];
#pragma unroll
    for (int e = 0; e < G::E; ++e) {
        const int q = t + G::NT * e;
        const int l = gwn(q, M);
        x[e] = (act && kept(l, N)) ? work[pr.off_w + (long)nidx(l, N) * M + y] : make_double2(0.0, 0.0);
    }
    const double2* twl = twall + gl_tw_base(M);
    gl_fft<M, CF, 1>(x, lds + c, lds + G::B1OFF + c, G::W, t, twl, act);
#pragma unroll
    for (int e = 0; e < G::E; ++e) {
        const double2 u = x[e];
        const double r2 = u.x * u.x + u.y * u.y;
        // (1 + i c) r2 u
        x[e] = make_double2(r2 * (u.x - cnl * u.y), r2 * (u.y + cnl * u.x));
    }
    __syncthreads();
    gl_fft<M, CF, -1>(x, lds + c, lds + G::B1OFF + c, G::W, t, twl, act);
    if (act) {
        const double s = 1.0 / M;
#pragma unroll
        for (int e = 0; e < G::E; ++e) {
            const int q = t + G::NT * e;
            const int l = gwn(q, M);
            if (kept(l, N)) work[pr.off_w + (long)nidx(l, N) * M + y] = cscale(x[e], s);
        }
    }
}

// FUSE: after the stage update, zero-pad the new stage input of the row and
// inverse-transform it along y (pass A of the next stage) into the workspace.
template <int M, class CF, bool FUSE>
__device__ __attribute__((noinline)) void rows_fwd_reg(const GLProb& prr, int line0, double2* work, double2* lds,
                                                       const GLStage& str, const double2* twall) {
    using G = GGeo<M, CF>;
    // Descriptors by value in scalar registers (every lane holds the same ones):
    // read through the references, every store of the stage update could (for the
    // compiler) change them, so each retained mode would reload them.
    GLProb pr;
    pr.N = __builtin_amdgcn_readfirstlane(prr.N);
    pr.off_s = wave_uniform(prr.off_s);
    pr.off_w = wave_uniform(prr.off_w);
    pr.off_e = wave_uniform(prr.off_e);
    const GLStage st = wave_uniform(str);
    const int t = threadIdx.x % G::NT, g = threadIdx.x / G::NT;
    const int row = line0 + g;
    const bool act = threadIdx.x < G::THREADS && row < pr.N;
    double2 x[G::E];
#pragma unroll
    for (int e = 0; e < G::E; ++e)
        x[e] = act ? work[pr.off_w + (long)row * M + t + G::NT * e] : make_double2(0.0, 0.0);
    const double2* twl = twall + gl_tw_base(M);
    gl_fft<M, CF, -1>(x, lds + g * M, lds + G::B1OFF + g * M, 1, t, twl, act);
    const bool store_v = !FUSE || st.mode == kGlRk4;
    stage_row<M, G::NT, G::E>(x, st.state, st.acc, st.v, st.etab, st.vin, st.rhs, st, pr, row, t, act, store_v);
    if constexpr (FUSE) {
        __syncthreads();
        gl_fft<M, CF, 1>(x, lds + g * M, lds + G::B1OFF + g * M, 1, t, twl, act);
        if (act) {
#pragma unroll
            for (int e = 0; e < G::E; ++e) work[pr.off_w + (long)row * M + t + G::NT * e] = x[e];
        }
    }
}

// ---------------- generic (any M) paths ------------------------------------
__device__ void rows_inv_gen(const GLProb& pr, int line0, const double2* src, double2* work, double2* lds) {
    const int M = pr.M, N = pr.N, W = pr.wrows;
    double2* A = lds;
    double2* B = lds + (long)W * M;
    for (int f = threadIdx.x; f < W * M; f += blockDim.x) {
        const int g = f / M, q = f - g * M;
        const int row = line0 + g, l = gwn(q, M);
        A[f] = (row < N && kept(l, N)) ? src[pr.off_s + (long)row * N + nidx(l, N)] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double2* R = lds_fft<1>(A, B, pr.rp, W, 1, M, false);
    for (int f = threadIdx.x; f < W * M; f += blockDim.x) {
        const int g = f / M, q = f - g * M;
        const int row = line0 + g;
        if (row < N) work[pr.off_w + (long)row * M + q] = R[f];
    }
}

__device__ void cols_gen(const GLProb& pr, int line0, double2* work, double2* lds, double cnl) {
    const int M = pr.M, N = pr.N, W = pr.wcols;
    double2* A = lds;
    double2* B = lds + (long)W * M;
    for (int f = threadIdx.x; f < W * M; f += blockDim.x) {
        const int q = f / W, c = f - q * W;
        const int y = line0 + c, l = gwn(q, M);
        A[f] = (y < M && kept(l, N)) ? work[pr.off_w + (long)nidx(l, N) * M + y] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double2* R = lds_fft<1>(A, B, pr.rp, W, W, 1, true);
    for (int f = threadIdx.x; f < W * M; f += blockDim.x) {
        const double2 u = R[f];
        const double r2 = u.x * u.x + u.y * u.y;
        R[f] = make_double2(r2 * (u.x - cnl * u.y), r2 * (u.y + cnl * u.x));
    }
    __syncthreads();
    double2* O = (R == A) ? B : A;
    double2* R2 = lds_fft<-1>(R, O, pr.rp, W, W, 1, true);
    const double s = 1.0 / M;
    for (int f = threadIdx.x; f < W * M; f += blockDim.x) {
        const int q = f / W, c = f - q * W;
        const int y = line0 + c, l = gwn(q, M);
        if (y < M && kept(l, N)) work[pr.off_w + (long)nidx(l, N) * M + y] = cscale(R2[f], s);
    }
}

__device__ void rows_fwd_gen(const GLProb& pr, int line0, double2* work, double2* lds, const GLStage& st,
                             bool fuse) {
    const int M = pr.M, N = pr.N, W = pr.wrows;
    double2* A = lds;
    double2* B = lds + (long)W * M;
    for (int f = threadIdx.x; f < W * M; f += blockDim.x) {
        const int g = f / M;
        const int row = line0 + g;
        A[f] = row < N ? work[pr.off_w + (long)row * M + (f - g * M)] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    double2* R = lds_fft<-1>(A, B, pr.rp, W, 1, M, false);
    const double s = -1.0 / M;
    const bool store_v = !fuse || st.mode == kGlRk4;
    for (int f = threadIdx.x; f < W * M; f += blockDim.x) {
        const int g = f / M, q = f - g * M;
        const int row = line0 + g, l = gwn(q, M);
        double2 vn = make_double2(0.0, 0.0);
        if (row < N && kept(l, N)) {
            const int ky = nidx(l, N);
            vn = stage_update(st, pr, pr.off_s + (long)row * N + ky, row, ky, cscale(R[f], s), store_v);
        }
        R[f] = vn;
    }
    if (!fuse) return;
    __syncthreads();
    double2* O = (R == A) ? B : A;
    double2* R2 = lds_fft<1>(R, O, pr.rp, W, 1, M, false);
    for (int f = threadIdx.x; f < W * M; f += blockDim.x) {
        const int g = f / M;
        const int row = line0 + g;
        if (row < N) work[pr.off_w + (long)row * M + (f - g * M)] = R2[f];
    }
}

// ---------------- pass kernels ---------------------------------------------
#define SGM_GL_SWITCH(KIND, CALL_REG)  \
    switch (KIND) {                     \
        case 0: CALL_REG(48); break;    \
        case 1: CALL_REG(96); break;    \
        case 2: CALL_REG(192); break;   \
        case 3: CALL_REG(288); break;   \
        case 4: CALL_REG(384); break;   \
        case 5: CALL_REG(576); break;   \
        case 6: CALL_REG(768); break;   \
        default: break;                 \
    }

template <class CF>
static int reg_w(int kind) {
    switch (kind) {
        case 0: return GGeo<48, CF>::W;
        case 1: return GGeo<96, CF>::W;
        case 2: return GGeo<192, CF>::W;
        case 3: return GGeo<288, CF>::W;
        case 4: return GGeo<384, CF>::W;
        case 5: return GGeo<576, CF>::W;
        case 6: return GGeo<768, CF>::W;
        default: return 0;
    }
}

// The items of a launch in 8 contiguous chunks, chunk x taken by the blocks
// b = x mod 8 (work-groups go to the 8 XCDs round-robin, block b to XCD b mod 8)
// in a stride loop: neighbouring column tiles share the cache lines at their
// edges (tiles of 4 or 5 columns are 64 or 80 bytes wide), and those then meet
// in one XCD's L2.  A persistent grid when gridDim.x is smaller than the item
// count, one block per item otherwise; a plain grid stride when the grid is not
// a multiple of 8.
struct ItemRange {
    int it, hi, step;
};
__device__ __forceinline__ ItemRange item_range(int n) {
    const int G = (int)gridDim.x, b = (int)blockIdx.x;
    if (G & 7) return {b, n, G};
    const int x = b & 7;
    return {(int)((long)n * x / 8) + (b >> 3), (int)((long)n * (x + 1) / 8), G >> 3};
}
template <class CF, bool GEN>
__global__ void __launch_bounds__(kGlThreads, kGlWavesPerSimd) k_gl_rows_inv(const GLProb* probs, const GLItem* items, int nitems,
                                                            const double2* src, double2* work, const double2* twtab) {
    extern __shared__ double2 lds[];
    if constexpr (!GEN) gl_load_tw_all(twtab, lds);
    for (ItemRange r = item_range(nitems); r.it < r.hi; r.it += r.step) {
        const GLItem item = items[r.it];
        const GLProb pr = probs[item.prob];
        if constexpr (GEN) {
            rows_inv_gen(pr, item.line0, src, work, lds);
        } else {
#define R_(MM) rows_inv_reg<MM, CF>(pr, item.line0, src, work, lds + kGlTwTotal, lds)
            SGM_GL_SWITCH(pr.kind, R_)
#undef R_
        }
        __syncthreads();
    }
}

template <class CF, bool GEN>
__global__ void __launch_bounds__(kGlThreads, kGlWavesPerSimd) k_gl_cols(const GLProb* probs, const GLItem* items, int nitems,
                                                        double2* work, double cnl, const double2* twtab) {
    extern __shared__ double2 lds[];
    if constexpr (!GEN) gl_load_tw_all(twtab, lds);
    for (ItemRange r = item_range(nitems); r.it < r.hi; r.it += r.step) {
        const GLItem item = items[r.it];
        const GLProb pr = probs[item.prob];
        if constexpr (GEN) {
            cols_gen(pr, item.line0, work, lds, cnl);
        } else {
#define C_(MM) cols_reg<MM, CF>(pr, item.line0, work, lds + kGlTwTotal, cnl, lds)
            SGM_GL_SWITCH(pr.kind, C_)
#undef C_
        }
        __syncthreads();
    }
}

template <class CF, bool GEN, bool FUSE>
__global__ void __launch_bounds__(kGlThreads, kGlWavesPerSimd) k_gl_rows_fwd(const GLProb* probs, const GLItem* items, int nitems,
                                                            double2* work, GLStage st, const double2* twtab) {
    extern __shared__ double2 lds[];
    if constexpr (!GEN) gl_load_tw_all(twtab, lds);
    for (ItemRange r = item_range(nitems); r.it < r.hi; r.it += r.step) {
        const GLItem item = items[r.it];
        const GLProb pr = probs[item.prob];
        if constexpr (GEN) {
            rows_fwd_gen(pr, item.line0, work, lds, st, FUSE);
        } else {
#define F_(MM) rows_fwd_reg<MM, CF, FUSE>(pr, item.line0, work, lds + kGlTwTotal, st, lds)
            SGM_GL_SWITCH(pr.kind, F_)
#undef F_
        }
        __syncthreads();
    }
}

// Launch table of one configuration.
struct GLKern {
    void (*rows_inv)(const GLProb*, const GLItem*, int, const double2*, double2*, const double2*);
    void (*cols)(const GLProb*, const GLItem*, int, double2*, double, const double2*);
    void (*rows_fwd)(const GLProb*, const GLItem*, int, double2*, GLStage, const double2*);
    void (*rows_fwd_fused)(const GLProb*, const GLItem*, int, double2*, GLStage, const double2*);
    int (*w)(int);
    int nb, ldsb;
};
template <class CF, bool GEN>
static GLKern glkern() {
    return {k_gl_rows_inv<CF, GEN>, k_gl_cols<CF, GEN>, k_gl_rows_fwd<CF, GEN, false>, k_gl_rows_fwd<CF, GEN, true>,
            reg_w<CF>, CF::NB, CF::LDSB};
}
static GLKern glkern_cfg(int cfg, bool gen) {
    if (gen) return glkern<GLCfgA, true>();
    switch (cfg) {
        case 1: return glkern<GLCfgB, false>();
        case 2: return glkern<GLCfgC, false>();
        default: return glkern<GLCfgA, false>();
    }
}

}  // namespace sgm

using namespace sgm;

// Work lists 0..kGlCfgs-1: register-specialised problems tiled for that
// configuration; list kGlCfgs: problems on the generic path.
constexpr int kGlLists = kGlCfgs + 1;

struct sgm_gl_s {
    sgm_gl_desc d;
    std::vector<int> N, M;
    std::vector<int64_t> off_s, off_w, off_e;
    std::vector<RadixPlan> rpN;   // FFT of length N (forward/backward helpers)
    std::vector<int> hasN;
    std::vector<RegKernels> rkN;
    // rows lists (passes A and C) and column lists (pass B)
    int nA[kGlLists] = {}, nB[kGlLists] = {};
    size_t lds[kGlLists] = {};
    bool cfg_ok[kGlCfgs] = {};
    int cfg = 0, gridmode = 0;
    int ncu = 256, lmax = 65536;
    void* dev = nullptr;         // probs + items + twiddles + etab
    GLProb* dprobs[kGlLists] = {};
    GLItem* ditemsA[kGlLists] = {};
    GLItem* ditemsB[kGlLists] = {};
    double2* etab = nullptr;
    double2* twtab = nullptr;    // two-level twiddle tables of the compiled padded lengths
    double2* v = nullptr;
    double2* acc = nullptr;
    double2* work = nullptr;
    hipStream_t cap = nullptr;   // private stream for graph capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void* graph_state = nullptr;
};

static int glkind(int M) {
    for (int i = 0; i < 7; ++i)
        if (kGlRegLen[i] == M) return i;
    return -1;
}

extern "C" sgm_status sgm_gl_destroy(sgm_gl g) {
    clear_error();
    if (!g) return SGM_OK;
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    if (g->cap) hipStreamDestroy(g->cap);
    hipFree(g->v);
    hipFree(g->acc);
    hipFree(g->work);
    hipFree(g->dev);
    delete g;
    return SGM_OK;
}

static int gl_grid(sgm_gl g, int k, int n) {
    if (g->gridmode == 1) return (n + 7) & ~7;  // one block per item (a multiple of 8: see item_range)
    const int per_cu = std::min(8, std::max(1, (int)(g->lmax / std::max<size_t>(g->lds[k], 1))));
    return std::min(n, g->ncu * per_cu);
}

// pass 0: rows inverse (A), 1: columns (B), 2: rows forward + stage update (C),
// 3: C fused with A of the next stage.
static sgm_status gl_pass(sgm_gl g, int pass, const double2* src, const GLStage& st, hipStream_t s) {
    const int lists[2] = {g->cfg, kGlCfgs};
    for (int k : lists) {
        const int n = pass == 1 ? g->nB[k] : g->nA[k];
        if (!n) continue;
        const GLKern kn = glkern_cfg(k == kGlCfgs ? 0 : k, k == kGlCfgs);
        const GLItem* items = pass == 1 ? g->ditemsB[k] : g->ditemsA[k];
        const dim3 grid(gl_grid(g, k, n)), block(kGlThreads);
        const GLProb* probs = g->dprobs[k];
        if (pass == 0)
            hipLaunchKernelGGL(kn.rows_inv, grid, block, g->lds[k], s, probs, items, n, src, g->work, g->twtab);
        else if (pass == 1)
            hipLaunchKernelGGL(kn.cols, grid, block, g->lds[k], s, probs, items, n, g->work, g->d.c, g->twtab);
        else
            hipLaunchKernelGGL(pass == 3 ? kn.rows_fwd_fused : kn.rows_fwd, grid, block, g->lds[k], s, probs, items, n,
                               g->work, st, g->twtab);
        SGM_HIP_TRY(hipGetLastError());
    }
    return SGM_OK;
}

static GLStage base_stage(sgm_gl g) {
    GLStage st{};
    st.v = g->v;
    st.acc = g->acc;
    st.etab = g->etab;
    st.ks = 6.283185307179586476925286766559 / g->d.L;
    st.b = g->d.b;
    st.c = g->d.c;
    st.dt = g->d.dt;
    st.edt = std::exp(g->d.dt / 2);
    return st;
}

// One time step: A(state), then per stage B and C, C of stages 0..2 fused
// with A of the following stage.
static sgm_status gl_enqueue_step(sgm_gl g, double2* state, hipStream_t s) {
    GLStage st = base_stage(g);
    st.mode = g->d.scheme == SGM_IFRK4 ? kGlIfRk4 : kGlRk4;
    st.state = state;
    sgm_status r = gl_pass(g, 0, state, st, s);
    for (int k = 0; k < 4 && r == SGM_OK; ++k) {
        st.stage = k;
        st.vin = k == 0 ? state : g->v;
        r = gl_pass(g, 1, nullptr, st, s);
        if (r == SGM_OK) r = gl_pass(g, k < 3 ? 3 : 2, nullptr, st, s);
    }
    return r;
}

// Cache key of a batch: device, scheme and the multiset of sizes.
static std::string gl_tune_key(sgm_gl g) {
    std::map<int, int> cnt;
    for (int n : g->N) ++cnt[n];
    std::string k = "gl " + tune_device_tag() + " scheme" + std::to_string(g->d.scheme);
    for (auto& [n, c] : cnt) k += " " + std::to_string(n) + "x" + std::to_string(c);
    return k;
}

// Times one step of each candidate configuration on a scratch state and keeps
// the fastest (or takes the choice stored for this device and batch shape).
// Runs on the creation stream before the batch is handed out.
static sgm_status gl_autotune(sgm_gl g, int64_t os, hipStream_t s) {
    const std::string key = gl_tune_key(g);
    std::vector<int> cached;
    if (tune_cache_get(key, cached) && cached.size() == 1 && cached[0] >= 0 && cached[0] < 2 * kGlCfgs &&
        g->cfg_ok[cached[0] / 2]) {
        g->cfg = cached[0] / 2;
        g->gridmode = cached[0] % 2;
        return SGM_OK;
    }
    double2* state = nullptr;
    if (hipMalloc(&state, (size_t)os * sizeof(double2)) != hipSuccess) {
        set_error("hipMalloc of the tuning state failed");
        return SGM_ERR_OOM;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    sgm_status r = SGM_OK;
    float best = 1e30f;
    int bcfg = 0, bgrid = 0;
    if (hipMemsetAsync(state, 0, (size_t)os * sizeof(double2), s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        set_error("tuning set-up failed");
        r = SGM_ERR_HIP;
    }
    for (int v = 0; v < 2 * kGlCfgs && r == SGM_OK; ++v) {
        if (!g->cfg_ok[v / 2]) continue;
        g->cfg = v / 2;
        g->gridmode = v % 2;
        r = gl_enqueue_step(g, state, s);
        float tmin = 1e30f;
        for (int rep = 0; rep < 3 && r == SGM_OK; ++rep) {
            hipEventRecord(e0, s);
            r = gl_enqueue_step(g, state, s);
            if (r == SGM_OK) r = gl_enqueue_step(g, state, s);
            hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) {
                set_error("tuning run failed");
                r = SGM_ERR_HIP;
                break;
            }
            float ms = 0;
            hipEventElapsedTime(&ms, e0, e1);
            tmin = std::min(tmin, ms);
        }
        if (r == SGM_OK && tmin < best) {
            best = tmin;
            bcfg = g->cfg;
            bgrid = g->gridmode;
        }
    }
    hipStreamSynchronize(s);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(state);
    g->cfg = bcfg;
    g->gridmode = bgrid;
    if (r == SGM_OK) tune_cache_put(key, {2 * bcfg + bgrid});
    return r;
}

extern "C" sgm_status sgm_gl_create(const sgm_gl_desc* desc, void* stream, sgm_gl* out) {
    clear_error();
    TraceRange trace_range("sgm_gl_create");
    SGM_CHECK_ARG(desc && out && desc->N, "null argument");
    *out = nullptr;
    const sgm_gl_desc& d = *desc;
    SGM_CHECK_ARG(d.count >= 1, "count must be >= 1");
    SGM_CHECK_ARG(d.L > 0 && std::isfinite(d.L) && std::isfinite(d.dt) && std::isfinite(d.b) && std::isfinite(d.c),
                  "L must be > 0 and all coefficients finite");
    SGM_CHECK_ARG(d.scheme == SGM_RK4 || d.scheme == SGM_IFRK4, "unknown scheme %d", d.scheme);
    SGM_CHECK_ARG(d.tune == 0 || d.tune == 1 || (d.tune >= 16 && d.tune < 16 + 2 * kGlCfgs), "invalid tune %d",
                  d.tune);
    for (int i = 0; i < d.count; ++i)
        if (d.N[i] < 2 || d.N[i] > 4096) {
            set_error("problem %d: N = %d outside 2..4096", i, d.N[i]);
            return SGM_ERR_UNSUPPORTED_SIZE;
        }
    sgm_gl_s* g = new (std::nothrow) sgm_gl_s();
    if (!g) return SGM_ERR_OOM;
    g->d = d;
    g->d.N = nullptr;
    const int n = d.count;
    g->N.assign(d.N, d.N + n);
    int64_t os = 0, ow = 0, oe = 0;
    // twiddle tables: one per distinct length (M_i and N_i)
    std::vector<int> lens;
    for (int i = 0; i < n; ++i) {
        int Mi = (3 * g->N[i]) / 2;
        g->M.push_back(Mi);
        g->off_s.push_back(os);
        g->off_w.push_back(ow);
        g->off_e.push_back(oe);
        os += (int64_t)g->N[i] * g->N[i];
        ow += (int64_t)g->N[i] * Mi;
        oe += g->N[i];
        lens.push_back(Mi);
        lens.push_back(g->N[i]);
    }
    g->off_s.push_back(os);
    std::sort(lens.begin(), lens.end());
    lens.erase(std::unique(lens.begin(), lens.end()), lens.end());
    int dev = 0;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&g->ncu, hipDeviceAttributeMultiprocessorCount, dev);
    hipDeviceGetAttribute(&g->lmax, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    // per list: problem descriptors (line tiling depends on the configuration)
    // and items, problems in decreasing size so the grid-stride loop balances
    std::vector<GLProb> hp[kGlLists];
    std::vector<GLItem> itA[kGlLists], itB[kGlLists];
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return g->N[a] > g->N[b]; });
    for (int k = 0; k < kGlLists; ++k) {
        hp[k].resize(n);
        for (int i = 0; i < n; ++i) {
            GLProb& pr = hp[k][i];
            pr.N = g->N[i];
            pr.M = g->M[i];
            pr.kind = glkind(pr.M);
            pr.off_s = g->off_s[i];
            pr.off_w = g->off_w[i];
            pr.off_e = g->off_e[i];
            pr.rp.L = pr.M;
            pr.rp.nst = factor_radices(pr.M, pr.rp.radix);
            size_t lds;
            if (k == kGlCfgs) {
                pr.wrows = pr.wcols = std::max(1, std::min(16, 4096 / pr.M));
                lds = 2 * sizeof(double2) * (size_t)pr.wrows * pr.M;
            } else {
                const GLKern kn = glkern_cfg(k, false);
                pr.wrows = pr.wcols = pr.kind >= 0 ? kn.w(pr.kind) : 1;
                // the two-level twiddle tables of every compiled length, then the exchange buffers
                lds = sizeof(double2) * ((size_t)kGlTwTotal + (size_t)kn.nb * pr.wrows * pr.M);
            }
            const bool mine = (k == kGlCfgs) == (pr.kind < 0);
            if (mine) g->lds[k] = std::max(g->lds[k], lds);
        }
        for (int i : order) {
            const GLProb& pr = hp[k][i];
            if ((k == kGlCfgs) != (pr.kind < 0)) continue;
            for (int r = 0; r < pr.N; r += pr.wrows) itA[k].push_back({i, r});
            for (int y = 0; y < pr.M; y += pr.wcols) itB[k].push_back({i, y});
        }
        g->nA[k] = (int)itA[k].size();
        g->nB[k] = (int)itB[k].size();
    }
    if (g->lds[kGlCfgs] > (size_t)g->lmax) {
        set_error("padded length too large for one work-group's LDS");
        sgm_gl_destroy(g);
        return SGM_ERR_UNSUPPORTED_SIZE;
    }
    for (int k = 0; k < kGlCfgs; ++k) g->cfg_ok[k] = g->lds[k] <= (size_t)g->lmax;
    // integrating factor table ex(q) = exp(-(1 + i b) k_q^2 dt/2), k_q = 2 pi/L * wavenumber
    std::vector<double> etab(2 * (size_t)oe);
    const long double twopi = 6.283185307179586476925286766559L;
    for (int i = 0; i < n; ++i)
        for (int q = 0; q < g->N[i]; ++q) {
            int l = q < (g->N[i] + 1) / 2 ? q : q - g->N[i];
            long double k = twopi / (long double)d.L * l;
            long double a = -k * k * (long double)d.dt / 2;
            long double mag = expl(a);
            etab[2 * (g->off_e[i] + q)] = (double)(mag * cosl(d.b * a));
            etab[2 * (g->off_e[i] + q) + 1] = (double)(mag * sinl(d.b * a));
        }
    // device blob: probs[k] | itemsA[k] | itemsB[k] | etab | GL twiddle tables | twiddles
    std::vector<char> blob;
    auto add = [&](const void* p, size_t bytes) {
        size_t off = (blob.size() + 255) & ~size_t(255);
        blob.resize(off + bytes);
        if (bytes && p) std::memcpy(blob.data() + off, p, bytes);
        return off;
    };
    size_t o_p[kGlLists], o_A[kGlLists], o_B[kGlLists];
    for (int k = 0; k < kGlLists; ++k) {
        o_p[k] = add(nullptr, n * sizeof(GLProb));
        o_A[k] = add(itA[k].data(), itA[k].size() * sizeof(GLItem));
        o_B[k] = add(itB[k].data(), itB[k].size() * sizeof(GLItem));
    }
    size_t o_e = add(etab.data(), etab.size() * sizeof(double));
    // per compiled length M: A[h] = exp(-2 pi i 16 h / M), h < M / 16, then B[l] = exp(-2 pi i l / M), l < 16
    std::vector<double> gtab;
    for (int k = 0; k < 7; ++k) {
        const int M = kGlRegLen[k];
        for (int j = 0; j < M / 16 + 16; ++j) {
            const int r = j < M / 16 ? 16 * j : j - M / 16;
            const long double a = -twopi * (long double)r / (long double)M;
            gtab.push_back((double)cosl(a));
            gtab.push_back((double)sinl(a));
        }
    }
    size_t o_gt = add(gtab.data(), gtab.size() * sizeof(double));
    std::vector<size_t> o_tw(lens.size());
    for (size_t j = 0; j < lens.size(); ++j) {
        std::vector<double> tw = twiddles(lens[j]);
        o_tw[j] = add(tw.data(), tw.size() * sizeof(double));
    }
    auto twptr = [&](char* base, int L) {
        size_t j = std::lower_bound(lens.begin(), lens.end(), L) - lens.begin();
        return reinterpret_cast<const double2*>(base + o_tw[j]);
    };
    hipError_t e = hipMalloc(&g->dev, blob.size());
    if (e != hipSuccess) { set_error("hipMalloc: %s", hipGetErrorString(e)); sgm_gl_destroy(g); return SGM_ERR_OOM; }
    char* base = static_cast<char*>(g->dev);
    // patch device twiddle pointers into the descriptors before upload
    for (int k = 0; k < kGlLists; ++k) {
        for (int i = 0; i < n; ++i) hp[k][i].rp.tw = twptr(base, g->M[i]);
        std::memcpy(blob.data() + o_p[k], hp[k].data(), n * sizeof(GLProb));
    }
    hipStream_t cs = static_cast<hipStream_t>(stream);
    e = hipMemcpyAsync(g->dev, blob.data(), blob.size(), hipMemcpyHostToDevice, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);  // the host staging buffer goes out of scope
    if (e != hipSuccess) { set_error("uploading the tables: %s", hipGetErrorString(e)); sgm_gl_destroy(g); return SGM_ERR_HIP; }
    for (int k = 0; k < kGlLists; ++k) {
        g->dprobs[k] = reinterpret_cast<GLProb*>(base + o_p[k]);
        g->ditemsA[k] = reinterpret_cast<GLItem*>(base + o_A[k]);
        g->ditemsB[k] = reinterpret_cast<GLItem*>(base + o_B[k]);
    }
    g->etab = reinterpret_cast<double2*>(base + o_e);
    g->twtab = reinterpret_cast<double2*>(base + o_gt);
    g->rpN.resize(n);
    g->hasN.resize(n);
    g->rkN.resize(n);
    for (int i = 0; i < n; ++i) {
        g->rpN[i].L = g->N[i];
        g->rpN[i].nst = factor_radices(g->N[i], g->rpN[i].radix);
        g->rpN[i].tw = twptr(base, g->N[i]);
        g->hasN[i] = reg_kernels_for(g->N[i], g->rkN[i]);
    }
    if (hipMalloc(&g->v, os * sizeof(double2)) != hipSuccess || hipMalloc(&g->acc, os * sizeof(double2)) != hipSuccess ||
        hipMalloc(&g->work, ow * sizeof(double2)) != hipSuccess) {
        set_error("hipMalloc of the stage buffers failed");
        sgm_gl_destroy(g);
        return SGM_ERR_OOM;
    }
    if (d.tune >= 16) {
        const int v = d.tune - 16;
        if (!g->cfg_ok[v / 2]) {
            set_error("configuration %d needs more LDS than a work-group has", v);
            sgm_gl_destroy(g);
            return SGM_ERR_UNSUPPORTED_SIZE;
        }
        g->cfg = v / 2;
        g->gridmode = v % 2;
    } else if (d.tune == 1) {
        sgm_status r = gl_autotune(g, os, cs);
        if (r != SGM_OK) { sgm_gl_destroy(g); return r; }
    }
    *out = g;
    return SGM_OK;
}

extern "C" sgm_status sgm_gl_count(sgm_gl g, int* count) {
    clear_error();
    SGM_CHECK_ARG(g && count, "null argument");
    *count = (int)g->N.size();
    return SGM_OK;
}

extern "C" sgm_status sgm_gl_variant(sgm_gl g, int* variant) {
    clear_error();
    SGM_CHECK_ARG(g && variant, "null argument");
    *variant = 2 * g->cfg + g->gridmode;
    return SGM_OK;
}

extern "C" sgm_status sgm_gl_offsets(sgm_gl g, int64_t* offsets) {
    clear_error();
    SGM_CHECK_ARG(g && offsets, "null argument");
    for (size_t i = 0; i < g->off_s.size(); ++i) offsets[i] = g->off_s[i];
    return SGM_OK;
}

extern "C" sgm_status sgm_gl_rhs(sgm_gl g, const void* u_hat, void* rhs, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_gl_rhs");
    SGM_CHECK_ARG(g && u_hat && rhs, "null argument");
    SGM_CHECK_ARG(u_hat != rhs, "u_hat and rhs must not alias");
    GLStage st = base_stage(g);
    st.mode = kGlRhs;
    st.vin = static_cast<const double2*>(u_hat);
    st.rhs = static_cast<double2*>(rhs);
    hipStream_t s = static_cast<hipStream_t>(stream);
    sgm_status r = gl_pass(g, 0, st.vin, st, s);
    if (r == SGM_OK) r = gl_pass(g, 1, nullptr, st, s);
    if (r == SGM_OK) r = gl_pass(g, 2, nullptr, st, s);
    return r;
}

extern "C" sgm_status sgm_gl_step(sgm_gl g, void* u_hat, int nsteps, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_gl_step");
    SGM_CHECK_ARG(g && u_hat, "null argument");
    SGM_CHECK_ARG(nsteps >= 0, "nsteps must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2* state = static_cast<double2*>(u_hat);
    if (!g->d.graph) {
        for (int i = 0; i < nsteps; ++i) {
            sgm_status r = gl_enqueue_step(g, state, s);
            if (r != SGM_OK) return r;
        }
        return SGM_OK;
    }
    if (!g->exec || g->graph_state != u_hat) {
        if (g->exec) { hipGraphExecDestroy(g->exec); g->exec = nullptr; }
        if (g->graph) { hipGraphDestroy(g->graph); g->graph = nullptr; }
        if (!g->cap) SGM_HIP_TRY(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
        SGM_HIP_TRY(hipStreamBeginCapture(g->cap, hipStreamCaptureModeRelaxed));
        sgm_status r = gl_enqueue_step(g, state, g->cap);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(g->cap, &graph);
        if (r != SGM_OK) { if (graph) hipGraphDestroy(graph); return r; }
        SGM_HIP_TRY(e);
        g->graph = graph;
        SGM_HIP_TRY(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
        g->graph_state = u_hat;
    }
    for (int i = 0; i < nsteps; ++i) SGM_HIP_TRY(hipGraphLaunch(g->exec, s));
    return SGM_OK;
}

// Physical <-> spectral helpers (not on the time-stepping path): per run of
// consecutive problems of one size (packed back to back), the contiguous y
// transform over all their rows, then the strided x transform with the
// problems as outer slabs: two launches per run, not per problem.
static sgm_status gl_transform(sgm_gl g, const double2* in, double2* out, int sign, hipStream_t s) {
    const size_t np = g->N.size();
    for (size_t i = 0; i < np;) {
        const int N = g->N[i];
        size_t j = i + 1;
        while (j < np && g->N[j] == N && g->off_s[j] == g->off_s[j - 1] + (int64_t)N * N) ++j;
        const int cnt = (int)(j - i);
        const double2* src = in + g->off_s[i];
        double2* dst = out + g->off_s[i];
        const double sc = sign < 0 ? 1.0 / N : 1.0;
        const long nlines = (long)cnt * N;
        if (g->hasN[i]) {
            const RegKernels& k = g->rkN[i];
            hipLaunchKernelGGL(sign < 0 ? k.c2c_f : k.c2c_b, dim3((unsigned)((nlines + k.W - 1) / k.W)), dim3(k.threads),
                               k.lds, s, src, dst, (int)nlines, g->rpN[i].tw, sc);
            SGM_HIP_TRY(hipGetLastError());
            SGM_HIP_TRY(launch_strided(k, sign, dst, dst, cnt, N, g->rpN[i].tw, sc, s));
        } else {
            int G = std::max(1, std::min(16, 2048 / N));
            SGM_HIP_TRY(launch_lines_c2c(src, dst, N, (int)nlines, G, g->rpN[i], sign, sc, s));
            int W = std::max(1, std::min(16, 2048 / N));
            SGM_HIP_TRY(launch_strided_c2c(dst, dst, N, cnt, N, W, g->rpN[i], sign, sc, s));
        }
        i = j;
    }
    return SGM_OK;
}

extern "C" sgm_status sgm_gl_forward(sgm_gl g, const void* u, void* u_hat, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_gl_forward");
    SGM_CHECK_ARG(g && u && u_hat, "null argument");
    SGM_CHECK_ARG(u != u_hat, "u and u_hat must not alias");
    return gl_transform(g, static_cast<const double2*>(u), static_cast<double2*>(u_hat), -1,
                        static_cast<hipStream_t>(stream));
}

extern "C" sgm_status sgm_gl_backward(sgm_gl g, const void* u_hat, void* u, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_gl_backward");
    SGM_CHECK_ARG(g && u && u_hat, "null argument");
    SGM_CHECK_ARG(u != u_hat, "u and u_hat must not alias");
    return gl_transform(g, static_cast<const double2*>(u_hat), static_cast<double2*>(u), 1,
                        static_cast<hipStream_t>(stream));
}
