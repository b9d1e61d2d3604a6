// Transform passes built on the register-resident FFT (compile-time lengths).
//
// Every block has W lines x NT threads per line (256 threads, 512 for the wide
// variant).  For
// strided passes (middle periodic axis, Chebyshev axis) lane -> (column c =
// lane % W, thread t = lane / W), so one warp-wide access covers W adjacent
// columns of a row; for contiguous lines lane -> (t = lane % NT, line =
// lane / NT), so it covers NT adjacent points of a line.
#include "fft_reg.h"
#include "kernels.h"
#include "kernels_reg.h"
#include "solve_seg.h"
#include "solve_seg_dev.h"

#include <map>
#include <mutex>

namespace sgm {

constexpr int kThreads = 256;
constexpr int kNTMAX = 32;
constexpr int kLdsBudget = 131072;

constexpr int cmin(int a, int b) { return a < b ? a : b; }

// Work-groups go to the 8 XCDs round-robin (block b to XCD b mod 8).  Renumber
// them so that each XCD walks a contiguous range of tiles: neighbouring tiles
// share the cache lines that straddle their boundary (rows of M/2+1 complex
// values are not line aligned), and those then meet in one L2.  A bijection
// on [0, gridDim.x) for any grid size.
__device__ __forceinline__ int xcd_block() {
    const int per = (int)(gridDim.x >> 3), b = (int)blockIdx.x;
    return b < 8 * per ? (b & 7) * per + (b >> 3) : b;
}

// Launch geometry of one variant: NTMAX bounds the threads per line (so
// E = L / NT points per thread), NB is the number of exchange buffers, TH the
// block size to fill, MAXR the largest radix of the stage schedule (8: radix-8
// stages where the power of two allows; 4: radix-4/2 only, more stages with
// fewer twiddle products each).
template <int L, int NTMAX_, int NB_, int TH = kThreads, int MAXR_ = 8>
struct Geo {
    static constexpr int NTMAX = NTMAX_;
    static constexpr int NB = NB_;
    static constexpr int MAXR = MAXR_;
    static constexpr Sched sd = make_sched(L, NTMAX, MAXR);
    static constexpr int NT = sd.NT;
    static constexpr int E = sd.E;
    // lines per block: fill TH threads unless the exchange buffers
    // (NB * W * L * 16 bytes) would exceed the LDS budget
    static constexpr int W = cmin(TH / NT, kLdsBudget / (16 * NB * L)) > 0 ? cmin(TH / NT, kLdsBudget / (16 * NB * L)) : 1;
    static constexpr int THREADS = W * NT;
    // offset of the second exchange buffer (elements)
    static constexpr int B1OFF = NB == 2 ? W * L : 0;
};

// Register FFT of one line whose twiddles are fetched up front, with the data,
// where they fit in registers (at most 16 per thread); otherwise each stage
// reads them from the table.
template <int L, class G, int SIGN, bool ALLOW = true>
struct LineFft {
    static constexpr int NTW = tw_count<L, G::NTMAX, G::MAXR>();
    static constexpr bool PRE = ALLOW && NTW <= 16;
    double2 w[PRE ? NTW : 1];
    __device__ __forceinline__ void load(int t, const double2* __restrict__ tw) {
        if constexpr (PRE) load_twiddles<L, G::NTMAX, SIGN, 0, G::MAXR>(w, t, tw);
    }
    __device__ __forceinline__ void run(double2* x, double2* b0, double2* b1, int ps, int t,
                                        const double2* __restrict__ tw) {
        if constexpr (PRE) reg_fft_pre<L, G::NTMAX, SIGN, G::NB, G::MAXR>(x, b0, b1, ps, t, w);
        else reg_fft<L, G::NTMAX, SIGN, G::NB, G::MAXR>(x, b0, b1, ps, t, tw);
    }
};

// ---------------------------------------------------------------------------
// contiguous lines
// ---------------------------------------------------------------------------
template <int L, class G>
__global__ void __launch_bounds__(G::THREADS) kr_lines_r2c(const double* __restrict__ in, double2* __restrict__ out,
                                                         int nlines, const double2* __restrict__ tw, double scale) {
    extern __shared__ double2 lds[];
    const int t = threadIdx.x % G::NT, g = threadIdx.x / G::NT;
    double2* b0 = lds + g * L;
    double2* b1 = lds + G::B1OFF + g * L;
    const long l0 = ((long)blockIdx.x * G::W + g) * 2;
    double2 x[G::E];
#pragma unroll
    for (int e = 0; e < G::E; ++e) {
        const int v = t + G::NT * e;
        // the physical input is read once per transform: non-temporal, so it does not
        // displace the spectral arrays the following passes read back from the MALL
        double re = l0 < nlines ? __builtin_nontemporal_load(&in[l0 * L + v]) : 0.0;
        double im = l0 + 1 < nlines ? __builtin_nontemporal_load(&in[(l0 + 1) * L + v]) : 0.0;
        x[e] = make_double2(re, im);
    }
    LineFft<L, G, -1> fft;
    fft.load(t, tw);
    fft.run(x, b0, b1, 1, t, tw);
    // Split the two real lines: X1_k = (Z_k + conj Z_{L-k}) / 2, X2_k = (Z_k - conj Z_{L-k}) / 2i.
    constexpr int Lh = L / 2 + 1;
    if constexpr (64 % G::NT == 0) {
        // Z_{L-k} for k = t + NT e sits in thread (NT - t) mod NT of the same line (own
        // index E - 1 - e, or E - e for t = 0), inside the same wave: lane shuffles.
        const int lane = threadIdx.x & 63;
        const int src = lane - t + (G::NT - t) % G::NT;
#pragma unroll
        for (int e = 0; e <= G::E / 2; ++e) {
            const double2 v = x[G::E - 1 - e];
            double2 zr = make_double2(__shfl(v.x, src), __shfl(v.y, src));
            if (t == 0) zr = x[(G::E - e) % G::E];
            zr = cconj(zr);
            const int k = t + G::NT * e;
            if (k < Lh) {
                const double2 z = x[e];
                double2 x1 = make_double2(0.5 * scale * (z.x + zr.x), 0.5 * scale * (z.y + zr.y));
                double2 d = csub(z, zr);
                double2 x2 = make_double2(0.5 * scale * d.y, -0.5 * scale * d.x);
                if (l0 < nlines) out[l0 * Lh + k] = x1;
                if (l0 + 1 < nlines) out[(l0 + 1) * Lh + k] = x2;
            }
        }
    } else {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < G::E; ++e) b0[t + G::NT * e] = x[e];
        __syncthreads();
        for (int k = t; k < Lh; k += G::NT) {
            double2 z = b0[k];
            double2 zr = cconj(b0[k == 0 ? 0 : L - k]);
            double2 x1 = make_double2(0.5 * scale * (z.x + zr.x), 0.5 * scale * (z.y + zr.y));
            double2 d = csub(z, zr);
            double2 x2 = make_double2(0.5 * scale * d.y, -0.5 * scale * d.x);
            if (l0 < nlines) out[l0 * Lh + k] = x1;
            if (l0 + 1 < nlines) out[(l0 + 1) * Lh + k] = x2;
        }
    }
}

template <int L, class G>
__global__ void __launch_bounds__(G::THREADS) kr_lines_c2r(const double2* __restrict__ in, double* __restrict__ out,
                                                         int nlines, const double2* __restrict__ tw) {
    extern __shared__ double2 lds[];
    const int t = threadIdx.x % G::NT, g = threadIdx.x / G::NT;
    double2* b0 = lds + g * L;
    double2* b1 = lds + G::B1OFF + g * L;
    const long l0 = ((long)xcd_block() * G::W + g) * 2;
    constexpr int Lh = L / 2 + 1;
    double2 x[G::E];
#pragma unroll
    for (int e = 0; e < G::E; ++e) {
        const int v = t + G::NT * e;
        const int k = v <= L / 2 ? v : L - v;
        double2 x1 = l0 < nlines ? in[l0 * Lh + k] : make_double2(0.0, 0.0);
        double2 x2 = l0 + 1 < nlines ? in[(l0 + 1) * Lh + k] : make_double2(0.0, 0.0);
        if (v == 0 || 2 * v == L) { x1.y = 0.0; x2.y = 0.0; }
        if (v > L / 2) { x1.y = -x1.y; x2.y = -x2.y; }
        x[e] = make_double2(x1.x - x2.y, x1.y + x2.x);
    }
    LineFft<L, G, 1> fft;
    fft.load(t, tw);
    fft.run(x, b0, b1, 1, t, tw);
#pragma unroll
    for (int e = 0; e < G::E; ++e) {
        const int v = t + G::NT * e;
        // physical output: written once, non-temporal like the forward pass's input
        if (l0 < nlines) __builtin_nontemporal_store(x[e].x, &out[l0 * L + v]);
        if (l0 + 1 < nlines) __builtin_nontemporal_store(x[e].y, &out[(l0 + 1) * L + v]);
    }
}

template <int L, class G, int SIGN>
__global__ void __launch_bounds__(G::THREADS) kr_lines_c2c(const double2* __restrict__ in, double2* __restrict__ out,
                                                         int nlines, const double2* __restrict__ tw, double scale) {
    extern __shared__ double2 lds[];
    const int t = threadIdx.x % G::NT, g = threadIdx.x / G::NT;
    double2* b0 = lds + g * L;
    double2* b1 = lds + G::B1OFF + g * L;
    const long ln = (long)xcd_block() * G::W + g;
    double2 x[G::E];
#pragma unroll
    for (int e = 0; e < G::E; ++e) x[e] = ln < nlines ? in[ln * L + t + G::NT * e] : make_double2(0.0, 0.0);
    LineFft<L, G, SIGN> fft;
    fft.load(t, tw);
    fft.run(x, b0, b1, 1, t, tw);
    if (ln < nlines) {
#pragma unroll
        for (int e = 0; e < G::E; ++e) out[ln * L + t + G::NT * e] = cscale(x[e], scale);
    }
}

// ---------------------------------------------------------------------------
// strided lines: data[o][e][c]
// ---------------------------------------------------------------------------
// Raw buffer access: a lane whose byte offset is kOob reads zeros and its store
// is dropped by the hardware range check, so predicated accesses need no
// branches and the compiler can count outstanding memory operations exactly.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kOob = 0x7fffffff;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)kBufRange, 0x00020000);
}
__device__ __forceinline__ double2 buf_ld(__amdgpu_buffer_rsrc_t r, int off) {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    double2 d;
    __builtin_memcpy(&d, &v, 16);
    return d;
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, int off, double2 d) {
    u32x4 v;
    __builtin_memcpy(&v, &d, 16);
    __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, 0);
}

// Persistent pass over tiles of W consecutive columns of the flattened
// (outer, inner) column index, so no tile is ragged except the very last one
// (a tile may straddle two slabs; each lane addresses its own slab).  With the
// grid a multiple of 8, XCD k walks tiles [k n / 8, (k + 1) n / 8), its blocks
// interleaved; otherwise the blocks stride over all tiles.  The next tile's
// loads are in flight during this tile's FFT.  The launch helper checks that
// every byte offset from a tile's first slab stays below kBufRange.
template <int L, class G, int SIGN>
__global__ void __launch_bounds__(G::THREADS) kr_strided(const double2* in, double2* out, int outer, int inner,
                                                         const double2* __restrict__ tw, double scale) {
    extern __shared__ double2 lds[];
    const int c = threadIdx.x % G::W, t = threadIdx.x / G::W;
    const long ncol = (long)outer * inner;
    const int ntiles = (int)((ncol + G::W - 1) / G::W);
    int nx, hi, b;
    if ((gridDim.x & 7) == 0) {
        const int xi = (int)(blockIdx.x & 7);
        nx = (int)(gridDim.x >> 3);
        hi = (int)((long)ntiles * (xi + 1) / 8);
        b = (int)((long)ntiles * xi / 8) + (int)(blockIdx.x >> 3);
    } else {
        nx = (int)gridDim.x;
        hi = ntiles;
        b = (int)blockIdx.x;
    }
    // twiddles from LDS: their reads do not queue behind the prefetch
    double2* twl = lds + G::NB * G::W * L;
    for (int i = threadIdx.x; i < L; i += G::THREADS) twl[i] = tw[i];
    __syncthreads();
    const int rs = inner * 16;
    // first slab of a tile (block-uniform) and this lane's column offset from it
    auto slab0 = [&](int bb) { return bb < hi ? (int)((long)bb * G::W / inner) : 0; };
    auto lane_off = [&](int bb, int o0) {
        const long g = (long)bb * G::W + c;
        if (bb >= hi || g >= ncol) return kOob;
        const int o = (int)(g / inner);
        return ((o - o0) * L * inner + (int)(g - (long)o * inner)) * 16;
    };
    double2 x[G::E], y[G::E];
    int o0 = slab0(b);
    int off = lane_off(b, o0);
    {
        const auto r = buf_rsrc(in + (long)o0 * L * inner);
#pragma unroll
        for (int e = 0; e < G::E; ++e) x[e] = buf_ld(r, off == kOob ? kOob : off + (t + G::NT * e) * rs);
    }
    while (b < hi) {
        const int bn = b + nx;
        const int o0n = slab0(bn);
        const int offn = lane_off(bn, o0n);
        {
            const auto r = buf_rsrc(in + (long)o0n * L * inner);
#pragma unroll
            for (int e = 0; e < G::E; ++e) y[e] = buf_ld(r, offn == kOob ? kOob : offn + (t + G::NT * e) * rs);
        }
        reg_fft<L, G::NTMAX, SIGN, G::NB, G::MAXR>(x, lds + c, lds + G::B1OFF + c, G::W, t, twl);
        {
            const auto r = buf_rsrc(out + (long)o0 * L * inner);
#pragma unroll
            for (int e = 0; e < G::E; ++e)
                buf_st(r, off == kOob ? kOob : off + (t + G::NT * e) * rs, cscale(x[e], scale));
        }
        __syncthreads();  // every exchange read done before the next tile's first write
#pragma unroll
        for (int e = 0; e < G::E; ++e) x[e] = y[e];
        off = offn;
        o0 = o0n;
        b = bn;
    }
}

// ---------------------------------------------------------------------------
// Chebyshev axis, forward (DCT-II + scalar product / projection)
// ---------------------------------------------------------------------------
// Waves per SIMD when a group's LDS (bytes) is the occupancy limit (160 KB per
// CU, four SIMDs): with at most two, a thread has 256 VGPRs and the
// per-position tables of E = 16 lines fit in registers too.
template <class G>
constexpr int lds_waves_per_simd(long lds_bytes) {
    return (int)((163840 / lds_bytes) * (G::THREADS / 64) / 4);
}
template <class G>
constexpr bool table_regs(long lds_bytes) {
    return G::E <= 8 || (G::E <= 16 && lds_waves_per_simd<G>(lds_bytes) <= 2);
}

constexpr bool kChebTwRegs = false;  // Chebyshev kernels: twiddles from the table (registers go to the tables)

__device__ __forceinline__ int makhoul_row(int v, int N) { return v < (N + 1) / 2 ? 2 * v : 2 * (N - 1 - v) + 1; }

// Sequential per-(column, parity) least-squares projection used for the
// biharmonic basis: boundary-functional projection then Givens + banded R.
__device__ void project_givens_lane(double2* col, int es, int n, int m, int nrot, const double* rot,
                                    const double* rt, const double* qt) {
    double2 s1 = make_double2(0.0, 0.0), s2 = make_double2(0.0, 0.0);
    for (int t = 0; t < m; ++t) {
        double2 v = col[t * es];
        double q1 = qt[2 * t], q2 = qt[2 * t + 1];
        s1.x += q1 * v.x; s1.y += q1 * v.y;
        s2.x += q2 * v.x; s2.y += q2 * v.y;
    }
    auto ld = [&](int t) {
        if (t >= m) return make_double2(0.0, 0.0);
        double2 v = col[t * es];
        double q1 = qt[2 * t], q2 = qt[2 * t + 1];
        return make_double2(v.x - q1 * s1.x - q2 * s2.x, v.y - q1 * s1.y - q2 * s2.y);
    };
    double2 w0 = ld(0), w1 = ld(1);
    double2 w2 = nrot == 2 ? ld(2) : make_double2(0.0, 0.0);
    for (int i = 0; i < n; ++i) {
        double c1 = rot[4 * i], s1r = rot[4 * i + 1];
        double2 a = w0, b = w1;
        w0 = make_double2(c1 * a.x + s1r * b.x, c1 * a.y + s1r * b.y);
        w1 = make_double2(-s1r * a.x + c1 * b.x, -s1r * a.y + c1 * b.y);
        if (nrot == 2) {
            double c2 = rot[4 * i + 2], s2r = rot[4 * i + 3];
            a = w0; b = w2;
            w0 = make_double2(c2 * a.x + s2r * b.x, c2 * a.y + s2r * b.y);
            w2 = make_double2(-s2r * a.x + c2 * b.x, -s2r * a.y + c2 * b.y);
            col[i * es] = w0;
            w0 = w1; w1 = w2;
            w2 = ld(i + 3);
        } else {
            col[i * es] = w0;
            w0 = w1;
            w1 = ld(i + 2);
        }
    }
    double2 x1 = make_double2(0.0, 0.0), x2 = make_double2(0.0, 0.0);
    for (int i = n - 1; i >= 0; --i) {
        double r0 = rt[3 * i], r1 = rt[3 * i + 1], r2 = rt[3 * i + 2];
        double2 z = col[i * es];
        double2 x = make_double2((z.x - r1 * x1.x - r2 * x2.x) * r0, (z.y - r1 * x1.y - r2 * x2.y) * r0);
        col[i * es] = x;
        x2 = x1; x1 = x;
    }
}

// The same projection with every (column, parity) chain cut into segments of
// R rows, one thread each (2 W nseg <= block threads).  The boundary-functional
// projection is two reductions; the Givens sweep and the banded back
// substitution are linear recurrences with a two-value state whose segment
// maps are plan constants, so each thread runs its segment from a zero state,
// the entering states follow from a short scan over the chain's segments, and
// the rows are corrected with the per-row state coefficients.  SC holds two
// complex values per segment.  Every thread of the block reaches the barriers.
__device__ void project_segmented(double2* B0, double2* SC, int W, int nseg, const ChebDev& cd) {
    constexpr int R = kProjSegRowsDev;
    const int task = threadIdx.x;
    const int ntask = 2 * W * nseg;
    const bool on = task < ntask;
    // chain-fastest: the threads of a wave take 2 W adjacent chains (one LDS row
    // segment per row step) for a few segments, not one chain's segments, whose rows
    // lie 16 rows apart and would hit the same LDS banks; task = u 2W + ch
    const int u = on ? task / (2 * W) : 0, ch = on ? task % (2 * W) : 0;
    const int p = ch / W, cc = ch - p * W;
    const int es = 2 * W;
    double2* col = B0 + p * W + cc;
    const int n = cd.npar[p], m = cd.mpar[p];
    const int nsp = (n + R - 1) / R;
    const bool seg_on = on && u < nsp;
    const int lo = u * R, hi = min(lo + R, n);
    const int t0 = lo, t1 = u == nsp - 1 ? m : min(lo + R, m);
    const double* qt = cd.qtab[p];
    // SC segment-major: slot (v, ch) at 2 (v 2W + ch), so the 2 W chains of one
    // segment are adjacent in the scans below
    double2* sc = SC + 2 * task;
    double2* chain_sc = SC + 2 * ch;
    const int vs = 4 * W;  // stride between a chain's segment slots
    // 1. projection onto the null space of the boundary functionals
    double2 s1 = make_double2(0.0, 0.0), s2 = make_double2(0.0, 0.0);
    if (seg_on)
        for (int tt = t0; tt < t1; ++tt) {
            const double2 v = col[tt * es];
            const double q1 = qt[2 * tt], q2 = qt[2 * tt + 1];
            s1.x += q1 * v.x; s1.y += q1 * v.y;
            s2.x += q2 * v.x; s2.y += q2 * v.y;
        }
    if (on) { sc[0] = s1; sc[1] = s2; }
    __syncthreads();
    s1 = make_double2(0.0, 0.0);
    s2 = make_double2(0.0, 0.0);
    if (on)
        for (int v = 0; v < nsp; ++v) {
            const double2 a = chain_sc[vs * v], b = chain_sc[vs * v + 1];
            s1.x += a.x; s1.y += a.y;
            s2.x += b.x; s2.y += b.y;
        }
    __syncthreads();
    if (seg_on)
        for (int tt = t0; tt < t1; ++tt) {
            const double2 v = col[tt * es];
            const double q1 = qt[2 * tt], q2 = qt[2 * tt + 1];
            col[tt * es] = make_double2(v.x - q1 * s1.x - q2 * s2.x, v.y - q1 * s1.y - q2 * s2.y);
        }
    __syncthreads();
    // 2. Givens sweep from a zero entering state; fresh input of row i is ld(i + 2)
    double2 fr[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int tt = lo + r + 2;
        fr[r] = (seg_on && lo + r < hi && tt < m) ? col[tt * es] : make_double2(0.0, 0.0);
    }
    const double2 ld0 = on ? col[0] : make_double2(0.0, 0.0), ld1 = on ? col[es] : make_double2(0.0, 0.0);
    __syncthreads();
    const double* ro = cd.rot[p];
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = lo + r;
        if (seg_on && i < hi) {
            const double c1 = ro[4 * i], sn1 = ro[4 * i + 1], c2 = ro[4 * i + 2], sn2 = ro[4 * i + 3];
            const double2 a1 = make_double2(c1 * a.x + sn1 * b.x, c1 * a.y + sn1 * b.y);
            const double2 b1 = make_double2(-sn1 * a.x + c1 * b.x, -sn1 * a.y + c1 * b.y);
            const double2 f = fr[r];
            col[i * es] = make_double2(c2 * a1.x + sn2 * f.x, c2 * a1.y + sn2 * f.y);
            a = b1;
            b = make_double2(-sn2 * a1.x + c2 * f.x, -sn2 * a1.y + c2 * f.y);
        }
    }
    if (on) { sc[0] = a; sc[1] = b; }
    __syncthreads();
    // 3. entering state of the segment: rows 0, 1 of the projected column, then
    //    the maps and zero-state outputs of the segments above
    {
        double2 sa = ld0, sb = ld1;
        const double* gm = cd.gmat[p];
        if (seg_on)
            for (int v = 0; v < u; ++v) {
                const double2 ha = chain_sc[vs * v], hb = chain_sc[vs * v + 1];
                const double m00 = gm[4 * v], m01 = gm[4 * v + 1], m10 = gm[4 * v + 2], m11 = gm[4 * v + 3];
                const double2 na = make_double2(m00 * sa.x + m01 * sb.x + ha.x, m00 * sa.y + m01 * sb.y + ha.y);
                const double2 nb = make_double2(m10 * sa.x + m11 * sb.x + hb.x, m10 * sa.y + m11 * sb.y + hb.y);
                sa = na;
                sb = nb;
            }
        const double* ga = cd.gal[p];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = lo + r;
            if (seg_on && i < hi) {
                const double g0 = ga[2 * i], g1 = ga[2 * i + 1];
                const double2 v = col[i * es];
                col[i * es] = make_double2(v.x + g0 * sa.x + g1 * sb.x, v.y + g0 * sa.y + g1 * sb.y);
            }
        }
    }
    __syncthreads();
    // 4. banded back substitution x_i = (z_i - R_i,i+1 x_i+1 - R_i,i+2 x_i+2) / R_ii from a
    //    zero state below the segment
    const double* rt = cd.rtab[p];
    double2 x1 = make_double2(0.0, 0.0), x2 = make_double2(0.0, 0.0);
#pragma unroll
    for (int r = R - 1; r >= 0; --r) {
        const int i = lo + r;
        if (seg_on && i < hi) {
            const double r0 = rt[3 * i], r1 = rt[3 * i + 1], r2 = rt[3 * i + 2];
            const double2 z = col[i * es];
            const double2 xv = make_double2((z.x - r1 * x1.x - r2 * x2.x) * r0, (z.y - r1 * x1.y - r2 * x2.y) * r0);
            col[i * es] = xv;
            x2 = x1;
            x1 = xv;
        }
    }
    if (on) { sc[0] = x1; sc[1] = x2; }
    __syncthreads();
    // 5. entering state (x_hi, x_hi+1) from the segments below, then the correction
    {
        double2 sa = make_double2(0.0, 0.0), sb = make_double2(0.0, 0.0);
        const double* bm = cd.bmat[p];
        if (seg_on)
            for (int v = nsp - 1; v > u; --v) {
                const double2 ga = chain_sc[vs * v], gb = chain_sc[vs * v + 1];
                const double m00 = bm[4 * v], m01 = bm[4 * v + 1], m10 = bm[4 * v + 2], m11 = bm[4 * v + 3];
                const double2 na = make_double2(m00 * sa.x + m01 * sb.x + ga.x, m00 * sa.y + m01 * sb.y + ga.y);
                const double2 nb = make_double2(m10 * sa.x + m11 * sb.x + gb.x, m10 * sa.y + m11 * sb.y + gb.y);
                sa = na;
                sb = nb;
            }
        const double* ba = cd.bal[p];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = lo + r;
            if (seg_on && i < hi) {
                const double b0 = ba[2 * i], b1 = ba[2 * i + 1];
                const double2 v = col[i * es];
                col[i * es] = make_double2(v.x + b0 * sa.x + b1 * sb.x, v.y + b0 * sa.y + b1 * sb.y);
            }
        }
    }
}

// Right-hand side rows of the segmented solve from the block's LDS tile
// (columns c0 .. c0 + W - 1, row l at B0[l W + col - c0]).
struct TileRhs {
    const double2* B0;
    int W, c0;
    __device__ __forceinline__ double2 operator()(int p, int i, int col) const { return B0[(p + 2 * i) * W + col - c0]; }
};

// Per-position tables of the backward Chebyshev pass (theta_k, beta_{k-2},
// gamma_{k-4} for own k = t + NT e), in registers where they fit.
template <int N, class G>
struct BwdTables {
    static constexpr bool PRE = table_regs<G>(16L * G::NB * N * G::W);
    double2 th[PRE ? G::E : 1];
    double bb[PRE ? G::E : 1], gg[PRE ? G::E : 1];
    __device__ __forceinline__ void load(const ChebDev& cd, int t) {
        if constexpr (PRE) {
            const bool has_gamma = cd.basis == SGM_SHEN_BIHARMONIC;
            const bool has_beta = cd.basis != SGM_CHEBYSHEV;
#pragma unroll
            for (int e = 0; e < G::E; ++e) {
                const int k = t + G::NT * e;
                th[e] = cd.theta[k];
                bb[e] = (has_beta && k >= 2) ? cd.beta[k - 2] : 0.0;
                gg[e] = (has_gamma && k >= 4) ? cd.gamma[k - 4] : 0.0;
            }
        }
    }
    __device__ __forceinline__ double2 theta(const ChebDev& cd, int e, int k) const {
        if constexpr (PRE) return th[e];
        else return cd.theta[k];
    }
    __device__ __forceinline__ double beta(const ChebDev& cd, int e, int k) const {
        if constexpr (PRE) return bb[e];
        else return cd.beta[k - 2];
    }
    __device__ __forceinline__ double gamma(const ChebDev& cd, int e, int k) const {
        if constexpr (PRE) return gg[e];
        else return cd.gamma[k - 4];
    }
};

// Backward along x of one column tile: x holds the own coefficients u_hat_l
// (l = t + NT e, zero for l >= nb) and B0 the whole tile, written before the
// last barrier.  Recombination to Chebyshev coefficients, DCT-III (one complex
// FFT), then the Makhoul-ordered store of the physical x values to out.
template <int N, class G, class TB>
__device__ __forceinline__ void cheb_bwd_tile(double2 (&x)[G::E], double2* B0, double2* B1, int c, int t, int c0,
                                              bool ok, int ncols, double2* out, const ChebDev& cd, const TB& tb,
                                              const double2* __restrict__ tw) {
    constexpr int W = G::W, NT = G::NT, E = G::E;
    const bool has_gamma = cd.basis == SGM_SHEN_BIHARMONIC;
    const bool has_beta = cd.basis != SGM_CHEBYSHEV;
    // Chebyshev coefficients c_k = u_k + beta_{k-2} u_{k-2} + gamma_{k-4} u_{k-4} (own k)
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + NT * e;
        double2 v = x[e];
        if (has_beta && k >= 2) {
            const double bb = tb.beta(cd, e, k);
            double2 u = B0[(k - 2) * W + c];
            v.x += bb * u.x; v.y += bb * u.y;
        }
        if (has_gamma && k >= 4) {
            const double gg = tb.gamma(cd, e, k);
            double2 u = B0[(k - 4) * W + c];
            v.x += gg * u.x; v.y += gg * u.y;
        }
        x[e] = v;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) B0[(t + NT * e) * W + c] = x[e];
    __syncthreads();
    // DCT-III input W_0 = 2 c_0, W_k = e^{i pi k/(2N)} (c_k - i c_{N-k})
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + NT * e;
        const double2 ck = x[e];
        if (k == 0) {
            x[e] = make_double2(2.0 * ck.x, 2.0 * ck.y);
        } else {
            const double2 cn = B0[(N - k) * W + c];
            const double2 d = make_double2(ck.x + cn.y, ck.y - cn.x);
            x[e] = cmul(cconj(tb.theta(cd, e, k)), d);
        }
    }
    __syncthreads();
    LineFft<N, G, 1, kChebTwRegs> fft;
    fft.load(t, tw);
    fft.run(x, B0 + c, B1 + c, W, t, tw);
    if (ok) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int v = t + NT * e;
            out[(long)makhoul_row(v, N) * ncols + c0 + c] = cscale(x[e], 0.5);
        }
    }
}

template <int N, class G, int MODE>
__global__ void __launch_bounds__(G::THREADS) kr_cheb_fwd(const double2* in, double2* out, ChebDev cd, int ncols,
                                                        const double2* __restrict__ tw, ChebSolve sv) {
    constexpr int W = G::W, NT = G::NT, E = G::E;
    extern __shared__ double2 lds[];
    // one N x W tile (B0), a second one only as the FFT's other exchange buffer,
    // then 2 NT x W scratch entries for the reductions
    double2* B0 = lds;
    double2* B1 = lds + G::B1OFF;
    double2* SC = lds + G::NB * N * W;
    const int c = threadIdx.x % W, t = threadIdx.x / W;
    const int c0 = xcd_block() * W;
    const bool ok = c0 + c < ncols;
    double2 x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int v = t + NT * e;
        x[e] = ok ? in[(long)makhoul_row(v, N) * ncols + c0 + c] : make_double2(0.0, 0.0);
    }
    // per-position table entries fetched with the data (short lines only: registers),
    // so their latency is not paid again after the FFT
    constexpr bool kSP = MODE == kScalarProduct || MODE == kScalarSolve;
    constexpr bool kPre = kSP ? E <= 8 : table_regs<G>(16L * (G::NB * N * W + 2 * NT * W));
    double2 thk[kPre ? E : 1];
    double fsk[kPre ? E : 1], gsk[kPre && kSP ? E : 1];
    if constexpr (kPre) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + NT * e;
            thk[e] = cd.theta[k];
            if constexpr (MODE == kProjCheb || MODE == kProjDirichlet) fsk[e] = cd.fscale[k];
            if constexpr (MODE == kProjBiharmonic) fsk[e] = cd.bscale[k];
            if constexpr (kSP) {
                fsk[e] = (k < cd.nb && k + 2 < N) ? cd.beta[k] : 0.0;
                gsk[e] = (k < cd.nb && k + 4 < N) ? cd.gamma[k] : 0.0;
            }
        }
    }
    LineFft<N, G, -1, kChebTwRegs> fft;
    fft.load(t, tw);
    fft.run(x, B0 + c, B1 + c, W, t, tw);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) B0[(t + NT * e) * W + c] = x[e];
    __syncthreads();
    // DCT-II post-processing: C_k for own k from V_k and V_{N-k}
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int k = t + NT * e;
        const int kn = k == 0 ? 0 : N - k;
        double2 V = x[e];
        double2 cv = cconj(B0[kn * W + c]);
        double2 a = make_double2(0.5 * (V.x + cv.x), 0.5 * (V.y + cv.y));
        double2 d = csub(V, cv);
        double2 b = make_double2(0.5 * d.y, -0.5 * d.x);
        double2 tk;
        if constexpr (kPre) tk = thk[e];
        else tk = cd.theta[k];
        x[e] = make_double2(tk.x * a.x - tk.y * a.y, tk.x * b.x - tk.y * b.y);  // C_k
    }
    __syncthreads();  // every V read before B0 is reused
    const int nb = cd.nb;
    if constexpr (kSP) {
#pragma unroll
        for (int e = 0; e < E; ++e) B0[(t + NT * e) * W + c] = x[e];
        __syncthreads();
        const double s = M_PI / N;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int l = t + NT * e;
            double2 v = make_double2(0.0, 0.0);
            if (l < nb) {
                v = x[e];
                double bb = 0.0, gg = 0.0;
                if constexpr (kPre) { bb = fsk[e]; gg = gsk[e]; }
                else { bb = l + 2 < N ? cd.beta[l] : 0.0; gg = l + 4 < N ? cd.gamma[l] : 0.0; }
                if (l + 2 < N) { double2 u = B0[(l + 2) * W + c]; v.x += bb * u.x; v.y += bb * u.y; }
                if (l + 4 < N) { double2 u = B0[(l + 4) * W + c]; v.x += gg * u.x; v.y += gg * u.y; }
                v = cscale(v, s);
            }
            if constexpr (MODE == kScalarProduct) {
                if (ok) out[(long)l * ncols + c0 + c] = v;
            } else {
                x[e] = v;
            }
        }
        if constexpr (MODE == kScalarSolve) {
            // f~ of the tile into LDS, then the Dirichlet Helmholtz solve of its chains:
            // wave p (0, 1) takes parity p of the W = 8 columns, 8 lanes of 16 rows per chain
            static_assert(W == 8 && G::THREADS >= 128, "fused solve needs 8-column tiles");
            __syncthreads();
#pragma unroll
            for (int e = 0; e < E; ++e) B0[(t + NT * e) * W + c] = x[e];
            __syncthreads();
            const int wv = threadIdx.x >> 6;
            if (wv < 2)
                segdev::solve_wave<SGM_SHEN_DIRICHLET, 8, kSegRows>(wv * ((ncols + W - 1) / W) + c0 / W,
                                                                   TileRhs{B0, W, c0}, segdev::GlobalOut{out, ncols},
                                                                   sv.tab, cd, sv.g, sv.alpha, cd.solve[0],
                                                                   cd.solve[1]);
        }
    } else if constexpr (MODE == kProjCheb) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + NT * e;
            double f;
            if constexpr (kPre) f = fsk[e];
            else f = cd.fscale[k];
            if (ok) out[(long)k * ncols + c0 + c] = cscale(x[e], f);
        }
    } else if constexpr (MODE == kProjDirichlet) {
        // c_k = fscale_k C_k; per parity p: lambda_p = (sum_k c_k) / (sum_k w_k) with w_0 = 1/2
        // and w_k = 1 otherwise; u_l = sum_{k <= l, k = l mod 2} (c_k - lambda_p w_k).  Along a
        // parity chain (chain index i <-> position p + 2i) the w prefix is i + 1 - [p = 0]/2, so
        // one segmented prefix sum of c yields both the chain total and every u_l.  NT is even:
        // all own positions of thread t have parity t & 1.
#pragma unroll
        for (int e = 0; e < E; ++e) {
            double f;
            if constexpr (kPre) f = fsk[e];
            else f = cd.fscale[t + NT * e];
            B0[(t + NT * e) * W + c] = cscale(x[e], f);
        }
        __syncthreads();
        // the NT/2 threads of parity p own consecutive chain segments of length seg
        const int p = t & 1, t2 = t >> 1;
        const int mp = (N - p + 1) / 2;
        constexpr int SEG = ((N + 1) / 2 + NT / 2 - 1) / (NT / 2);
        const int seg = (mp + NT / 2 - 1) / (NT / 2);
        const int i0 = t2 * seg;
        double2 pre[SEG];
        double2 run = make_double2(0.0, 0.0);
#pragma unroll
        for (int r = 0; r < SEG; ++r) {
            const int i = i0 + r;
            if (r < seg && i < mp) {
                const double2 v = B0[(p + 2 * i) * W + c];
                run.x += v.x; run.y += v.y;
            }
            pre[r] = run;
        }
        SC[t * W + c] = run;
        __syncthreads();
        double2 below = make_double2(0.0, 0.0), tot = make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < NT / 2; ++u) {
            const double2 v = SC[(2 * u + p) * W + c];
            if (u < t2) { below.x += v.x; below.y += v.y; }
            tot.x += v.x; tot.y += v.y;
        }
        const double w0 = p == 0 ? 0.5 : 0.0;
        const double wsum = (double)mp - w0;
        const double2 lam = make_double2(tot.x / wsum, tot.y / wsum);
#pragma unroll
        for (int r = 0; r < SEG; ++r) {
            const int i = i0 + r;
            if (r < seg && i < mp) {
                const int l = p + 2 * i;
                const double wp = (double)(i + 1) - w0;
                const double2 u = make_double2(below.x + pre[r].x - lam.x * wp, below.y + pre[r].y - lam.y * wp);
                if (ok) out[(long)l * ncols + c0 + c] = l < nb ? u : make_double2(0.0, 0.0);
            }
        }
    } else {  // kProjBiharmonic
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = t + NT * e;
            double f;
            if constexpr (kPre) f = fsk[e];
            else f = cd.bscale[k];
            B0[k * W + c] = cscale(x[e], f);
        }
        __syncthreads();
        constexpr int R = kProjSegRowsDev;
        const int nseg = (max(cd.npar[0], cd.npar[1]) + R - 1) / R;
        if (2 * W * nseg <= G::THREADS && 2 * nseg <= NT) {
            project_segmented(B0, SC, W, nseg, cd);
        } else {
            const int lane = threadIdx.x;
            if (lane < 2 * W) {
                const int p = lane / W, cc = lane - p * W;
                project_givens_lane(B0 + p * W + cc, 2 * W, cd.npar[p], cd.mpar[p], 2, cd.rot[p], cd.rtab[p],
                                    cd.qtab[p]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int l = t + NT * e;
            if (ok) out[(long)l * ncols + c0 + c] = l < nb ? B0[l * W + c] : make_double2(0.0, 0.0);
        }
    }
}

// ---------------------------------------------------------------------------
// Chebyshev axis, backward (recombination + DCT-III)
// ---------------------------------------------------------------------------
template <int N, class G>
__global__ void __launch_bounds__(G::THREADS) kr_cheb_bwd(const double2* in, double2* out, ChebDev cd, int ncols,
                                                        const double2* __restrict__ tw) {
    constexpr int W = G::W, NT = G::NT, E = G::E;
    extern __shared__ double2 lds[];
    double2* B0 = lds;
    double2* B1 = lds + G::B1OFF;
    const int c = threadIdx.x % W, t = threadIdx.x / W;
    const int c0 = xcd_block() * W;
    const bool ok = c0 + c < ncols;
    const int nb = cd.nb;
    double2 x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int l = t + NT * e;
        x[e] = (ok && l < nb) ? in[(long)l * ncols + c0 + c] : make_double2(0.0, 0.0);
    }
    // table entries fetched with the data
    BwdTables<N, G> tb;
    tb.load(cd, t);
#pragma unroll
    for (int e = 0; e < E; ++e) B0[(t + NT * e) * W + c] = x[e];
    __syncthreads();
    cheb_bwd_tile<N, G>(x, B0, B1, c, t, c0, ok, ncols, out, cd, tb, tw);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <int L, class G>
static void fill_g(RegKernels& k) {
    k.L = L;
    k.W = G::W;
    k.threads = G::THREADS;
    k.lds = sizeof(double2) * (size_t)G::NB * G::W * L;
    k.lds_str = k.lds + sizeof(double2) * (size_t)L;
    k.lds_cheb = sizeof(double2) * ((size_t)G::NB * G::W * L + 2 * (size_t)G::NT * G::W);
    k.r2c = kr_lines_r2c<L, G>;
    k.c2r = kr_lines_c2r<L, G>;
    k.c2c_f = kr_lines_c2c<L, G, -1>;
    k.c2c_b = kr_lines_c2c<L, G, 1>;
    k.str_f = kr_strided<L, G, -1>;
    k.str_b = kr_strided<L, G, 1>;
    k.cf_sp = kr_cheb_fwd<L, G, kScalarProduct>;
    k.cf_cheb = kr_cheb_fwd<L, G, kProjCheb>;
    k.cf_dir = kr_cheb_fwd<L, G, kProjDirichlet>;
    k.cf_bih = kr_cheb_fwd<L, G, kProjBiharmonic>;
    if constexpr (L == 256 && G::W == 8 && G::THREADS == 256) k.cf_spsolve = kr_cheb_fwd<L, G, kScalarSolve>;
    else k.cf_spsolve = nullptr;
    k.cb = kr_cheb_bwd<L, G>;
}

// Variant v: 0 = (32 threads per line max, two buffers), 1 = (32, one buffer),
// 2 = (16, two buffers), 3 = (16, one buffer), 4 = (64, one buffer), 5 = (32,
// one buffer, 512-thread blocks: twice the lines per block, so the strided
// passes move 256-byte row segments), 6 = variant 1 and 7 = variant 3 with a
// radix-4/2 stage schedule instead of radix 8.  The hot lengths 128, 256, 512
// carry 0..3 and 5..7 (512 and 1024 also 4); the others have variant 0 only.
template <int L>
static bool fill_v(int v, RegKernels& k) {
    switch (v) {
        case 0: fill_g<L, Geo<L, 32, 2>>(k); return true;
        case 1: fill_g<L, Geo<L, 32, 1>>(k); return true;
        case 2: fill_g<L, Geo<L, 16, 2>>(k); return true;
        case 3: fill_g<L, Geo<L, 16, 1>>(k); return true;
        case 5: fill_g<L, Geo<L, 32, 1, 512>>(k); return true;
        case 6: fill_g<L, Geo<L, 32, 1, kThreads, 4>>(k); return true;
        case 7: fill_g<L, Geo<L, 16, 1, kThreads, 4>>(k); return true;
        default: return false;
    }
}
// Lengths whose 32-thread geometry needs E = 16: variant 4 = (64 threads per
// line, one buffer), half the lines and LDS per block.
template <int L>
static bool fill_v64(int v, RegKernels& k) {
    if (v == 4) { fill_g<L, Geo<L, 64, 1>>(k); return true; }
    return fill_v<L>(v, k);
}
template <int L>
static bool fill0(int v, RegKernels& k) {
    if (v != 0) return false;
    fill_g<L, Geo<L, 32, 2>>(k);
    return true;
}

bool reg_kernels_for(int L, RegKernels& k, int variant) {
    k.variant = variant;
    switch (L) {
        case 16: return fill0<16>(variant, k);
        case 32: return fill0<32>(variant, k);
        case 64: return fill0<64>(variant, k);
        case 128: return fill_v<128>(variant, k);
        case 256: return fill_v<256>(variant, k);
        case 512: return fill_v64<512>(variant, k);
        case 1024:
            if (variant == 4) { fill_g<1024, Geo<1024, 64, 1>>(k); return true; }
            return fill0<1024>(variant, k);
        case 48: return fill0<48>(variant, k);
        case 96: return fill0<96>(variant, k);
        case 192: return fill0<192>(variant, k);
        case 384: return fill0<384>(variant, k);
        case 768: return fill0<768>(variant, k);
        case 144: return fill0<144>(variant, k);
        case 288: return fill0<288>(variant, k);
        case 576: return fill0<576>(variant, k);
        default: return false;
    }
}

// Occupancy-sized grid of a persistent kernel, cached per (kernel, device).
static long resident_grid(const void* f, int threads, size_t lds) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, long> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 8;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find({f, dev});
    if (it != cache.end()) return it->second;
    int per = 0, cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, threads, lds) != hipSuccess || per < 1) per = 1;
    long g = (long)per * cus;
    g = g < 8 ? 8 : g - g % 8;
    cache[{f, dev}] = g;
    return g;
}

hipError_t launch_strided(const RegKernels& k, int sign, const double2* in, double2* out, int outer, int inner,
                          const double2* tw, double scale, hipStream_t s) {
    const long ncol = (long)outer * inner;
    if (ncol <= 0) return hipSuccess;
    if (!strided_fits(k, inner)) return hipErrorInvalidValue;
    auto f = sign < 0 ? k.str_f : k.str_b;
    const long tiles = (ncol + k.W - 1) / k.W;
    long grid = resident_grid(reinterpret_cast<const void*>(f), k.threads, k.lds_str);
    if (tiles < grid) grid = (tiles + 7) / 8 * 8;
    hipLaunchKernelGGL(f, dim3((unsigned)grid), dim3(k.threads), k.lds_str, s, in, out, outer, inner, tw, scale);
    return hipGetLastError();
}

}  // namespace sgm
