// Batched mixed-radix Stockham FFT on LDS (device code, header-only).
//
// A work-group holds `nlines` lines of length L in LDS; element e of line ln
// sits at buf[ln * ls + e * es].  Each stage of radix P computes L/P
// butterflies per line: inputs are read at stride L/P, multiplied by the
// twiddles exp(SIGN 2 pi i r k / (P m)) (k = i mod m, m = product of the
// earlier radices), transformed by a length-P DFT and written at
// j + r m with j = (i - k) P + k (self-sorting, natural order out).
// Stages ping-pong between two LDS buffers.  SIGN = -1 is the forward
// (e^{-i...}) direction, +1 the backward one; neither scales.
#pragma once
#include "common.h"

namespace sgm {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// Multiply by SIGN * i.
template <int SIGN>
__device__ __forceinline__ double2 mul_si(double2 a) {
    return SIGN < 0 ? make_double2(a.y, -a.x) : make_double2(-a.y, a.x);
}
// Table twiddle w = exp(-2 pi i r / L); the backward direction uses its conjugate.
template <int SIGN>
__device__ __forceinline__ double2 twiddle(const double2* tw, int r) {
    double2 w = tw[r];
    return SIGN < 0 ? w : cconj(w);
}

template <int P, int SIGN>
struct Dft;

template <int SIGN>
struct Dft<2, SIGN> {
    __device__ __forceinline__ static void run(double2* x) {
        double2 a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    }
};

template <int SIGN>
struct Dft<3, SIGN> {
    __device__ __forceinline__ static void run(double2* x) {
        const double h = 0.86602540378443864676;  // sqrt(3)/2
        double2 t = cadd(x[1], x[2]);
        double2 u = csub(x[1], x[2]);
        double2 m = make_double2(x[0].x - 0.5 * t.x, x[0].y - 0.5 * t.y);
        double2 v = mul_si<SIGN>(cscale(u, h));
        x[0] = cadd(x[0], t);
        x[1] = cadd(m, v);
        x[2] = csub(m, v);
    }
};

template <int SIGN>
struct Dft<4, SIGN> {
    __device__ __forceinline__ static void run(double2* x) {
        double2 a = cadd(x[0], x[2]);
        double2 b = csub(x[0], x[2]);
        double2 c = cadd(x[1], x[3]);
        double2 d = mul_si<SIGN>(csub(x[1], x[3]));
        x[0] = cadd(a, c);
        x[2] = csub(a, c);
        x[1] = cadd(b, d);
        x[3] = csub(b, d);
    }
};

template <int SIGN>
struct Dft<5, SIGN> {
    __device__ __forceinline__ static void run(double2* x) {
        const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;
        const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;
        double2 a1 = cadd(x[1], x[4]), a2 = cadd(x[2], x[3]);
        double2 b1 = csub(x[1], x[4]), b2 = csub(x[2], x[3]);
        double2 x0 = x[0];
        double2 p1 = make_double2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
        double2 p2 = make_double2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
        double2 q1 = mul_si<SIGN>(make_double2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
        double2 q2 = mul_si<SIGN>(make_double2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
        x[0] = cadd(x0, cadd(a1, a2));
        x[1] = cadd(p1, q1);
        x[4] = csub(p1, q1);
        x[2] = cadd(p2, q2);
        x[3] = csub(p2, q2);
    }
};

template <int SIGN>
struct Dft<7, SIGN> {
    __device__ __forceinline__ static void run(double2* x) {
        const double c[3] = {0.62348980185873353053, -0.22252093395631440429, -0.90096886790241912624};
        const double s[3] = {0.78183148246802980871, 0.97492791218182360702, 0.43388373911755812048};
        double2 a[3], b[3];
        for (int q = 0; q < 3; ++q) {
            a[q] = cadd(x[q + 1], x[6 - q]);
            b[q] = csub(x[q + 1], x[6 - q]);
        }
        double2 x0 = x[0];
        double2 y[7];
        y[0] = cadd(x0, cadd(a[0], cadd(a[1], a[2])));
        for (int q = 1; q <= 3; ++q) {
            double2 pr = x0, qi = make_double2(0.0, 0.0);
            for (int r = 1; r <= 3; ++r) {
                int e = (q * r) % 7;  // cos(2 pi e/7), sin(2 pi e/7) with e in 1..6
                double ce, se;
                if (e <= 3) { ce = c[e - 1]; se = s[e - 1]; }
                else { ce = c[7 - e - 1]; se = -s[7 - e - 1]; }
                pr.x += ce * a[r - 1].x; pr.y += ce * a[r - 1].y;
                qi.x += se * b[r - 1].x; qi.y += se * b[r - 1].y;
            }
            double2 v = mul_si<SIGN>(qi);
            y[q] = cadd(pr, v);
            y[7 - q] = csub(pr, v);
        }
        for (int q = 0; q < 7; ++q) x[q] = y[q];
    }
};

template <int SIGN>
struct Dft<8, SIGN> {
    __device__ __forceinline__ static void run(double2* x) {
        const double h = 0.70710678118654752440;
        double2 e[4] = {x[0], x[2], x[4], x[6]};
        double2 o[4] = {x[1], x[3], x[5], x[7]};
        Dft<4, SIGN>::run(e);
        Dft<4, SIGN>::run(o);
        // W8^q = exp(SIGN 2 pi i q / 8)
        double2 t1 = make_double2(h * (o[1].x - SIGN * o[1].y), h * (o[1].y + SIGN * o[1].x));
        double2 t2 = mul_si<SIGN>(o[2]);
        double2 t3 = make_double2(h * (-o[3].x - SIGN * o[3].y), h * (-o[3].y + SIGN * o[3].x));
        x[0] = cadd(e[0], o[0]);
        x[4] = csub(e[0], o[0]);
        x[1] = cadd(e[1], t1);
        x[5] = csub(e[1], t1);
        x[2] = cadd(e[2], t2);
        x[6] = csub(e[2], t2);
        x[3] = cadd(e[3], t3);
        x[7] = csub(e[3], t3);
    }
};

template <int P, int SIGN>
__device__ __forceinline__ void stage_bfly(const double2* __restrict__ src, double2* __restrict__ dst, int i,
                                           int Lp, int m, int L, int base, int es, const double2* tw) {
    int k = i % m;
    double2 x[P];
#pragma unroll
    for (int r = 0; r < P; ++r) x[r] = src[base + (i + r * Lp) * es];
    if (m > 1) {
        int step = k * (L / (P * m));
#pragma unroll
        for (int r = 1; r < P; ++r) x[r] = cmul(x[r], twiddle<SIGN>(tw, r * step));
    }
    Dft<P, SIGN>::run(x);
    int j = (i - k) * P + k;
#pragma unroll
    for (int r = 0; r < P; ++r) dst[base + (j + r * m) * es] = x[r];
}

// Radix-P stage for any P dividing L (naive length-P DFT, O(P^2)).
template <int SIGN>
__device__ void stage_generic(const double2* __restrict__ src, double2* __restrict__ dst, int i, int P, int Lp,
                              int m, int L, int base, int es, const double2* tw) {
    int k = i % m;
    int step = k * (L / (P * m));
    int j = (i - k) * P + k;
    for (int q = 0; q < P; ++q) {
        double2 acc = make_double2(0.0, 0.0);
        for (int r = 0; r < P; ++r) {
            double2 v = src[base + (i + r * Lp) * es];
            // total phase index: r*step (input twiddle) + (q*r mod P) * Lp (DFT kernel)
            int idx = (r * step + ((q * r) % P) * Lp) % L;
            double2 w = twiddle<SIGN>(tw, idx);
            acc = cadd(acc, cmul(v, w));
        }
        dst[base + (j + q * m) * es] = acc;
    }
}

// Transform `nlines` lines held in buffer `a` (scratch `b` of the same size).
// line_fastest: consecutive threads take consecutive lines (column-tile
// layout, es > 1) instead of consecutive butterflies of one line (row layout).
// Returns the buffer that holds the result.  Ends with a barrier.
template <int SIGN>
__device__ double2* lds_fft(double2* a, double2* b, const RadixPlan& rp, int nlines, int es, int ls,
                            bool line_fastest) {
    const int L = rp.L;
    int m = 1;
    double2* src = a;
    double2* dst = b;
    for (int s = 0; s < rp.nst; ++s) {
        const int P = rp.radix[s];
        const int Lp = L / P;
        const int total = nlines * Lp;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            int ln, i;
            if (line_fastest) { ln = t % nlines; i = t / nlines; }
            else { ln = t / Lp; i = t - ln * Lp; }
            const int base = ln * ls;
            switch (P) {
                case 2: stage_bfly<2, SIGN>(src, dst, i, Lp, m, L, base, es, rp.tw); break;
                case 3: stage_bfly<3, SIGN>(src, dst, i, Lp, m, L, base, es, rp.tw); break;
                case 4: stage_bfly<4, SIGN>(src, dst, i, Lp, m, L, base, es, rp.tw); break;
                case 5: stage_bfly<5, SIGN>(src, dst, i, Lp, m, L, base, es, rp.tw); break;
                case 7: stage_bfly<7, SIGN>(src, dst, i, Lp, m, L, base, es, rp.tw); break;
                case 8: stage_bfly<8, SIGN>(src, dst, i, Lp, m, L, base, es, rp.tw); break;
                default: stage_generic<SIGN>(src, dst, i, P, Lp, m, L, base, es, rp.tw); break;
            }
        }
        __syncthreads();
        double2* t = src;
        src = dst;
        dst = t;
        m *= P;
    }
    return src;
}

}  // namespace sgm
