// Register-resident mixed-radix Stockham FFT for compile-time lengths
// L = 2^a 3^b (device code, header-only).
//
// NT threads cooperate on one line; thread t owns the E = L/NT positions
// t + NT*e (e = 0..E-1).  Every radix p of the schedule divides E, so the
// inputs of a stage's butterflies i = t + NT*q (q < E/p), read at stride L/p,
// are the thread's own positions.  A stage's outputs land at j + r*m
// (j = (i - k) p + k, k = i mod m, m = product of the earlier radices); they
// are exchanged through LDS, except after the last stage, where m = L/p makes
// j + r*m = i + r*L/p an own position again.  So a line goes
// global -> registers -> (stage, LDS exchange)* -> stage -> registers -> global.
#pragma once
#include "fft_lds.h"

namespace sgm {

struct Sched {
    int L, E, NT, nst;
    int rad[16];
};

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }
constexpr int clcm(int a, int b) { return a / cgcd(a, b) * b; }

// Radix schedule: 3s first, then 8s (or 4s when MAXR = 4), with one 4 or 2 for the
// remaining power of two.  E = lcm(radices) * 2^j, the smallest such that
// NT = L/E <= NTMAX.
constexpr Sched make_sched(int L, int NTMAX, int MAXR = 8) {
    Sched s{};
    s.L = L;
    int a = 0, b = 0, r = L;
    while (r % 2 == 0) { r /= 2; ++a; }
    while (r % 3 == 0) { r /= 3; ++b; }
    if (r != 1) { s.nst = -1; return s; }
    int n = 0;
    for (int i = 0; i < b; ++i) s.rad[n++] = 3;
    if (MAXR >= 8) {
        int r8 = a / 3, rem = a % 3;
        if (rem == 1 && r8 > 0) { --r8; s.rad[n++] = 4; s.rad[n++] = 4; }
        else if (rem == 1) s.rad[n++] = 2;
        else if (rem == 2) s.rad[n++] = 4;
        for (int i = 0; i < r8; ++i) s.rad[n++] = 8;
    } else {
        for (int i = 0; i < a / 2; ++i) s.rad[n++] = 4;
        if (a % 2) s.rad[n++] = 2;
    }
    s.nst = n;
    int E = 1;
    for (int i = 0; i < n; ++i) E = clcm(E, s.rad[i]);
    while (L / E > NTMAX && L % (2 * E) == 0) E *= 2;
    s.E = E;
    s.NT = L / E;
    return s;
}

constexpr int sched_m(const Sched& s, int S) {
    int m = 1;
    for (int i = 0; i < S; ++i) m *= s.rad[i];
    return m;
}

// Twiddles a thread uses over the whole transform: stage S >= 1 needs p - 1
// per butterfly q (stage 0 has m = 1 and none).
template <int L, int NTMAX, int MAXR = 8>
constexpr int tw_count() {
    constexpr Sched sd = make_sched(L, NTMAX, MAXR);
    int n = 0;
    for (int S = 1; S < sd.nst; ++S) n += (sd.E / sd.rad[S]) * (sd.rad[S] - 1);
    return n;
}

// Fetch those twiddles into w (stage by stage, butterfly q, then r = 1..p-1),
// so a kernel can issue them together with its data loads.
template <int L, int NTMAX, int SIGN, int S = 0, int MAXR = 8>
__device__ __forceinline__ void load_twiddles(double2* w, int t, const double2* __restrict__ tw) {
    constexpr Sched sd = make_sched(L, NTMAX, MAXR);
    if constexpr (S < sd.nst) {
        constexpr int p = sd.rad[S];
        constexpr int m = sched_m(sd, S);
        constexpr int Q = sd.E / p;
        if constexpr (m > 1) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int k = (t + sd.NT * q) % m;
                const int step = k * (L / (p * m));
#pragma unroll
                for (int r = 1; r < p; ++r) w[q * (p - 1) + r - 1] = twiddle<SIGN>(tw, r * step);
            }
            load_twiddles<L, NTMAX, SIGN, S + 1, MAXR>(w + Q * (p - 1), t, tw);
        } else {
            load_twiddles<L, NTMAX, SIGN, S + 1, MAXR>(w, t, tw);
        }
    }
}

// Exchange buffer addressing for one line: position v lives at base[v * ps].
// Stages alternate between two buffers so one barrier per exchange suffices.
// With PRE, w holds this thread's twiddles in load_twiddles order.
template <int L, int NTMAX, int SIGN, int S, int NBUF, int MAXR, bool PRE = false>
__device__ __forceinline__ void reg_stages(double2* x, double2* b0, double2* b1, int ps, int t,
                                           const double2* __restrict__ tw, bool act, const double2* w = nullptr) {
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
                if constexpr (PRE) {
#pragma unroll
                    for (int r = 1; r < p; ++r) y[r] = cmul(y[r], w[q * (p - 1) + r - 1]);
                } else {
                    const int step = k * (L / (p * m));
#pragma unroll
                    for (int r = 1; r < p; ++r) y[r] = cmul(y[r], twiddle<SIGN>(tw, r * step));
                }
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
            // one buffer: every thread must have read it before the next stage writes
            if constexpr (NBUF == 1 && S + 1 < sd.nst - 1) __syncthreads();
            reg_stages<L, NTMAX, SIGN, S + 1, NBUF, MAXR, PRE>(x, b0, b1, ps, t, tw, act,
                                                             m > 1 && PRE ? w + Q * (p - 1) : w);
        }
    }
}

// Transform the line held in x (own positions t + NT*e) in place.
// b0/b1: this line's two exchange buffers (position stride ps).  Contains
// barriers: every thread of the block must call it the same number of times.
// Threads with act == false take part in the barriers only (no LDS traffic);
// their x is left undefined.  NBUF = 2 alternates two exchange buffers (one
// barrier per exchange); NBUF = 1 reuses b0 (two barriers, half the LDS).
template <int L, int NTMAX, int SIGN, int NBUF = 2, int MAXR = 8>
__device__ __forceinline__ void reg_fft(double2* x, double2* b0, double2* b1, int ps, int t,
                                        const double2* __restrict__ tw, bool act = true) {
    reg_stages<L, NTMAX, SIGN, 0, NBUF, MAXR>(x, b0, b1, ps, t, tw, act);
}

// The same with the twiddles already in w (load_twiddles<L, NTMAX, SIGN>).
template <int L, int NTMAX, int SIGN, int NBUF = 2, int MAXR = 8>
__device__ __forceinline__ void reg_fft_pre(double2* x, double2* b0, double2* b1, int ps, int t, const double2* w) {
    reg_stages<L, NTMAX, SIGN, 0, NBUF, MAXR, true>(x, b0, b1, ps, t, nullptr, true, w);
}

}  // namespace sgm
