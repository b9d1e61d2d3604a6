// Per-wavenumber Galerkin solves with each chain split over K lanes.
//
// The system of one (column, parity) chain is the one solved by the
// one-lane-per-chain kernel:
//   M x = f,  M = band (offsets -P..Q) + sum_r U_r(i) V_r(j) [j >= i + S],
// eliminated bottom-up with the state
//   rx[d] = x_{i+1+d},  rs[r] = sum_{j >= i+S} V_r(j) x_j   (d < Q, r < NR)
// kept as affine functions c + w . (x_i, .., x_{i-P+1}) of the window.  The
// w parts depend on the matrix only; the c parts are linear in f.
//
// Here the n rows of a chain are cut into K segments of at most R rows (R = 16
// or 8, chosen per plan), one lane each, with the segment's rows held in
// registers:
//  1. w at the bottom of every segment comes from a table filled by a plain
//     sequential sweep of the w recurrence (it depends on kappa^2 and alpha
//     only and is cached per plan);
//  2. each lane eliminates its segment with the incoming c state left
//     symbolic, c = h + Mat c_in, which gives the segment's map
//     c_out = H + Mat c_in (nothing is stored per row);
//  3. a K-step scan over the lanes of the chain (wave shuffles) fixes c_in;
//  4. a second, concrete elimination from the exact entering state leaves
//     a_i and b_i of every row in registers;
//  5. the top-down recovery x_i = a_i + b_i . (x_{i-1}, ..) runs the same
//     way: symbolic in the window entering the segment, a scan, then the
//     final sweep that writes x.
// f is read once and x written once: no workspace traffic.
#include <algorithm>

#include "kernels.h"
#include "solve_seg.h"
#include "solve_seg_dev.h"

namespace sgm {

namespace {

using namespace segdev;

// w state at the bottom of every segment but the last: one lane per chain.
template <int KIND>
__global__ void __launch_bounds__(256) k_seg_table(ChebDev cd, ColGeom g, double alpha, int R, int K, double* tab) {
    using T = SegTraits<KIND>;
    constexpr int P = T::P, Q = T::Q, NR = T::NR, WS = T::WS;
    const int chain = blockIdx.x * blockDim.x + threadIdx.x;
    if (chain >= 2 * g.ncols) return;
    const int p = chain / g.ncols, col = chain - p * g.ncols;
    const int n = cd.npar[p];
    double mu1, mu2;
    chain_mu(g, KIND, col, alpha, mu1, mu2);
    double wx[Q][P], ws[NR][P], Vnext[NR];
#pragma unroll
    for (int d = 0; d < Q; ++d)
#pragma unroll
        for (int e = 0; e < P; ++e) wx[d][e] = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        Vnext[r] = 0.0;
#pragma unroll
        for (int e = 0; e < P; ++e) ws[r][e] = 0.0;
    }
    auto store = [&](int s) {
        double* o = tab + ((long)s * 2 * g.ncols + chain) * WS;
#pragma unroll
        for (int d = 0; d < Q; ++d)
#pragma unroll
            for (int e = 0; e < P; ++e) o[d * P + e] = wx[d][e];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int e = 0; e < P; ++e) o[(Q + r) * P + e] = ws[r][e];
    };
    // boundaries at or beyond n see the zero state
    for (int s = K - 2; s >= 0 && (s + 1) * R >= n; --s) store(s);
    for (int i = n - 1; i >= R; --i) {
        double band[2 * P + 1], U[NR], V[NR], b[P];
        row_coeffs<KIND>(cd.solve[p], p, i, n, mu1, mu2, band, U, V);
        w_step<KIND>(band, U, V, Vnext, (i - 1 + T::S) < n, wx, ws, b);
#pragma unroll
        for (int r = 0; r < NR; ++r) Vnext[r] = V[r];
        if (i % R == 0 && i / R - 1 <= K - 2) store(i / R - 1);
    }
}

// Lane layout: a wave holds C = 64/K adjacent columns of one parity, lane
// = seg * C + column; waves ordered parity-major.
template <int KIND, int K, int R>
__global__ void __launch_bounds__(256) k_solve_seg(const double2* in, double2* out, const double* tab, ChebDev cd,
                                                   ColGeom g, double alpha) {
    constexpr int C = 64 / K;
    const int gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (gw >= 2 * ((g.ncols + C - 1) / C)) return;  // whole wave past the end
    solve_wave<KIND, K, R>(gw, GlobalRhs{in, g.ncols}, GlobalOut{out, g.ncols}, tab, cd, g, alpha, cd.solve[0],
                           cd.solve[1]);
}

template <int KIND, int K, int R>
hipError_t launch_seg_k(const double2* in, double2* out, const double* tab, const ChebDev& cd, const ColGeom& g,
                        double alpha, hipStream_t s) {
    constexpr int C = 64 / K;
    const long waves = 2L * ((g.ncols + C - 1) / C);
    const long blocks = (waves + 3) / 4;
    hipLaunchKernelGGL((k_solve_seg<KIND, K, R>), dim3((unsigned)blocks), dim3(256), 0, s, in, out, tab, cd, g, alpha);
    return hipGetLastError();
}

template <int KIND, int R>
hipError_t launch_seg_lanes(int K, const double2* in, double2* out, const double* tab, const ChebDev& cd,
                            const ColGeom& g, double alpha, hipStream_t s) {
    switch (K) {
        case 1: return launch_seg_k<KIND, 1, R>(in, out, tab, cd, g, alpha, s);
        case 2: return launch_seg_k<KIND, 2, R>(in, out, tab, cd, g, alpha, s);
        case 4: return launch_seg_k<KIND, 4, R>(in, out, tab, cd, g, alpha, s);
        case 8: return launch_seg_k<KIND, 8, R>(in, out, tab, cd, g, alpha, s);
        case 16: return launch_seg_k<KIND, 16, R>(in, out, tab, cd, g, alpha, s);
        default: return hipErrorInvalidValue;
    }
}

template <int KIND>
hipError_t launch_seg_rows(int K, int R, const double2* in, double2* out, const double* tab, const ChebDev& cd,
                           const ColGeom& g, double alpha, hipStream_t s) {
    if (R == 16) return launch_seg_lanes<KIND, 16>(K, in, out, tab, cd, g, alpha, s);
    if (R == 8) return launch_seg_lanes<KIND, 8>(K, in, out, tab, cd, g, alpha, s);
    return hipErrorInvalidValue;
}

}  // namespace

int seg_lanes(int nmax, int R) {
    if (R != 8 && R != 16) return 0;
    int K = 1;
    while (K * R < nmax) K *= 2;
    return K <= kSegMaxLanes ? K : 0;
}

size_t seg_table_doubles(int kind, int K, int ncols) {
    const int WS = kind == SGM_SHEN_BIHARMONIC ? SegTraits<SGM_SHEN_BIHARMONIC>::WS : SegTraits<SGM_SHEN_DIRICHLET>::WS;
    return K > 1 ? (size_t)(K - 1) * 2 * ncols * WS : 0;
}

hipError_t launch_seg_table(double* tab, const ChebDev& cd, const ColGeom& g, int kind, int K, int R, double alpha,
                            hipStream_t s) {
    if (K <= 1) return hipSuccess;
    const int blocks = (2 * g.ncols + 255) / 256;
    switch (kind) {
        case SGM_SHEN_DIRICHLET:
            hipLaunchKernelGGL(k_seg_table<SGM_SHEN_DIRICHLET>, dim3(blocks), dim3(256), 0, s, cd, g, alpha, R, K, tab);
            break;
        case SGM_LEG_DIRICHLET:
            hipLaunchKernelGGL(k_seg_table<SGM_LEG_DIRICHLET>, dim3(blocks), dim3(256), 0, s, cd, g, alpha, R, K, tab);
            break;
        case SGM_SHEN_NEUMANN:
            hipLaunchKernelGGL(k_seg_table<SGM_SHEN_NEUMANN>, dim3(blocks), dim3(256), 0, s, cd, g, alpha, R, K, tab);
            break;
        case SGM_LEG_NEUMANN:
            hipLaunchKernelGGL(k_seg_table<SGM_LEG_NEUMANN>, dim3(blocks), dim3(256), 0, s, cd, g, alpha, R, K, tab);
            break;
        default:
            hipLaunchKernelGGL(k_seg_table<SGM_SHEN_BIHARMONIC>, dim3(blocks), dim3(256), 0, s, cd, g, alpha, R, K,
                               tab);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_solve_seg(const double2* in, double2* out, const double* tab, const ChebDev& cd, const ColGeom& g,
                            int kind, int K, int R, double alpha, hipStream_t s) {
    switch (kind) {
        case SGM_SHEN_DIRICHLET: return launch_seg_rows<SGM_SHEN_DIRICHLET>(K, R, in, out, tab, cd, g, alpha, s);
        case SGM_LEG_DIRICHLET: return launch_seg_rows<SGM_LEG_DIRICHLET>(K, R, in, out, tab, cd, g, alpha, s);
        case SGM_SHEN_NEUMANN: return launch_seg_rows<SGM_SHEN_NEUMANN>(K, R, in, out, tab, cd, g, alpha, s);
        case SGM_LEG_NEUMANN: return launch_seg_rows<SGM_LEG_NEUMANN>(K, R, in, out, tab, cd, g, alpha, s);
        default: return launch_seg_rows<SGM_SHEN_BIHARMONIC>(K, R, in, out, tab, cd, g, alpha, s);
    }
}

}  // namespace sgm
