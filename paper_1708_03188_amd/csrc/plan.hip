// Tensor-product space plans and the C ABI for transforms and solves.
#include <array>
#include <cstdarg>
#include <cstring>
#include <tuple>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "derivative.h"
#include "kernels.h"
#include "kernels_reg.h"
#include "legendre.h"
#include "solve_chain.h"
#include "small.h"
#include "solve_seg.h"
#include "tables.h"
#include "tune_cache.h"

static_assert(sgm::kProjSegRowsDev == sgm::kProjSegRows, "projection segment length mismatch");

namespace sgm {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}
void clear_error() { g_last_error.clear(); }

// Upload helper: packs several host vectors into one device allocation.
struct Blob {
    std::vector<char> host;
    size_t add(const void* p, size_t bytes) {
        size_t off = (host.size() + 255) & ~size_t(255);
        host.resize(off + bytes);
        if (bytes) std::memcpy(host.data() + off, p, bytes);
        return off;
    }
    size_t add(const std::vector<double>& v) { return add(v.data(), v.size() * sizeof(double)); }
};

static int max_lds_bytes() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 65536;
    return v;
}

}  // namespace sgm

using namespace sgm;

// Workspace of sgm_backward_noalloc: the backward x pass writes its output here
// instead of the plan's workspace.  One copy per device, kept until the process
// ends; host code uses only the device address fetched by noalloc_scratch().
static constexpr size_t kNoAllocScratchElems = ((size_t)32 << 20) / sizeof(double2);  // 32 MiB
static __device__ __align__(256) double2 scratch[kNoAllocScratchElems];

// Device address of `scratch` on the current device (looked up once per device).
static sgm_status noalloc_scratch(double2** out) {
    static std::mutex mu;
    static std::map<int, double2*> addr;
    int dev = 0;
    SGM_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it == addr.end()) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error("hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
            return SGM_ERR_HIP;
        }
        it = addr.emplace(dev, static_cast<double2*>(ptr)).first;
    }
    *out = it->second;
    return SGM_OK;
}

struct sgm_plan_s {
    sgm_plan_desc d;
    int N, M1, M2, ndim, r2c;
    int spec_last;   // length of the last spectral axis
    int64_t phys[3], spec[3];
    int64_t nspec;   // complex elements of the spectral array
    void* blob = nullptr;
    void* work = nullptr;
    RadixPlan rpx, rpy, rpz;  // rpy: middle axis (ndim=3) ; rpz: last axis
    // Legendre-family x axis: fragment-ordered forward, backward and scalar-product
    // matrices (in blob) and the points
    bool leg = false;
    const double* leg_fwd = nullptr;
    const double* leg_bwd = nullptr;
    const double* leg_sp = nullptr;
    std::vector<double> xpts;
    ChebDev cd;
    ColGeom geom;
    int G_last, W_mid, W_cheb, W_solve;
    // segmented solves: lanes per chain (0 = chains too long), boundary table
    // valid for seg_alpha once seg_ok
    int seg_K = 0;
    int seg_R = kSegRows;  // rows per lane (chosen by the autotuner: 16 or 8)
    // small 2D spaces: every transform in one kernel (tables in the blob)
    bool small = false;
    SmallDev sd{};
    double* seg_tab = nullptr;
    bool seg_ok = false;
    double seg_alpha = 0.0;
    // register-FFT kernels for axis lengths with a compiled instance
    bool hx = false, hy = false, hz = false;
    RegKernels rkx, rky, rkz;
    // per-pass timing
    unsigned timing = 0;   // bit k: bracket passes of kind k
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    double pass_ms[SGM_NPASS] = {0};
    int64_t pass_cnt[SGM_NPASS] = {0};
};

// Brackets one pass launch with events when the plan's timing is enabled.
struct PassTimer {
    sgm_plan_s* p;
    int kind;
    hipStream_t s;
    hipEvent_t e1 = nullptr, e2 = nullptr;
    PassTimer(sgm_plan_s* p_, int k, hipStream_t s_) : p(p_), kind(k), s(s_) {
        if (!((p->timing >> kind) & 1u)) return;
        e1 = take();
        e2 = take();
        if (e1) hipEventRecord(e1, s);
    }
    hipEvent_t take() {
        hipEvent_t e = nullptr;
        if (!p->ev_pool.empty()) { e = p->ev_pool.back(); p->ev_pool.pop_back(); }
        // timing-only events: no system-scope fence (no cache write-back at the
        // record), so the interval is the pass itself
        else if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) e = nullptr;
        return e;
    }
    ~PassTimer() {
        if (!((p->timing >> kind) & 1u) || !e1 || !e2) return;
        hipEventRecord(e2, s);
        p->pending.push_back({kind, {e1, e2}});
    }
};

static sgm_status make_radix(int L, RadixPlan& rp) {
    rp.L = L;
    rp.nst = factor_radices(L, rp.radix);
    rp.tw = nullptr;
    if (rp.nst > kMaxStages) {
        set_error("FFT length %d needs too many stages", L);
        return SGM_ERR_UNSUPPORTED_SIZE;
    }
    return SGM_OK;
}

template <typename F, typename... A>
static hipError_t launch_k(F f, long blocks, int threads, size_t lds, hipStream_t s, A... args) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(threads), lds, s, args...);
    return hipGetLastError();
}

static int pick_tile(int L, int want, size_t (*bytes)(int, int), int lds_max) {
    int w = want;
    while (w > 1 && bytes(L, w) > (size_t)lds_max) w /= 2;
    return w;
}

static sgm_status fourier_forward(sgm_plan p, const void* u, double2* uh, hipStream_t s);
static sgm_status fourier_backward(sgm_plan p, double2* w, void* u, hipStream_t s);
static hipError_t cheb_forward_pass(sgm_plan p, double2* data, int mode, hipStream_t s);
extern "C" sgm_status sgm_forward(sgm_plan p, const void* u, void* u_hat, void* stream);
extern "C" sgm_status sgm_backward(sgm_plan p, const void* u_hat, void* u, void* stream);

// Autotuner: for every axis with register kernels, time each compiled variant
// (threads per line, exchange buffers, block size, radix schedule) on the plan's
// own passes and keep the fastest; then the rows per lane of the segmented
// solves.  Choices (three variants and the rows per lane) are remembered per
// process, keyed by the plan geometry, and in the tune-cache file keyed by the
// device and the geometry.
struct TuneKey {
    int ndim, basis, N, M1, M2, kind;
    bool operator<(const TuneKey& o) const {
        return std::tie(ndim, basis, N, M1, M2, kind) < std::tie(o.ndim, o.basis, o.N, o.M1, o.M2, o.kind);
    }
};
static std::map<TuneKey, std::array<int, 4>> g_tuned;
static std::mutex g_tune_mu;

// Pass-timer bits of each axis's passes (x: forward projection and backward;
// y: middle pair; z: last pair).
static const unsigned kAxisPasses[3] = {(1u << 4) | (1u << 6), (1u << 2) | (1u << 3), (1u << 0) | (1u << 1)};

// Time of the given passes in one forward + backward step: best of 8 steps per
// pass (after one untimed step), so the other axes' passes add no noise.
static float axis_pass_ms(sgm_plan p, void* u, void* uh, unsigned mask, hipStream_t s) {
    const unsigned saved = p->timing;
    p->timing = 0;
    sgm_forward(p, u, uh, s);
    sgm_backward(p, uh, u, s);
    p->timing = mask;
    for (int r = 0; r < 8; ++r) {
        sgm_forward(p, u, uh, s);
        sgm_backward(p, uh, u, s);
    }
    p->timing = saved;
    float best[SGM_NPASS];
    for (float& b : best) b = 1e30f;
    for (auto& pe : p->pending) {
        float t = 1e30f;
        if (hipEventSynchronize(pe.second.second) != hipSuccess ||
            hipEventElapsedTime(&t, pe.second.first, pe.second.second) != hipSuccess)
            t = 1e30f;
        best[pe.first] = std::min(best[pe.first], t);
        p->ev_pool.push_back(pe.second.first);
        p->ev_pool.push_back(pe.second.second);
    }
    p->pending.clear();
    float sum = 0.f;
    for (int i = 0; i < SGM_NPASS; ++i)
        if (((mask >> i) & 1u) && best[i] < 1e29f) sum += best[i];
    return sum;
}

// Take stored choices if every one names a compiled variant that fits.
static bool apply_tuned(sgm_plan p, const std::array<int, 4>& v, int lds_max) {
    const int Llast = p->ndim == 3 ? p->M2 : p->M1;
    RegKernels k[3];
    const bool has[3] = {p->hx, p->hy, p->hz};
    const int L[3] = {p->N, p->M1, Llast};
    for (int a = 0; a < 3; ++a) {
        if (!has[a]) continue;
        if (v[a] < 0 || v[a] >= kRegVariants || !reg_kernels_for(L[a], k[a], v[a])) return false;
        if ((a == 0 ? k[a].lds_cheb : a == 1 ? k[a].lds_str : k[a].lds) > (size_t)lds_max) return false;
        if (a == 1 && !strided_fits(k[a], p->spec_last)) return false;
    }
    if (v[3] != 8 && v[3] != kSegRows) return false;
    if (p->hx) p->rkx = k[0];
    if (p->hy) p->rky = k[1];
    if (p->hz) p->rkz = k[2];
    p->seg_R = v[3];
    return true;
}

static bool biharmonic_basis(int basis) { return basis == SGM_SHEN_BIHARMONIC || basis == SGM_LEG_BIHARMONIC; }
static int solve_kind(int basis) { return biharmonic_basis(basis) ? SGM_SHEN_BIHARMONIC : basis; }
static int table_kind(int basis) { return biharmonic_basis(basis) ? SGM_SHEN_BIHARMONIC : SGM_SHEN_DIRICHLET; }
// Bases whose solves run the segmented kernels.
static bool seg_basis(int basis) { return basis != SGM_CHEBYSHEV && basis != SGM_LEGENDRE; }

// Time of the segmented solve at R rows per lane (table filled, best of three
// launches in place on uh); 1e30 where the chains are too long for R.
static float solve_rows_ms(sgm_plan p, void* uh, int R, hipStream_t s) {
    const int nmax = std::max(p->cd.npar[0], p->cd.npar[1]);
    const int K = seg_lanes(nmax, R);
    if (K <= 0) return 1e30f;
    const int kind = solve_kind(p->d.basis);
    const double alpha = kind == SGM_SHEN_BIHARMONIC ? 0.0 : 1.0;
    const size_t nt = seg_table_doubles(kind, K, p->geom.ncols);
    double* tab = nullptr;
    if (nt > 0 && hipMalloc(&tab, nt * sizeof(double)) != hipSuccess) return 1e30f;
    float best = 1e30f;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
        launch_seg_table(tab, p->cd, p->geom, kind, K, R, alpha, s) == hipSuccess) {
        double2* d = static_cast<double2*>(uh);
        if (launch_solve_seg(d, d, tab, p->cd, p->geom, kind, K, R, alpha, s) == hipSuccess) {
            for (int r = 0; r < 3; ++r) {
                float t = 1e30f;
                if (hipEventRecord(e0, s) != hipSuccess ||
                    launch_solve_seg(d, d, tab, p->cd, p->geom, kind, K, R, alpha, s) != hipSuccess ||
                    hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&t, e0, e1) != hipSuccess)
                    t = 1e30f;
                best = std::min(best, t);
            }
        }
    }
    hipStreamSynchronize(s);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(tab);
    return best;
}

static std::string plan_tune_key(sgm_plan p) {
    char b[160];
    snprintf(b, sizeof(b), "plan %s ndim%d basis%d %dx%dx%d kind%d", tune_device_tag().c_str(), p->ndim, p->d.basis,
             p->N, p->M1, p->M2, p->d.kind_last);
    return b;
}

static sgm_status autotune_plan(sgm_plan p, int lds_max, hipStream_t s) {
    TuneKey key{p->ndim, p->d.basis, p->N, p->M1, p->M2, p->d.kind_last};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end() && apply_tuned(p, it->second, lds_max)) return SGM_OK;
    }
    const std::string fkey = plan_tune_key(p);
    std::vector<int> cached;
    if (tune_cache_get(fkey, cached) && (cached.size() == 3 || cached.size() == 4)) {
        // three values: an entry from before the solve was tuned (16 rows per lane)
        const std::array<int, 4> v{cached[0], cached[1], cached[2], cached.size() == 4 ? cached[3] : kSegRows};
        if (apply_tuned(p, v, lds_max)) {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tuned[key] = v;
            return SGM_OK;
        }
    }
    const size_t phys_bytes = (size_t)p->phys[0] * p->phys[1] * p->phys[2] * (p->r2c ? sizeof(double) : sizeof(double2));
    void* u = nullptr;
    void* uh = nullptr;
    if (hipMalloc(&u, phys_bytes) != hipSuccess) return SGM_ERR_OOM;
    if (hipMalloc(&uh, (size_t)p->nspec * sizeof(double2)) != hipSuccess) { hipFree(u); return SGM_ERR_OOM; }
    if (hipMemsetAsync(u, 0, phys_bytes, s) != hipSuccess ||
        hipMemsetAsync(uh, 0, (size_t)p->nspec * sizeof(double2), s) != hipSuccess) {
        hipFree(u);
        hipFree(uh);
        set_error("tuning set-up failed");
        return SGM_ERR_HIP;
    }
    const int Llast = p->ndim == 3 ? p->M2 : p->M1;
    std::array<int, 4> best{0, 0, 0, kSegRows};
    struct Ax { bool has; RegKernels* rk; int L; int idx; };
    Ax axes[3] = {{p->hx, &p->rkx, p->N, 0}, {p->hy, &p->rky, p->M1, 1}, {p->hz, &p->rkz, Llast, 2}};
    for (auto& ax : axes) {
        if (!ax.has || p->small) continue;  // a small space runs no per-axis pass
        float tbest = 1e30f;
        for (int v = 0; v < kRegVariants; ++v) {
            RegKernels cand;
            if (!reg_kernels_for(ax.L, cand, v)) continue;
            if ((ax.idx == 0 ? cand.lds_cheb : ax.idx == 1 ? cand.lds_str : cand.lds) > (size_t)lds_max) continue;
            if (ax.idx == 1 && !strided_fits(cand, p->spec_last)) continue;
            RegKernels saved = *ax.rk;
            *ax.rk = cand;
            const float t = axis_pass_ms(p, u, uh, kAxisPasses[ax.idx], s);
            *ax.rk = saved;
            if (t < tbest) { tbest = t; best[ax.idx] = v; }
        }
        reg_kernels_for(ax.L, *ax.rk, best[ax.idx]);
    }
    // rows per lane of the segmented solve (lanes per chain follow from the chain length)
    if (seg_basis(p->d.basis)) {
        float tbest = 1e30f;
        for (int R : {kSegRows, 8}) {
            const float t = solve_rows_ms(p, uh, R, s);
            if (t < tbest) { tbest = t; best[3] = R; }
        }
        p->seg_R = best[3];
    }
    hipStreamSynchronize(s);
    hipFree(u);
    hipFree(uh);
    tune_cache_put(fkey, {best[0], best[1], best[2], best[3]});
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = best;
    return SGM_OK;
}

extern "C" {

int sgm_version(void) { return 1; }

sgm_status sgm_autotune_forget(void) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
    return SGM_OK;
}

sgm_status sgm_autotune_cache_path(char* buf, int len) {
    clear_error();
    SGM_CHECK_ARG(buf && len > 0, "null buffer");
    const std::string p = tune_cache_path();
    SGM_CHECK_ARG((int)p.size() < len, "buffer too small (%d bytes needed)", (int)p.size() + 1);
    std::memcpy(buf, p.c_str(), p.size() + 1);
    return SGM_OK;
}

const char* sgm_last_error(void) { return g_last_error.c_str(); }

const char* sgm_status_string(sgm_status s) {
    switch (s) {
        case SGM_OK: return "ok";
        case SGM_ERR_INVALID_ARG: return "invalid argument";
        case SGM_ERR_UNSUPPORTED_SIZE: return "unsupported size";
        case SGM_ERR_HIP: return "HIP runtime error";
        case SGM_ERR_OOM: return "out of device memory";
        case SGM_ERR_UNIMPLEMENTED: return "not implemented";
        case SGM_ERR_SINGULAR: return "singular system";
        default: return "unknown status";
    }
}

// Kind of the segmented solve kernels for a basis: the Helmholtz kinds evaluate
// their rows in closed form, so each basis is its own kind; the biharmonic kind
// reads its rows from the plan's table, Chebyshev and Legendre alike.  The
// table-driven generic and chain kernels read every Helmholtz basis's rows, which
// have the Dirichlet shape (band + a rank-1 tail, zero for the Legendre bases), as
// SGM_SHEN_DIRICHLET.

sgm_status sgm_plan_create(const sgm_plan_desc* desc, void* stream, sgm_plan* out) {
    clear_error();
    TraceRange trace_range("sgm_plan_create");
    SGM_CHECK_ARG(desc && out, "null argument");
    *out = nullptr;
    const sgm_plan_desc& d = *desc;
    SGM_CHECK_ARG(d.ndim == 2 || d.ndim == 3, "ndim must be 2 or 3 (got %d)", d.ndim);
    SGM_CHECK_ARG(d.basis == SGM_SHEN_DIRICHLET || d.basis == SGM_SHEN_BIHARMONIC || d.basis == SGM_CHEBYSHEV ||
                      d.basis == SGM_SHEN_NEUMANN || is_legendre_basis(d.basis),
                  "unknown basis %d", d.basis);
    SGM_CHECK_ARG(d.kind_last == SGM_R2C || d.kind_last == SGM_C2C, "unknown kind_last %d", d.kind_last);
    const bool leg = is_legendre_basis(d.basis);
    int minN = (d.basis == SGM_SHEN_DIRICHLET || d.basis == SGM_SHEN_NEUMANN || d.basis == SGM_LEG_DIRICHLET ||
                d.basis == SGM_LEG_NEUMANN)
                   ? 3
               : (d.basis == SGM_SHEN_BIHARMONIC || d.basis == SGM_LEG_BIHARMONIC) ? 5
                                                                                    : 2;
    if (leg && d.N > kLegMaxN) {
        set_error("Legendre spaces support N <= %d (got %d)", kLegMaxN, d.N);
        return SGM_ERR_UNSUPPORTED_SIZE;
    }
    int M2 = d.ndim == 3 ? d.M2 : 1;
    if (d.N < minN || d.M1 < 1 || M2 < 1 || d.N > 65536 || d.M1 > 65536 || M2 > 65536) {
        set_error("unsupported sizes N=%d M1=%d M2=%d for basis %d", d.N, d.M1, M2, d.basis);
        return SGM_ERR_UNSUPPORTED_SIZE;
    }
    SGM_CHECK_ARG(d.Ly >= 0 && d.Lz >= 0, "negative period");
    if (d.basis == SGM_SHEN_NEUMANN && d.N > kDxMaxN) {
        set_error("the Neumann basis supports N <= %d (its projection runs in the derivative pass)", kDxMaxN);
        return SGM_ERR_UNSUPPORTED_SIZE;
    }
    sgm_plan_s* p = new (std::nothrow) sgm_plan_s();
    if (!p) return SGM_ERR_OOM;
    p->d = d;
    p->N = d.N;
    p->M1 = d.M1;
    p->M2 = M2;
    p->ndim = d.ndim;
    p->r2c = d.kind_last == SGM_R2C;
    int Llast = d.ndim == 3 ? M2 : d.M1;
    p->spec_last = p->r2c ? Llast / 2 + 1 : Llast;
    p->phys[0] = d.N; p->phys[1] = d.M1; p->phys[2] = d.ndim == 3 ? M2 : 1;
    p->spec[0] = d.N;
    if (d.ndim == 3) { p->spec[1] = d.M1; p->spec[2] = p->spec_last; }
    else { p->spec[1] = p->spec_last; p->spec[2] = 1; }
    p->nspec = p->spec[0] * p->spec[1] * p->spec[2];

    sgm_status st;
    if ((st = make_radix(d.N, p->rpx)) != SGM_OK) { delete p; return st; }
    if (d.ndim == 3 && (st = make_radix(d.M1, p->rpy)) != SGM_OK) { delete p; return st; }
    if ((st = make_radix(Llast, p->rpz)) != SGM_OK) { delete p; return st; }

    ChebTables ct;
    LegTables lt;
    std::string err;
    if (leg ? !build_leg_tables(d.basis, d.N, lt, err) : !build_cheb_tables(d.basis, d.N, ct, err)) {
        set_error("%s", err.c_str());
        delete p;
        return SGM_ERR_UNSUPPORTED_SIZE;
    }
    if (leg) {
        ct.basis = d.basis;
        ct.N = d.N;
        ct.nb = lt.nb;
        for (int q = 0; q < 2; ++q) {
            ct.npar[q] = lt.npar[q];
            ct.mpar[q] = lt.mpar[q];
            ct.solve[q] = lt.solve[q];
        }
        ct.beta = lt.beta;
        ct.gamma = lt.gamma;
        p->xpts = lt.x;
    } else {
        p->xpts.resize(d.N);
        for (int j = 0; j < d.N; ++j) p->xpts[j] = std::cos((2 * j + 1) * 3.14159265358979323846 / (2.0 * d.N));
    }
    Blob b;
    // Small 2D spaces (N, M <= 64, not biharmonic: its projection matrix is
    // ill-conditioned) run every transform in one kernel, except where the plan
    // pins register-kernel variants or asks for the generic kernels.
    const bool small = d.ndim == 2 && d.N <= kSmallMaxN && d.M1 <= kSmallMaxM && !biharmonic_basis(d.basis) &&
                       (d.autotune == 0 || d.autotune == 1);
    size_t o_small = 0;
    if (small) {
        std::vector<double> sv;
        if (!build_small_tables(d.basis, d.N, d.M1, p->r2c, leg ? &lt.fwd : nullptr, leg ? &lt.sp : nullptr,
                                leg ? &lt.bwd : nullptr, sv, err)) {
            set_error("%s", err.c_str());
            delete p;
            return SGM_ERR_UNSUPPORTED_SIZE;
        }
        o_small = b.add(sv);
    }
    size_t o_lf = 0, o_lb = 0, o_ls = 0;
    if (leg) {
        o_lf = b.add(leg_pack(lt.fwd, d.N));
        o_lb = b.add(leg_pack(lt.bwd, d.N));
        o_ls = b.add(leg_pack(lt.sp, d.N));
    }
    size_t o_twx = b.add(twiddles(d.N));
    size_t o_twy = d.ndim == 3 ? b.add(twiddles(d.M1)) : 0;
    size_t o_twz = b.add(twiddles(Llast));
    size_t o_theta = b.add(ct.theta), o_beta = b.add(ct.beta), o_gamma = b.add(ct.gamma);
    size_t o_bs = b.add(ct.bscale), o_fs = b.add(ct.fscale);
    size_t o_rot[2], o_rt[2], o_sv[2], o_qt[2], o_gal[2], o_gm[2], o_bal[2], o_bm[2];
    for (int q = 0; q < 2; ++q) {
        o_qt[q] = b.add(ct.qtab[q]);
        o_rot[q] = b.add(ct.rot[q]);
        o_rt[q] = b.add(ct.rtab[q]);
        o_gal[q] = b.add(ct.gal[q]);
        o_gm[q] = b.add(ct.gmat[q]);
        o_bal[q] = b.add(ct.bal[q]);
        o_bm[q] = b.add(ct.bmat[q]);
        o_sv[q] = b.add(ct.solve[q]);
    }
    hipError_t e = hipMalloc(&p->blob, b.host.size());
    if (e != hipSuccess) { set_error("hipMalloc tables: %s", hipGetErrorString(e)); delete p; return SGM_ERR_OOM; }
    hipStream_t cs = static_cast<hipStream_t>(stream);
    e = hipMemcpyAsync(p->blob, b.host.data(), b.host.size(), hipMemcpyHostToDevice, cs);
    if (e == hipSuccess) e = hipStreamSynchronize(cs);  // the host staging buffer goes out of scope
    if (e != hipSuccess) { set_error("uploading the tables: %s", hipGetErrorString(e)); hipFree(p->blob); delete p; return SGM_ERR_HIP; }
    e = hipMalloc(&p->work, (size_t)p->nspec * sizeof(double2));
    if (e != hipSuccess) { set_error("hipMalloc workspace: %s", hipGetErrorString(e)); hipFree(p->blob); delete p; return SGM_ERR_OOM; }
    char* base = static_cast<char*>(p->blob);
    auto D = [&](size_t off) { return reinterpret_cast<const double*>(base + off); };
    p->rpx.tw = reinterpret_cast<const double2*>(base + o_twx);
    if (d.ndim == 3) p->rpy.tw = reinterpret_cast<const double2*>(base + o_twy);
    p->rpz.tw = reinterpret_cast<const double2*>(base + o_twz);
    ChebDev& cd = p->cd;
    cd.basis = d.basis; cd.N = d.N; cd.nb = ct.nb;
    for (int q = 0; q < 2; ++q) {
        cd.npar[q] = ct.npar[q]; cd.mpar[q] = ct.mpar[q];
        cd.rot[q] = D(o_rot[q]); cd.rtab[q] = D(o_rt[q]); cd.solve[q] = D(o_sv[q]); cd.qtab[q] = D(o_qt[q]);
        cd.gal[q] = D(o_gal[q]); cd.gmat[q] = D(o_gm[q]); cd.bal[q] = D(o_bal[q]); cd.bmat[q] = D(o_bm[q]);
    }
    cd.theta = reinterpret_cast<const double2*>(base + o_theta);
    cd.beta = D(o_beta); cd.gamma = D(o_gamma); cd.bscale = D(o_bs); cd.fscale = D(o_fs);
    if (leg) {
        p->leg = true;
        p->leg_fwd = D(o_lf);
        p->leg_bwd = D(o_lb);
        p->leg_sp = D(o_ls);
    }
    if (small) {
        SmallDev& sd = p->sd;
        sd.N = d.N;
        sd.M = d.M1;
        sd.r2c = p->r2c ? 1 : 0;
        sd.Mc = p->spec_last;
        const size_t nF = 2 * (size_t)sd.M * sd.Mc;
        sd.F = reinterpret_cast<const double2*>(base + o_small);
        sd.G = reinterpret_cast<const double2*>(base + o_small + nF * sizeof(double));
        for (int m = 0; m < 3; ++m) sd.P[m] = D(o_small + (2 * nF + (size_t)m * d.N * d.N) * sizeof(double));
        p->small = true;
    }

    const double twopi = 6.283185307179586476925286766559;
    double Ly = d.Ly > 0 ? d.Ly : twopi, Lz = d.Lz > 0 ? d.Lz : twopi;
    ColGeom& g = p->geom;
    g.ncols = (int)(p->spec[1] * p->spec[2]);
    g.nlast = p->spec_last;
    g.Mlast = Llast;
    g.last_r2c = p->r2c;
    if (d.ndim == 3) {
        g.Mmid = d.M1;
        g.sy = (twopi / Ly) * (twopi / Ly);
        g.sz = (twopi / Lz) * (twopi / Lz);
    } else {
        g.Mmid = 1;
        g.sy = 0.0;
        g.sz = (twopi / Ly) * (twopi / Ly);
    }
    int lds = max_lds_bytes();
    p->G_last = pick_tile(Llast, Llast >= 2048 ? 1 : 2048 / Llast, lds_bytes_lines, lds);
    if (p->G_last > 16) p->G_last = 16;
    p->W_mid = d.ndim == 3 ? pick_tile(d.M1, 16, lds_bytes_strided, lds) : 1;
    p->W_cheb = leg ? 1 : pick_tile(d.N, d.N <= 256 ? 16 : 8, lds_bytes_cheb, lds);
    int ws = d.N <= 256 ? 16 : 8;
    while (ws > 1 && lds_bytes_solve(d.N, ws, table_kind(d.basis)) > (size_t)lds) ws /= 2;
    p->W_solve = ws;
    if (lds_bytes_lines(Llast, p->G_last) > (size_t)lds || (!leg && lds_bytes_cheb(d.N, p->W_cheb) > (size_t)lds) ||
        (d.ndim == 3 && lds_bytes_strided(d.M1, p->W_mid) > (size_t)lds)) {
        set_error("axis length too large for one work-group's LDS (%d bytes)", lds);
        hipFree(p->work); hipFree(p->blob); delete p;
        return SGM_ERR_UNSUPPORTED_SIZE;
    }
    if (d.autotune != 2) {
        // autotune >= 16 pins variant (autotune - 16) where it exists (diagnostics)
        const int v0 = d.autotune >= 16 ? d.autotune - 16 : 0;
        auto pick = [&](int L, RegKernels& k) { return reg_kernels_for(L, k, v0) || reg_kernels_for(L, k, 0); };
        p->hx = !leg && pick(d.N, p->rkx);
        p->hy = d.ndim == 3 && pick(d.M1, p->rky);
        p->hz = pick(Llast, p->rkz);
        if (p->hx && p->rkx.lds_cheb > (size_t)lds) p->hx = false;
        if (p->hy && (p->rky.lds_str > (size_t)lds || !strided_fits(p->rky, p->spec_last))) p->hy = false;
        if (p->hz && p->rkz.lds > (size_t)lds) p->hz = false;
        if (d.autotune == 1) {
            sgm_status st2 = autotune_plan(p, lds, cs);
            if (st2 != SGM_OK) { hipFree(p->work); hipFree(p->blob); delete p; return st2; }
        }
    }
    if (d.basis != SGM_CHEBYSHEV && d.basis != SGM_LEGENDRE && d.autotune != 2) {
        p->seg_K = seg_lanes(std::max(cd.npar[0], cd.npar[1]), p->seg_R);
        const size_t nt = seg_table_doubles(solve_kind(d.basis), p->seg_K, g.ncols);
        if (p->seg_K > 0 && nt > 0 && hipMalloc(&p->seg_tab, nt * sizeof(double)) != hipSuccess) {
            set_error("hipMalloc solve table failed");
            hipFree(p->work); hipFree(p->blob); delete p;
            return SGM_ERR_OOM;
        }
    }
    *out = p;
    return SGM_OK;
}

sgm_status sgm_plan_timing(sgm_plan p, int enable) {
    clear_error();
    SGM_CHECK_ARG(p, "null plan");
    p->timing = (enable & SGM_TIMING_ONLY) ? (unsigned)(enable & 0xff) : (enable ? 0xffu : 0u);
    return SGM_OK;
}

sgm_status sgm_plan_solve_layout(sgm_plan p, int* lanes, int* rows) {
    clear_error();
    SGM_CHECK_ARG(p && lanes && rows, "null argument");
    *lanes = p->seg_K;
    *rows = p->seg_K > 0 ? p->seg_R : 0;
    return SGM_OK;
}

sgm_status sgm_plan_set_solve_rows(sgm_plan p, int rows) {
    clear_error();
    SGM_CHECK_ARG(p, "null plan");
    SGM_CHECK_ARG(rows == 8 || rows == kSegRows, "rows per lane must be 8 or %d (got %d)", kSegRows, rows);
    SGM_CHECK_ARG(seg_basis(p->d.basis) && p->d.autotune != 2, "the plan has no segmented solve");
    const int K = seg_lanes(std::max(p->cd.npar[0], p->cd.npar[1]), rows);
    SGM_CHECK_ARG(K > 0, "chains of %d rows are too long for %d rows per lane",
                  std::max(p->cd.npar[0], p->cd.npar[1]), rows);
    const size_t nt = seg_table_doubles(solve_kind(p->d.basis), K, p->geom.ncols);
    // the old table may still be read by queued solves
    if (p->seg_tab) SGM_HIP_TRY(hipDeviceSynchronize());
    double* tab = nullptr;
    if (nt > 0 && hipMalloc(&tab, nt * sizeof(double)) != hipSuccess) {
        set_error("hipMalloc solve table failed");
        return SGM_ERR_OOM;
    }
    hipFree(p->seg_tab);
    p->seg_tab = tab;
    p->seg_K = K;
    p->seg_R = rows;
    p->seg_ok = false;
    return SGM_OK;
}

sgm_status sgm_plan_variants(sgm_plan p, int variant[3]) {
    clear_error();
    SGM_CHECK_ARG(p && variant, "null argument");
    variant[0] = p->hx ? p->rkx.variant : -1;
    variant[1] = p->hy ? p->rky.variant : -1;
    variant[2] = p->hz ? p->rkz.variant : -1;
    return SGM_OK;
}

sgm_status sgm_plan_pass_times(sgm_plan p, double ms[SGM_NPASS], int64_t count[SGM_NPASS], int reset) {
    clear_error();
    SGM_CHECK_ARG(p && ms && count, "null argument");
    for (auto& pe : p->pending) {
        float t = 0.f;
        SGM_HIP_TRY(hipEventSynchronize(pe.second.second));
        SGM_HIP_TRY(hipEventElapsedTime(&t, pe.second.first, pe.second.second));
        p->pass_ms[pe.first] += t;
        p->pass_cnt[pe.first] += 1;
        p->ev_pool.push_back(pe.second.first);
        p->ev_pool.push_back(pe.second.second);
    }
    p->pending.clear();
    for (int i = 0; i < SGM_NPASS; ++i) { ms[i] = p->pass_ms[i]; count[i] = p->pass_cnt[i]; }
    if (reset)
        for (int i = 0; i < SGM_NPASS; ++i) { p->pass_ms[i] = 0; p->pass_cnt[i] = 0; }
    return SGM_OK;
}

sgm_status sgm_plan_destroy(sgm_plan p) {
    clear_error();
    if (!p) return SGM_OK;
    for (auto& pe : p->pending) { hipEventDestroy(pe.second.first); hipEventDestroy(pe.second.second); }
    for (auto e : p->ev_pool) hipEventDestroy(e);
    hipFree(p->seg_tab);
    hipFree(p->work);
    hipFree(p->blob);
    delete p;
    return SGM_OK;
}

sgm_status sgm_plan_points(sgm_plan p, double* x) {
    clear_error();
    SGM_CHECK_ARG(p && x, "null argument");
    for (int j = 0; j < p->N; ++j) x[j] = p->xpts[j];
    return SGM_OK;
}

sgm_status sgm_plan_shapes(sgm_plan p, int64_t phys[3], int64_t spec[3]) {
    clear_error();
    SGM_CHECK_ARG(p && phys && spec, "null argument");
    for (int i = 0; i < 3; ++i) { phys[i] = p->phys[i]; spec[i] = p->spec[i]; }
    return SGM_OK;
}

static sgm_status fourier_forward(sgm_plan p, const void* u, double2* uh, hipStream_t s) {
    int Llast = p->ndim == 3 ? p->M2 : p->M1;
    int nlines = p->ndim == 3 ? p->N * p->M1 : p->N;
    {
        PassTimer t(p, 0, s);
        const RegKernels& k = p->rkz;
        if (p->r2c) {
            if (p->hz)
                SGM_HIP_TRY(launch_k(k.r2c, (nlines + 2 * k.W - 1) / (2 * k.W), k.threads, k.lds, s,
                                     static_cast<const double*>(u), uh, nlines, p->rpz.tw, 1.0 / Llast));
            else
                SGM_HIP_TRY(launch_lines_r2c(static_cast<const double*>(u), uh, Llast, nlines, p->G_last, p->rpz,
                                             1.0 / Llast, s));
        } else {
            if (p->hz)
                SGM_HIP_TRY(launch_k(k.c2c_f, (nlines + k.W - 1) / k.W, k.threads, k.lds, s,
                                     static_cast<const double2*>(u), uh, nlines, p->rpz.tw, 1.0 / Llast));
            else
                SGM_HIP_TRY(launch_lines_c2c(static_cast<const double2*>(u), uh, Llast, nlines, p->G_last, p->rpz,
                                             -1, 1.0 / Llast, s));
        }
    }
    if (p->ndim == 3) {
        PassTimer t(p, 2, s);
        const RegKernels& k = p->rky;
        if (p->hy)
            SGM_HIP_TRY(launch_strided(k, -1, uh, uh, p->N, p->spec_last, p->rpy.tw, 1.0 / p->M1, s));
        else
            SGM_HIP_TRY(launch_strided_c2c(uh, uh, p->M1, p->N, p->spec_last, p->W_mid, p->rpy, -1, 1.0 / p->M1, s));
    }
    return SGM_OK;
}

// Derivative-pass arguments for coefficients in p's space going to a space with
// basis dst on the same grid (orders ox, oy, oz).
static DxArgs dx_args(sgm_plan p, int src_basis, int dst_basis, int ox, int oy, int oz) {
    const double twopi = 6.283185307179586476925286766559;
    auto per = [twopi](double L) { return L > 0 ? L : twopi; };
    DxArgs x;
    x.N = p->N;
    x.ncols = p->geom.ncols;
    x.src_basis = src_basis;
    x.nb_src = src_basis == SGM_CHEBYSHEV ? p->N : p->cd.nb;
    x.beta = p->cd.beta;
    x.gamma = p->cd.gamma;
    x.dst_basis = dst_basis;
    x.leg = is_legendre_basis(src_basis) ? 1 : 0;
    // Neumann targets: sum over each parity of q_k^2 h_k (see DxArgs)
    x.k4[0] = x.k4[1] = 0.0;
    for (int k = 0; k < p->N; ++k) {
        const double q = x.leg ? (double)k * (k + 1) : (double)k * k, h = x.leg ? (2.0 * k + 1.0) / 2.0 : 1.0;
        x.k4[k & 1] += q * q * h;
    }
    x.ox = ox;
    x.oy = oy;
    x.oz = oz;
    x.ndim = p->ndim;
    x.nlast = p->geom.nlast;
    x.Mmid = p->geom.Mmid;
    x.Mlast = p->geom.Mlast;
    x.last_r2c = p->geom.last_r2c;
    x.ky = twopi / per(p->d.Ly);
    x.kz = twopi / per(p->d.Lz);
    return x;
}

static hipError_t cheb_forward_pass(sgm_plan p, double2* data, int mode, hipStream_t s) {
    if (p->leg)
        return launch_leg_pass(mode == kProject ? p->leg_fwd : p->leg_sp, reinterpret_cast<const double*>(data),
                               reinterpret_cast<double*>(data), p->N, 2L * p->geom.ncols, s);
    if (mode == kProject && p->cd.basis == SGM_SHEN_NEUMANN) {
        // Neumann: Chebyshev interpolation coefficients, then their projection onto
        // the space (in place: the Chebyshev-source projection reads only its own rows)
        hipError_t e;
        if (!p->hx) {
            ChebDev cc = p->cd;
            cc.basis = SGM_CHEBYSHEV;
            cc.nb = p->N;
            e = launch_cheb_fwd(data, data, cc, p->geom.ncols, p->W_cheb, p->rpx, mode, s);
        } else {
            const RegKernels& k = p->rkx;
            e = launch_k(k.cf_cheb, (p->geom.ncols + k.W - 1) / k.W, k.threads, k.lds_cheb, s, (const double2*)data,
                         data, p->cd, p->geom.ncols, p->rpx.tw, ChebSolve{nullptr, p->geom, 0.0});
        }
        if (e != hipSuccess) return e;
        return launch_dx_project(data, data, dx_args(p, SGM_CHEBYSHEV, SGM_SHEN_NEUMANN, 0, 0, 0), s);
    }
    if (!p->hx) return launch_cheb_fwd(data, data, p->cd, p->geom.ncols, p->W_cheb, p->rpx, mode, s);
    const RegKernels& k = p->rkx;
    auto f = k.cf_sp;
    if (mode == kProject)
        f = p->cd.basis == SGM_SHEN_DIRICHLET ? k.cf_dir : p->cd.basis == SGM_SHEN_BIHARMONIC ? k.cf_bih : k.cf_cheb;
    return launch_k(f, (p->geom.ncols + k.W - 1) / k.W, k.threads, k.lds_cheb, s, (const double2*)data, data, p->cd,
                    p->geom.ncols, p->rpx.tw, ChebSolve{nullptr, p->geom, 0.0});
}

sgm_status sgm_forward(sgm_plan p, const void* u, void* u_hat, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_forward");
    SGM_CHECK_ARG(p && u && u_hat, "null argument");
    SGM_CHECK_ARG(u != u_hat, "u and u_hat must not alias");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2* uh = static_cast<double2*>(u_hat);
    if (p->small) {
        PassTimer t(p, 4, s);
        SGM_HIP_TRY(launch_small_pass(u, uh, p->sd, kSmallForward, s));
        return SGM_OK;
    }
    sgm_status st = fourier_forward(p, u, uh, s);
    if (st != SGM_OK) return st;
    PassTimer t(p, 4, s);
    SGM_HIP_TRY(cheb_forward_pass(p, uh, kProject, s));
    return SGM_OK;
}

sgm_status sgm_scalar_product(sgm_plan p, const void* f, void* f_tilde, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_scalar_product");
    SGM_CHECK_ARG(p && f && f_tilde, "null argument");
    SGM_CHECK_ARG(f != f_tilde, "f and f_tilde must not alias");
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2* ft = static_cast<double2*>(f_tilde);
    if (p->small) {
        PassTimer t(p, 5, s);
        SGM_HIP_TRY(launch_small_pass(f, ft, p->sd, kSmallScalar, s));
        return SGM_OK;
    }
    sgm_status st = fourier_forward(p, f, ft, s);
    if (st != SGM_OK) return st;
    PassTimer t(p, 5, s);
    SGM_HIP_TRY(cheb_forward_pass(p, ft, kScalarProduct, s));
    return SGM_OK;
}

// Backward transform with the x pass writing into the spectral-sized workspace w
// (the plan's own, or the allocation-free entry point's static one).
static sgm_status backward_via(sgm_plan p, const void* u_hat, void* u, double2* w, hipStream_t s) {
    if (p->small) {
        PassTimer t(p, 6, s);
        SGM_HIP_TRY(launch_small_pass(u_hat, u, p->sd, kSmallBackward, s));
        return SGM_OK;
    }
    {
        PassTimer t(p, 6, s);
        if (p->leg)
            SGM_HIP_TRY(launch_leg_pass(p->leg_bwd, static_cast<const double*>(u_hat), reinterpret_cast<double*>(w), p->N,
                                        2L * p->geom.ncols, s));
        else if (p->hx)
            SGM_HIP_TRY(launch_k(p->rkx.cb, (p->geom.ncols + p->rkx.W - 1) / p->rkx.W, p->rkx.threads, p->rkx.lds, s,
                                 static_cast<const double2*>(u_hat), w, p->cd, p->geom.ncols, p->rpx.tw));
        else
            SGM_HIP_TRY(launch_cheb_bwd(static_cast<const double2*>(u_hat), w, p->cd, p->geom.ncols, p->W_cheb,
                                        p->rpx, s));
    }
    return fourier_backward(p, w, u, s);
}

sgm_status sgm_backward(sgm_plan p, const void* u_hat, void* u, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_backward");
    SGM_CHECK_ARG(p && u && u_hat, "null argument");
    SGM_CHECK_ARG(u != u_hat, "u and u_hat must not alias");
    return backward_via(p, u_hat, u, static_cast<double2*>(p->work), static_cast<hipStream_t>(stream));
}

sgm_status sgm_backward_noalloc(sgm_plan p, const void* u_hat, void* u, void* stream) {
    clear_error();
    SGM_CHECK_ARG(p && u && u_hat, "null argument");
    SGM_CHECK_ARG(u != u_hat, "u and u_hat must not alias");
    SGM_CHECK_ARG((size_t)p->nspec <= kNoAllocScratchElems,
                  "spectral array of %lld complex elements exceeds the allocation-free workspace (%zu elements, "
                  "%zu MiB)",
                  (long long)p->nspec, kNoAllocScratchElems, kNoAllocScratchElems * sizeof(double2) >> 20);
    double2* w = nullptr;
    sgm_status st = noalloc_scratch(&w);
    if (st != SGM_OK) return st;
    return backward_via(p, u_hat, u, w, static_cast<hipStream_t>(stream));
}

// Backward Fourier passes (middle axis in place, then the last axis) from the
// x-physical workspace w to u.
static sgm_status fourier_backward(sgm_plan p, double2* w, void* u, hipStream_t s) {
    if (p->ndim == 3) {
        PassTimer t(p, 3, s);
        const RegKernels& k = p->rky;
        if (p->hy)
            SGM_HIP_TRY(launch_strided(k, 1, w, w, p->N, p->spec_last, p->rpy.tw, 1.0, s));
        else
            SGM_HIP_TRY(launch_strided_c2c(w, w, p->M1, p->N, p->spec_last, p->W_mid, p->rpy, 1, 1.0, s));
    }
    int Llast = p->ndim == 3 ? p->M2 : p->M1;
    int nlines = p->ndim == 3 ? p->N * p->M1 : p->N;
    PassTimer t(p, 1, s);
    const RegKernels& k = p->rkz;
    if (p->r2c) {
        if (p->hz)
            SGM_HIP_TRY(launch_k(k.c2r, (nlines + 2 * k.W - 1) / (2 * k.W), k.threads, k.lds, s, (const double2*)w,
                                 static_cast<double*>(u), nlines, p->rpz.tw));
        else
            SGM_HIP_TRY(launch_lines_c2r(w, static_cast<double*>(u), Llast, nlines, p->G_last, p->rpz, s));
    } else {
        if (p->hz)
            SGM_HIP_TRY(launch_k(k.c2c_b, (nlines + k.W - 1) / k.W, k.threads, k.lds, s, (const double2*)w,
                                 static_cast<double2*>(u), nlines, p->rpz.tw, 1.0));
        else
            SGM_HIP_TRY(launch_lines_c2c(w, static_cast<double2*>(u), Llast, nlines, p->G_last, p->rpz, 1, 1.0, s));
    }
    return SGM_OK;
}

static bool helmholtz_basis(int basis) {
    return basis == SGM_SHEN_DIRICHLET || basis == SGM_LEG_DIRICHLET || basis == SGM_SHEN_NEUMANN ||
           basis == SGM_LEG_NEUMANN;
}

// Checks shared by the Helmholtz entry points: the basis, alpha >= 0, and for the
// Neumann basis alpha > 0 (at kappa = 0 and alpha = 0 the constant leaves the
// system singular).
static sgm_status helmholtz_args(sgm_plan p, double alpha) {
    SGM_CHECK_ARG(helmholtz_basis(p->d.basis),
                  "Helmholtz solve needs a Shen-Dirichlet or Shen-Neumann basis (Chebyshev or Legendre)");
    SGM_CHECK_ARG(alpha >= 0.0, "alpha must be >= 0 (got %g)", alpha);
    if ((p->d.basis == SGM_SHEN_NEUMANN || p->d.basis == SGM_LEG_NEUMANN) && alpha == 0.0) {
        set_error("Neumann basis: alpha = 0 leaves the constant mode of the zero wavenumber undetermined");
        return SGM_ERR_SINGULAR;
    }
    return SGM_OK;
}

// Segmented solve where the chains fit, else one lane per chain.  The
// boundary table is refilled (one extra launch) when alpha changes.
static sgm_status seg_table_for(sgm_plan p, int kind, double alpha, hipStream_t s);

static sgm_status solve_dispatch(sgm_plan p, int kind, double alpha, const void* f, void* u, hipStream_t s) {
    if (p->seg_K > 0) {
        sgm_status st = seg_table_for(p, kind, alpha, s);
        if (st != SGM_OK) return st;
        SGM_HIP_TRY(launch_solve_seg(static_cast<const double2*>(f), static_cast<double2*>(u), p->seg_tab, p->cd,
                                     p->geom, kind, p->seg_K, p->seg_R, alpha, s));
        return SGM_OK;
    }
    SGM_HIP_TRY(launch_solve_chain(static_cast<const double2*>(f), static_cast<double2*>(u),
                                   static_cast<double*>(p->work), p->cd, p->geom, table_kind(kind), alpha, s));
    return SGM_OK;
}

// Boundary-state table of the segmented solve for this alpha (refilled when alpha changes).
static sgm_status seg_table_for(sgm_plan p, int kind, double alpha, hipStream_t s) {
    if (!p->seg_ok || p->seg_alpha != alpha) {
        SGM_HIP_TRY(launch_seg_table(p->seg_tab, p->cd, p->geom, kind, p->seg_K, p->seg_R, alpha, s));
        p->seg_ok = true;
        p->seg_alpha = alpha;
    }
    return SGM_OK;
}

sgm_status sgm_helmholtz_solve_physical(sgm_plan p, double alpha, const void* f, void* u_hat, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_helmholtz_solve_physical");
    SGM_CHECK_ARG(p && f && u_hat, "null argument");
    SGM_CHECK_ARG(f != u_hat, "f and u_hat must not alias");
    sgm_status st = helmholtz_args(p, alpha);
    if (st != SGM_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double2* uh = static_cast<double2*>(u_hat);
    if (p->small) {
        {
            PassTimer t(p, 5, s);
            SGM_HIP_TRY(launch_small_pass(f, uh, p->sd, kSmallScalar, s));
        }
        return sgm_helmholtz_solve(p, alpha, uh, uh, stream);
    }
    st = fourier_forward(p, f, uh, s);
    if (st != SGM_OK) return st;
    if (p->d.basis == SGM_SHEN_DIRICHLET && p->hx && p->rkx.cf_spsolve && p->seg_K == 8 && p->seg_R == kSegRows &&
        p->d.autotune != 2) {
        if ((st = seg_table_for(p, SGM_SHEN_DIRICHLET, alpha, s)) != SGM_OK) return st;
        PassTimer t(p, 5, s);
        const RegKernels& k = p->rkx;
        SGM_HIP_TRY(launch_k(k.cf_spsolve, (p->geom.ncols + k.W - 1) / k.W, k.threads, k.lds_cheb, s,
                             (const double2*)uh, uh, p->cd, p->geom.ncols, p->rpx.tw,
                             ChebSolve{p->seg_tab, p->geom, alpha}));
        return SGM_OK;
    }
    {
        PassTimer t(p, 5, s);
        SGM_HIP_TRY(cheb_forward_pass(p, uh, kScalarProduct, s));
    }
    return sgm_helmholtz_solve(p, alpha, uh, uh, stream);
}

sgm_status sgm_helmholtz_solve(sgm_plan p, double alpha, const void* f_tilde, void* u_hat, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_helmholtz_solve");
    SGM_CHECK_ARG(p && f_tilde && u_hat, "null argument");
    {
        const sgm_status st = helmholtz_args(p, alpha);
        if (st != SGM_OK) return st;
    }
    PassTimer t(p, 7, static_cast<hipStream_t>(stream));
    if (p->d.autotune == 2)
        SGM_HIP_TRY(launch_solve(static_cast<const double2*>(f_tilde), static_cast<double2*>(u_hat), p->cd, p->geom,
                                 p->W_solve, table_kind(p->d.basis), alpha, static_cast<hipStream_t>(stream)));
    else
        return solve_dispatch(p, solve_kind(p->d.basis), alpha, f_tilde, u_hat, static_cast<hipStream_t>(stream));
    return SGM_OK;
}

sgm_status sgm_project_derivative(sgm_plan p, sgm_plan target, const int order[3], const void* u_hat, void* du_hat,
                                  void* stream) {
    clear_error();
    TraceRange trace_range("sgm_project_derivative");
    SGM_CHECK_ARG(p && target && order && u_hat && du_hat, "null argument");
    SGM_CHECK_ARG(u_hat != du_hat, "u_hat and du_hat must not alias");
    const sgm_plan_desc &a = p->d, &b = target->d;
    if (p->leg)
        SGM_CHECK_ARG(b.basis == SGM_LEGENDRE || b.basis == SGM_LEG_DIRICHLET || b.basis == SGM_LEG_NEUMANN,
                      "target basis of a Legendre-family space must be SGM_LEGENDRE, SGM_LEG_DIRICHLET or "
                      "SGM_LEG_NEUMANN");
    else
        SGM_CHECK_ARG(b.basis == SGM_CHEBYSHEV || b.basis == SGM_SHEN_DIRICHLET || b.basis == SGM_SHEN_NEUMANN,
                      "target basis must be SGM_CHEBYSHEV, SGM_SHEN_DIRICHLET or SGM_SHEN_NEUMANN");
    SGM_CHECK_ARG(a.ndim == b.ndim && p->N == target->N && p->M1 == target->M1 && p->M2 == target->M2 &&
                      a.kind_last == b.kind_last,
                  "target plan must have the same grid (ndim, N, M1, M2, kind_last)");
    const double twopi = 6.283185307179586476925286766559;
    auto per = [twopi](double L) { return L > 0 ? L : twopi; };
    SGM_CHECK_ARG(per(a.Ly) == per(b.Ly) && per(a.Lz) == per(b.Lz), "target plan must have the same periods");
    for (int i = 0; i < 3; ++i)
        SGM_CHECK_ARG(order[i] >= 0 && order[i] <= 8, "derivative order %d along axis %d outside 0..8", order[i], i);
    SGM_CHECK_ARG(a.ndim == 3 || order[2] == 0, "2D plan: order[2] must be 0");
    if (p->N > kDxMaxN) {
        set_error("derivative pass supports N <= %d (plan has %d)", kDxMaxN, p->N);
        return SGM_ERR_UNSUPPORTED_SIZE;
    }
    const DxArgs x = dx_args(p, p->cd.basis, b.basis, order[0], order[1], order[2]);
    SGM_HIP_TRY(launch_dx_project(static_cast<const double2*>(u_hat), static_cast<double2*>(du_hat), x,
                                  static_cast<hipStream_t>(stream)));
    return SGM_OK;
}

sgm_status sgm_biharmonic_solve(sgm_plan p, const void* f_tilde, void* u_hat, void* stream) {
    clear_error();
    TraceRange trace_range("sgm_biharmonic_solve");
    SGM_CHECK_ARG(p && f_tilde && u_hat, "null argument");
    SGM_CHECK_ARG(biharmonic_basis(p->d.basis), "biharmonic solve needs a Shen-biharmonic basis (Chebyshev or Legendre)");
    PassTimer t(p, 7, static_cast<hipStream_t>(stream));
    if (p->d.autotune == 2)
        SGM_HIP_TRY(launch_solve(static_cast<const double2*>(f_tilde), static_cast<double2*>(u_hat), p->cd, p->geom,
                                 p->W_solve, SGM_SHEN_BIHARMONIC, 0.0, static_cast<hipStream_t>(stream)));
    else
        return solve_dispatch(p, SGM_SHEN_BIHARMONIC, 0.0, f_tilde, u_hat, static_cast<hipStream_t>(stream));
    return SGM_OK;
}

}  // extern "C"
