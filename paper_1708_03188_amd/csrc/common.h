// Internal helpers shared by the libsgm translation units (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/sgm.h"

namespace sgm {

// Named range around one ABI call, for profilers (rocprofv3 --marker-trace);
// without a profiler attached the push and pop cost a few nanoseconds.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePush(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

// Thread-local detail string behind sgm_last_error().
void set_error(const char* fmt, ...);
void clear_error();

#define SGM_HIP_TRY(expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) {                                                            \
            ::sgm::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),        \
                             __FILE__, __LINE__);                                          \
            return SGM_ERR_HIP;                                                            \
        }                                                                                  \
    } while (0)

#define SGM_CHECK_ARG(cond, ...)                                                           \
    do {                                                                                   \
        if (!(cond)) {                                                                     \
            ::sgm::set_error(__VA_ARGS__);                                                 \
            return SGM_ERR_INVALID_ARG;                                                    \
        }                                                                                  \
    } while (0)

constexpr int kMaxStages = 24;

// Mixed-radix schedule of one FFT length; `tw` points at L twiddles
// exp(-2 pi i r / L), r = 0..L-1, in a plan-owned device table.
struct RadixPlan {
    int L;
    int nst;
    int radix[kMaxStages];
    const double2* tw;
};

// Factor L into the stage radices used by the LDS Stockham kernels.
// Powers of two become radix-8/4/2 stages, 3, 5 and 7 get their own
// codelets, any other prime factor runs through the generic radix-p path.
int factor_radices(int L, int* radix);

// Device-resident tables owned by a plan or a GL batch.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
};

}  // namespace sgm
