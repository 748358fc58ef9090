// Shared host/device plumbing of the ocpamg library: the context, device
// allocations through the caller's allocator, error propagation, and the
// device-side reduction helpers (64-wide wavefronts on CDNA4).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "../../include/ocpamg.h"

namespace ocp {

// ------------------------------------------------------------------ errors
struct Error {
    int code;
    std::string msg;
};

[[noreturn]] inline void fail(int code, const std::string &msg) { throw Error{code, msg}; }

#define OCP_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            ::ocp::fail(OCP_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define OCP_LAUNCH_CHECK() OCP_HIP(hipGetLastError())

// Number of partial-sum slots a grid reduction may use (fixed grid size for
// the reduction kernels, so their summation order never depends on the GPU).
constexpr int kRedBlocks = 32768;
constexpr int kRedSlots = 8;  // independent reductions that may be in flight

// Device-resident scalars of one CG solve (one per context).
struct CgScalars {
    double ff;        // f.f
    double tol2;      // rtol^2 * (f.f or r0.z0)
    double gamma;     // r.z of the current iterate
    double gamma0;    // r0.z0
    double alpha, beta;
    double pq;        // p.Aq
    double rr;        // r.r
    double rz_new;    // r.z after the preconditioner
    double gamma_prev; // r.z of the previous iterate (flexible beta)
    int32_t flag;     // 0 running, 1 converged, 2 breakdown
    int32_t iter;     // completed iterations
    int32_t stop_mode;
    int32_t maxit;
};

}  // namespace ocp

struct ocp_ctx {
    hipStream_t stream = nullptr;
    ocp_alloc_fn alloc = nullptr;
    ocp_free_fn free_fn = nullptr;
    void *user = nullptr;
    int device = 0;
    std::string last_error;
    // reduction scratch
    double *red_partials = nullptr;     // [kRedSlots][kRedBlocks]
    unsigned *red_counters = nullptr;   // [kRedSlots]
    double *red_out = nullptr;          // [kRedSlots] results
    ocp::CgScalars *cg = nullptr;       // device scalars
    void *pinned = nullptr;             // small pinned host staging buffer (4 KiB)
    int32_t *dev_flag = nullptr;        // general device error/overflow flag
    bool active_solve = false;          // a step-API solve holds the CG scalars
    // pcg_solve_noalloc: while set, device buffers are carved in order from
    // [bump_base, bump_base + bump_cap) instead of coming from the allocator
    char *bump_base = nullptr;
    size_t bump_cap = 0, bump_off = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // live kernel timing (ocp_profile_enable): event pairs around selected
    // launches, resolved after each solve
    bool profile = false;
    int prof_iter = 0;                       // host iteration tag of new records
    struct ProfRec { int kernel; int iter; hipEvent_t a, b; };
    std::vector<ProfRec> prof_recs;
    std::vector<hipEvent_t> prof_pool;
    double prof_ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t prof_launches[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

namespace ocp {

// --------------------------------------------------------------- allocation
void *dev_alloc(ocp_ctx *ctx, size_t bytes);
void dev_free(ocp_ctx *ctx, void *p);
// Scratch region of the allocation-free solve on the context's device (the
// library's fixed-size device array, looked up at context creation).
char *scratch_region(const ocp_ctx *ctx);
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Owning device buffer allocated through the context's allocator.
template <typename T>
struct DevBuf {
    ocp_ctx *ctx = nullptr;
    T *ptr = nullptr;
    size_t count = 0;
    DevBuf() = default;
    DevBuf(ocp_ctx *c, size_t n) { reset(c, n); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept { swap(o); }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            swap(o);
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void swap(DevBuf &o) noexcept {
        std::swap(ctx, o.ctx);
        std::swap(ptr, o.ptr);
        std::swap(count, o.count);
    }
    void reset(ocp_ctx *c, size_t n) {
        release();
        ctx = c;
        count = n;
        ptr = n ? static_cast<T *>(dev_alloc(c, n * sizeof(T))) : nullptr;
    }
    void release() {
        if (ptr) dev_free(ctx, ptr);
        ptr = nullptr;
        count = 0;
    }
    T *get() const { return ptr; }
    size_t size() const { return count; }
};

// Copy a few bytes device -> host through the pinned staging buffer and wait.
void read_back(ocp_ctx *ctx, void *host, const void *dev, size_t bytes);
void sync(ocp_ctx *ctx);

// Column source of a sliced-ELL pass: plain columns, or (code != nullptr)
// 4-bit codes into the slice's dictionary of column offsets.
struct SellCols {
    const int32_t *col;
    const uint32_t *code;
    const int32_t *cp;
    const int32_t *dict;
};

inline unsigned grid_for(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    return (unsigned)(g < 1 ? 1 : g);
}

// --------------------------------------------------------------- primitives
// Exclusive prefix sum of n int32 counts into out[0..n] (out[n] = total).
// Returns the total (synchronizes).
int64_t scan_exclusive(ocp_ctx *ctx, const int32_t *in, int32_t *out, int64_t n);
// Device max / sum of n doubles into a host value (synchronizes).
double reduce_max_abs(ocp_ctx *ctx, const double *v, int64_t n);
double reduce_dot(ocp_ctx *ctx, const double *a, const double *b, int64_t n);
void fill_zero_bytes(ocp_ctx *ctx, void *p, size_t bytes);

// Live kernel timing: prof_begin/prof_end bracket one launch (no-ops unless
// profiling is on); prof_resolve adds the durations of records whose host
// iteration tag is below `valid_iters` and recycles the events.
int prof_begin(ocp_ctx *ctx, int kernel);
void prof_end(ocp_ctx *ctx, int rec);
void prof_resolve(ocp_ctx *ctx, int valid_iters);

// Run f, turning internal errors into a status code and ctx->last_error.
// Refused while a step-API solve (pcg_begin .. pcg_end) holds the context.
int run_guarded(ocp_ctx *ctx, const std::function<void()> &f);
// The same without that check, for the step API's own calls.
int run_step(ocp_ctx *ctx, const std::function<void()> &f);

}  // namespace ocp

// ------------------------------------------------------------ device helpers
#ifdef __HIPCC__
namespace ocp {
namespace dev {

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over `G` consecutive lanes (G a power of two <= 64); result in all of them.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// Block-wide sum in a fixed order (wave sums, then wave 0 adds them in order).
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double ws[BLOCK / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) ws[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) s += ws[w];
    }
    __syncthreads();
    return s;  // valid in thread 0
}

// Grid reduction epilogue.  Every block calls this once with its block
// partial (valid in thread 0).  The last block to arrive sums the partials
// in block order -- a fixed order, so the result is bitwise reproducible --
// and returns true in all of its threads with *total set in thread 0.
template <int BLOCK>
__device__ __forceinline__ bool grid_sum_last(double block_partial, double *partials,
                                              unsigned *counter, double *total) {
    __shared__ bool am_last;
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = block_partial;
        __threadfence();
        unsigned t = atomicAdd(counter, 1u);
        am_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!am_last) return false;
    __threadfence();
    double s = 0.0;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += BLOCK)
        s += __hip_atomic_load(&partials[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s = block_sum<BLOCK>(s);
    if (threadIdx.x == 0) {
        *total = s;
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return true;
}

}  // namespace dev
}  // namespace ocp
#endif
