// Context, allocation and device primitives (scan, reductions) of ocpamg.
#include <cmath>
#include <cstdio>
#include <mutex>

#include "common.h"

namespace ocp {

void *dev_alloc(ocp_ctx *ctx, size_t bytes) {
    if (bytes == 0) return nullptr;
    void *p = nullptr;
    if (ctx->bump_base) {
        const size_t b = align256(bytes);
        if (ctx->bump_off + b > ctx->bump_cap)
            fail(OCP_ERR_UNSUPPORTED, "the solve needs more than the " + std::to_string(ctx->bump_cap >> 20) +
                                          " MiB scratch region of pcg_solve_noalloc");
        p = ctx->bump_base + ctx->bump_off;
        ctx->bump_off += b;
        return p;
    }
    if (ctx->alloc) {
        p = ctx->alloc(bytes, ctx->user);
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) p = nullptr;
    }
    if (!p) fail(OCP_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    return p;
}

void dev_free(ocp_ctx *ctx, void *p) {
    if (!p) return;
    if (ctx->bump_base && static_cast<char *>(p) >= ctx->bump_base &&
        static_cast<char *>(p) < ctx->bump_base + ctx->bump_cap)
        return;   // carved from the scratch region: nothing to release
    if (ctx->free_fn)
        ctx->free_fn(p, ctx->user);
    else
        (void)hipFree(p);
}

void sync(ocp_ctx *ctx) { OCP_HIP(hipStreamSynchronize(ctx->stream)); }

// ------------------------------------------------------- scratch region
// Device memory of pcg_solve_noalloc: one fixed array per GPU, held from the
// library's first use on that GPU until the process ends.  Host code never
// passes `scratch` itself anywhere (in host code the name is a host-side
// stand-in, not the device address): its device address is looked up once
// per device, with that device current, when a context is created there, and
// only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static void scratch_lookup(int device) {
    if (device < 0 || device >= kMaxDevices) fail(OCP_ERR_UNSUPPORTED, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void *p = nullptr;
    OCP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(OCP_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch region");
    g_scratch_ptr[device] = static_cast<char *>(p);
}

char *scratch_region(const ocp_ctx *ctx) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (ctx->device >= 0 && ctx->device < kMaxDevices) ? g_scratch_ptr[ctx->device] : nullptr;
}

void read_back(ocp_ctx *ctx, void *host, const void *dev, size_t bytes) {
    if (bytes > 4096) fail(OCP_ERR_INVALID_ARG, "read_back larger than the staging buffer");
    OCP_HIP(hipMemcpyAsync(ctx->pinned, dev, bytes, hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    std::memcpy(host, ctx->pinned, bytes);
}

// ------------------------------------------------------------------- fills
__global__ void k_fill_zero_u32(uint32_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0u;
}
__global__ void k_fill_zero_u8(uint8_t *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0u;
}

// Zero a device range with a kernel (no memset node, so it is safe inside a
// captured graph).
void fill_zero_bytes(ocp_ctx *ctx, void *p, size_t bytes) {
    if (!bytes) return;
    if ((reinterpret_cast<uintptr_t>(p) % 4 == 0) && bytes % 4 == 0) {
        int64_t n = (int64_t)(bytes / 4);
        unsigned g = grid_for(n, 256);
        if (g > 65536) g = 65536;
        k_fill_zero_u32<<<g, 256, 0, ctx->stream>>>(static_cast<uint32_t *>(p), n);
    } else {
        int64_t n = (int64_t)bytes;
        unsigned g = grid_for(n, 256);
        if (g > 65536) g = 65536;
        k_fill_zero_u8<<<g, 256, 0, ctx->stream>>>(static_cast<uint8_t *>(p), n);
    }
    OCP_LAUNCH_CHECK();
}

// -------------------------------------------------------------------- scan
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

// Block-wide exclusive scan of one int64 per thread; returns the exclusive
// prefix of this thread and the block total through *total.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *total) {
    __shared__ int64_t wsum[kScanBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int64_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int64_t woff = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanBlock / 64; ++w) {
        if (w < wid) woff += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return woff + inc - v;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_tile_sums(const int32_t *in, int64_t n,
                                                               int64_t *sums) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    int64_t tot;
    (void)block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of the tile sums in place, chunk by chunk.
__global__ void __launch_bounds__(kScanBlock) k_scan_sums(int64_t *sums, int64_t m, int64_t *total) {
    int64_t carry = 0;
    for (int64_t c = 0; c < m; c += kScanBlock) {
        int64_t i = c + threadIdx.x;
        int64_t v = i < m ? sums[i] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_scan(v, &tot);
        if (i < m) sums[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(const int32_t *in, int64_t n,
                                                           const int64_t *sums, int32_t *out,
                                                           const int64_t *total) {
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan(s, &tot) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = (int32_t)ex;
        ex += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (int32_t)*total;
}

int64_t scan_exclusive(ocp_ctx *ctx, const int32_t *in, int32_t *out, int64_t n) {
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles < 1) tiles = 1;
    DevBuf<int64_t> sums(ctx, (size_t)tiles + 1);
    int64_t *total = sums.get() + tiles;
    k_scan_tile_sums<<<(unsigned)tiles, kScanBlock, 0, ctx->stream>>>(in, n, sums.get());
    OCP_LAUNCH_CHECK();
    k_scan_sums<<<1, kScanBlock, 0, ctx->stream>>>(sums.get(), tiles, total);
    OCP_LAUNCH_CHECK();
    k_scan_apply<<<(unsigned)tiles, kScanBlock, 0, ctx->stream>>>(in, n, sums.get(), out, total);
    OCP_LAUNCH_CHECK();
    int64_t t = 0;
    read_back(ctx, &t, total, sizeof(t));
    if (t > INT32_MAX) fail(OCP_ERR_UNSUPPORTED, "prefix sum exceeds the int32 index range");
    return t;
}

// -------------------------------------------------------------- reductions
constexpr int kRedBlock = 256;

__global__ void __launch_bounds__(kRedBlock) k_max_abs(const double *v, int64_t n, double *partials) {
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kRedBlock)
        m = fmax(m, fabs(v[i]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    __shared__ double ws[kRedBlock / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kRedBlock / 64; ++w) m = fmax(m, ws[w]);
        partials[blockIdx.x] = m;
    }
}

// one block: max of the partials (a max is exact in any order)
__global__ void __launch_bounds__(kRedBlock) k_max_fin(const double *partials, unsigned nb, double *out) {
    double m = 0.0;
    for (unsigned b = threadIdx.x; b < nb; b += kRedBlock) m = fmax(m, partials[b]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    __shared__ double ws[kRedBlock / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kRedBlock / 64; ++w) m = fmax(m, ws[w]);
        *out = m;
    }
}

__global__ void __launch_bounds__(kRedBlock) k_dot(const double *a, const double *b, int64_t n,
                                                   double *partials, unsigned *counter, double *out) {
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kRedBlock)
        s += a[i] * b[i];
    s = dev::block_sum<kRedBlock>(s);
    double tot;
    if (dev::grid_sum_last<kRedBlock>(s, partials, counter, &tot) && threadIdx.x == 0) *out = tot;
}

static unsigned red_grid(int64_t n) {
    int64_t g = (n + kRedBlock - 1) / kRedBlock;
    if (g > kRedBlocks) g = kRedBlocks;
    if (g < 1) g = 1;
    return (unsigned)g;
}

double reduce_max_abs(ocp_ctx *ctx, const double *v, int64_t n) {
    const unsigned nb = red_grid(n);
    k_max_abs<<<nb, kRedBlock, 0, ctx->stream>>>(v, n, ctx->red_partials);
    k_max_fin<<<1, kRedBlock, 0, ctx->stream>>>(ctx->red_partials, nb, ctx->red_out);
    OCP_LAUNCH_CHECK();
    double r;
    read_back(ctx, &r, ctx->red_out, sizeof(r));
    return r;
}

double reduce_dot(ocp_ctx *ctx, const double *a, const double *b, int64_t n) {
    k_dot<<<red_grid(n), kRedBlock, 0, ctx->stream>>>(a, b, n, ctx->red_partials, ctx->red_counters,
                                                      ctx->red_out);
    OCP_LAUNCH_CHECK();
    double r;
    read_back(ctx, &r, ctx->red_out, sizeof(r));
    return r;
}

// ------------------------------------------------------------ kernel timing
static hipEvent_t pool_event(ocp_ctx *ctx) {
    if (!ctx->prof_pool.empty()) {
        hipEvent_t e = ctx->prof_pool.back();
        ctx->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    OCP_HIP(hipEventCreate(&e));
    return e;
}

int prof_begin(ocp_ctx *ctx, int kernel) {
    if (!ctx->profile) return -1;
    ocp_ctx::ProfRec r{kernel, ctx->prof_iter, pool_event(ctx), pool_event(ctx)};
    OCP_HIP(hipEventRecord(r.a, ctx->stream));
    ctx->prof_recs.push_back(r);
    return (int)ctx->prof_recs.size() - 1;
}

void prof_end(ocp_ctx *ctx, int rec) {
    if (rec < 0) return;
    OCP_HIP(hipEventRecord(ctx->prof_recs[rec].b, ctx->stream));
}

void prof_resolve(ocp_ctx *ctx, int valid_iters) {
    if (ctx->prof_recs.empty()) return;
    OCP_HIP(hipStreamSynchronize(ctx->stream));
    for (auto &r : ctx->prof_recs) {
        // iteration launches only: the initial application (iter -1) follows
        // the solve's allocations and its first event pair has been seen to
        // read several ms above the kernel's own duration in a trace
        if (r.iter >= 0 && r.iter < valid_iters && r.kernel >= 0 && r.kernel < 8) {
            float ms = 0.f;
            OCP_HIP(hipEventElapsedTime(&ms, r.a, r.b));
            ctx->prof_ms[r.kernel] += ms;
            ctx->prof_launches[r.kernel] += 1;
        }
        ctx->prof_pool.push_back(r.a);
        ctx->prof_pool.push_back(r.b);
    }
    ctx->prof_recs.clear();
}

}  // namespace ocp

using namespace ocp;

extern "C" int ocp_profile_enable(ocp_ctx *ctx, int32_t on) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    ctx->profile = on != 0;
    for (int k = 0; k < 8; ++k) {
        ctx->prof_ms[k] = 0.0;
        ctx->prof_launches[k] = 0;
    }
    return OCP_OK;
}

extern "C" int ocp_profile_read(ocp_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms) {
    if (!ctx || kernel < 0 || kernel >= 8 || !launches || !total_ms) return OCP_ERR_INVALID_ARG;
    *launches = ctx->prof_launches[kernel];
    *total_ms = ctx->prof_ms[kernel];
    return OCP_OK;
}

// ------------------------------------------------------------------- C-ABI
namespace {
template <typename F>
int guarded(ocp_ctx *ctx, F &&f) {
    try {
        f();
        if (ctx) ctx->last_error.clear();
        return OCP_OK;
    } catch (const Error &e) {
        if (ctx) ctx->last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        if (ctx) ctx->last_error = "host allocation failed";
        return OCP_ERR_OOM;
    } catch (...) {
        if (ctx) ctx->last_error = "unexpected internal error";
        return OCP_ERR_HIP;
    }
}
}  // namespace

extern "C" const char *ocp_version(void) { return "ocpamg 0.1 (gfx950)"; }

extern "C" int ocp_ctx_create(void *stream, ocp_alloc_fn alloc, ocp_free_fn free_fn, void *user,
                              ocp_ctx **out) {
    if (!out) return OCP_ERR_INVALID_ARG;
    *out = nullptr;
    if ((alloc == nullptr) != (free_fn == nullptr)) return OCP_ERR_INVALID_ARG;
    ocp_ctx *ctx = new (std::nothrow) ocp_ctx();
    if (!ctx) return OCP_ERR_OOM;
    ctx->stream = static_cast<hipStream_t>(stream);
    ctx->alloc = alloc;
    ctx->free_fn = free_fn;
    ctx->user = user;
    int rc = guarded(ctx, [&] {
        OCP_HIP(hipGetDevice(&ctx->device));
        scratch_lookup(ctx->device);   // the context's device is current here
        ctx->red_partials = static_cast<double *>(dev_alloc(ctx, sizeof(double) * kRedSlots * kRedBlocks));
        ctx->red_counters = static_cast<unsigned *>(dev_alloc(ctx, sizeof(unsigned) * 64));
        ctx->red_out = static_cast<double *>(dev_alloc(ctx, sizeof(double) * 64));
        ctx->cg = static_cast<CgScalars *>(dev_alloc(ctx, sizeof(CgScalars)));
        ctx->dev_flag = static_cast<int32_t *>(dev_alloc(ctx, sizeof(int32_t) * 64));
        fill_zero_bytes(ctx, ctx->red_counters, sizeof(unsigned) * 64);
        fill_zero_bytes(ctx, ctx->dev_flag, sizeof(int32_t) * 64);
        OCP_HIP(hipHostMalloc(&ctx->pinned, 4096, hipHostMallocDefault));
        OCP_HIP(hipEventCreate(&ctx->ev0));
        OCP_HIP(hipEventCreate(&ctx->ev1));
        sync(ctx);
    });
    if (rc != OCP_OK) {
        ocp_ctx_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return OCP_OK;
}

extern "C" void ocp_ctx_destroy(ocp_ctx *ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    dev_free(ctx, ctx->red_partials);
    dev_free(ctx, ctx->red_counters);
    dev_free(ctx, ctx->red_out);
    dev_free(ctx, ctx->cg);
    dev_free(ctx, ctx->dev_flag);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    for (auto &r : ctx->prof_recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->prof_pool) (void)hipEventDestroy(e);
    delete ctx;
}

extern "C" const char *ocp_last_error(const ocp_ctx *ctx) {
    return ctx ? ctx->last_error.c_str() : "null context";
}

// exported to the other translation units
namespace ocp {
int run_guarded(ocp_ctx *ctx, const std::function<void()> &f) {
    if (ctx && ctx->active_solve) {
        ctx->last_error = "a solve started with pcg_begin is active on this context (end it first)";
        return OCP_ERR_INVALID_ARG;
    }
    return guarded(ctx, f);
}
int run_step(ocp_ctx *ctx, const std::function<void()> &f) { return guarded(ctx, f); }
}  // namespace ocp
