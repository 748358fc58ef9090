// Conversion of the fine-level CSR matrix to sliced ELLPACK (64-row slices).
#include "kernels.h"
#include "system.h"

namespace ocp {

// width of every slice = its longest row
__global__ void k_sell_widths(int32_t n, const int32_t *__restrict__ rp, int32_t *__restrict__ w64) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int len = t < n ? rp[t + 1] - rp[t] : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const int v = __shfl_xor(len, o, 64);
        len = v > len ? v : len;
    }
    if (lane == 0) w64[t / kSellC] = len * kSellC;
}

__global__ void k_sell_slice_w(int64_t nslices, const int32_t *__restrict__ w64, int32_t *__restrict__ w) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nslices) w[s] = w64[s] / kSellC;
}

template <typename VT>
__global__ void k_sell_fill(int32_t n, int64_t nslices, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                            const VT *__restrict__ val, const int32_t *__restrict__ sp, const int32_t *__restrict__ sw,
                            int32_t *__restrict__ scol, VT *__restrict__ sval) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = t / kSellC;
    const int lane = (int)(t % kSellC);
    if (s >= nslices) return;
    const int row = (int)t;
    const int b = row < n ? rp[row] : 0;
    const int len = row < n ? rp[row + 1] - b : 0;
    const int64_t base = sp[s] + lane;
    const int w = sw[s];
    // eight entries of the row are read before they are written (the reads
    // of a lane are scattered across rows; the writes of a wavefront are
    // consecutive)
    constexpr int U = 8;
    for (int j0 = 0; j0 < w; j0 += U) {
        int c[U];
        VT v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u;
            const bool in = j < len;
            c[u] = (in && scol) ? col[b + j] : (row < n ? row : 0);
            v[u] = in ? val[b + j] : VT(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int j = j0 + u;
            if (j < w) {
                if (scol) scol[base + (int64_t)j * kSellC] = c[u];
                sval[base + (int64_t)j * kSellC] = v[u];
            }
        }
    }
}

// Build the slice structure and column array (values follow with sell_values).
void sell_build(ocp_ctx *ctx, Sell &S, int32_t n, const int32_t *rp, const int32_t *col, const double *val) {
    S.n = n;
    S.nslices = (n + kSellC - 1) / kSellC;
    DevBuf<int32_t> w64(ctx, (size_t)S.nslices + 1);
    k_sell_widths<<<grid_for((int64_t)S.nslices * kSellC, 256), 256, 0, ctx->stream>>>(n, rp, w64.get());
    OCP_LAUNCH_CHECK();
    S.sw.reset(ctx, (size_t)S.nslices);
    k_sell_slice_w<<<grid_for(S.nslices, 256), 256, 0, ctx->stream>>>(S.nslices, w64.get(), S.sw.get());
    OCP_LAUNCH_CHECK();
    S.sp.reset(ctx, (size_t)S.nslices + 1);
    S.nnz_padded = scan_exclusive(ctx, w64.get(), S.sp.get(), S.nslices);
    S.col.reset(ctx, (size_t)S.nnz_padded);
    S.val.reset(ctx, (size_t)S.nnz_padded);
    k_sell_fill<double><<<grid_for((int64_t)S.nslices * kSellC, 256), 256, 0, ctx->stream>>>(
        n, S.nslices, rp, col, val, S.sp.get(), S.sw.get(), S.col.get(), S.val.get());
    OCP_LAUNCH_CHECK();
}

// Single-precision values of an existing slice structure.
void sell_values32(ocp_ctx *ctx, const Sell &S, const int32_t *rp, const float *val32, DevBuf<float> &out) {
    out.reset(ctx, (size_t)S.nnz_padded);
    k_sell_fill<float><<<grid_for((int64_t)S.nslices * kSellC, 256), 256, 0, ctx->stream>>>(
        S.n, S.nslices, rp, nullptr, val32, S.sp.get(), S.sw.get(), nullptr, out.get());
    OCP_LAUNCH_CHECK();
}

}  // namespace ocp
