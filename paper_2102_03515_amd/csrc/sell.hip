// Conversion of the fine-level CSR matrix to sliced ELLPACK (64-row slices).
#include <algorithm>
#include <climits>

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

// Column codes, one wavefront per slice (sell_code_regs): the entries'
// offsets col - row are read back from the slice's columns.
template <int MAXW>
__device__ __forceinline__ void sell_code_slice(int64_t s, int w, int rr, int lane, int64_t base,
                                                const int32_t *__restrict__ scol, const int32_t *__restrict__ cp,
                                                uint32_t *__restrict__ code, int32_t *__restrict__ dict,
                                                int32_t *overflow) {
    int d[MAXW];
#pragma unroll
    for (int j = 0; j < MAXW; ++j) d[j] = j < w ? scol[base + (int64_t)j * kSellC] - rr : 0;
    dev::sell_code_regs<MAXW>(s, w, lane, d, cp, code, dict, overflow);
}

__global__ void __launch_bounds__(256) k_sell_code(int32_t n, int64_t nslices, const int32_t *__restrict__ sp,
                                                   const int32_t *__restrict__ sw, const int32_t *__restrict__ scol,
                                                   const int32_t *__restrict__ cp, uint32_t *__restrict__ code,
                                                   int32_t *__restrict__ dict, int32_t *overflow) {
    const int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSellC;
    const int lane = threadIdx.x & 63;
    if (s >= nslices) return;   // uniform over the wavefront
    const int w = sw[s];
    const int row = (int)(s * kSellC) + lane;
    const int rr = row < n ? row : 0;
    const int64_t base = sp[s] + lane;
    if (w <= 16)
        sell_code_slice<16>(s, w, rr, lane, base, scol, cp, code, dict, overflow);
    else if (w <= 32)
        sell_code_slice<32>(s, w, rr, lane, base, scol, cp, code, dict, overflow);
    else if (lane == 0)
        atomicOr(overflow, 1);   // wider slices stay uncoded
}

__global__ void k_sell_code_words(int64_t nslices, const int32_t *__restrict__ sw, int32_t *__restrict__ words) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nslices) words[s] = (sw[s] + 7) / 8 * kSellC;
}

// Slice widths and offsets of the CSR matrix, with the column and value
// arrays allocated (filled by sell_build or by the caller).
void sell_layout(ocp_ctx *ctx, Sell &S, int32_t n, const int32_t *rp) {
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
}

// Code words, offsets and dictionaries of a slice layout, allocated, with
// the overflow flag cleared (the codes themselves follow).
void sell_code_layout(ocp_ctx *ctx, Sell &S) {
    DevBuf<int32_t> words(ctx, (size_t)S.nslices + 1);
    k_sell_code_words<<<grid_for(S.nslices, 256), 256, 0, ctx->stream>>>(S.nslices, S.sw.get(), words.get());
    OCP_LAUNCH_CHECK();
    S.cp.reset(ctx, (size_t)S.nslices + 1);
    const int64_t nwords = scan_exclusive(ctx, words.get(), S.cp.get(), S.nslices);
    S.code.reset(ctx, (size_t)std::max<int64_t>(nwords, 1));
    S.dict.reset(ctx, (size_t)S.nslices * kSellDict);
    fill_zero_bytes(ctx, ctx->dev_flag, sizeof(int32_t));
}

// Codes are kept only if every slice fitted the dictionary.
void sell_code_finish(ocp_ctx *ctx, Sell &S) {
    int32_t over = 0;
    read_back(ctx, &over, ctx->dev_flag, sizeof(over));
    if (over) {
        S.code.release();
        S.cp.release();
        S.dict.release();
    }
}

// Column codes of filled slices.
void sell_codes(ocp_ctx *ctx, Sell &S) {
    sell_code_layout(ctx, S);
    k_sell_code<<<grid_for((int64_t)S.nslices * kSellC, 256), 256, 0, ctx->stream>>>(
        S.n, S.nslices, S.sp.get(), S.sw.get(), S.col.get(), S.cp.get(), S.code.get(), S.dict.get(), ctx->dev_flag);
    OCP_LAUNCH_CHECK();
    sell_code_finish(ctx, S);
}

// The whole sliced-ELL copy of a CSR matrix: layout, columns and values, codes.
void sell_build(ocp_ctx *ctx, Sell &S, int32_t n, const int32_t *rp, const int32_t *col, const double *val) {
    sell_layout(ctx, S, n, rp);
    k_sell_fill<double><<<grid_for((int64_t)S.nslices * kSellC, 256), 256, 0, ctx->stream>>>(
        n, S.nslices, rp, col, val, S.sp.get(), S.sw.get(), S.col.get(), S.val.get());
    OCP_LAUNCH_CHECK();
    sell_codes(ctx, S);
}

// Single-precision values of an existing slice structure.
void sell_values32(ocp_ctx *ctx, const Sell &S, const int32_t *rp, const float *val32, DevBuf<float> &out) {
    out.reset(ctx, (size_t)S.nnz_padded);
    k_sell_fill<float><<<grid_for((int64_t)S.nslices * kSellC, 256), 256, 0, ctx->stream>>>(
        S.n, S.nslices, rp, nullptr, val32, S.sp.get(), S.sw.get(), nullptr, out.get());
    OCP_LAUNCH_CHECK();
}

}  // namespace ocp
