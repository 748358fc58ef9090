// Device building blocks shared by the SpMV, CG and V-cycle kernels.
//
// Rows are processed by groups of G consecutive lanes of a 64-wide wavefront
// (G = 4/8/16/32/64), each lane striding over the row's entries and the group
// reducing with cross-lane shuffles.  A block of 256 threads handles a tile of
// consecutive rows; tiles are assigned to blocks so that the 8 XCDs (which
// receive blocks round-robin) each stream one contiguous slab of rows, which
// keeps the gathered x-vector entries of a slab in that XCD's L2.
// Matrix values and column indices are read with non-temporal loads so that
// the single-use matrix stream does not evict the reused x-vector from cache.
#pragma once

#include <climits>
#include "common.h"

namespace ocp {

constexpr int kBlock = 256;
constexpr int kMaxPartials = 16384;   // per reduction slot

struct RowLaunch {
    unsigned blocks;
    int iters;       // row passes per block
    int rows_per_pass;
};

// Tile shape for n rows with G lanes per row: at most kMaxPartials/2 blocks so
// that the grid reductions stay cheap.
inline RowLaunch row_launch(int64_t n, int G) {
    RowLaunch L;
    L.rows_per_pass = kBlock / G;
    const int64_t max_blocks = kMaxPartials / 2;
    int64_t iters = (n + (int64_t)L.rows_per_pass * max_blocks - 1) / ((int64_t)L.rows_per_pass * max_blocks);
    if (iters < 1) iters = 1;
    L.iters = (int)iters;
    int64_t rows_per_block = (int64_t)L.rows_per_pass * L.iters;
    int64_t b = (n + rows_per_block - 1) / rows_per_block;
    L.blocks = (unsigned)(b < 1 ? 1 : b);
    return L;
}

// Elementwise tile shape: one element per thread and pass.
inline RowLaunch vec_launch(int64_t n) { return row_launch(n, 1); }

#ifdef __HIPCC__
namespace dev {

// Logical tile of physical block b: XCD x = b mod 8 gets a contiguous run of
// tiles.  A bijection on [0, nb) for any nb.
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned nb) {
    const unsigned q = nb >> 3, r = nb & 7u, x = b & 7u, k = b >> 3;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

template <typename T>
__device__ __forceinline__ T ldnt(const T *p) {
    return __builtin_nontemporal_load(p);
}

// sum_k val[k] * xf(col[k]) over one row, by G lanes; result in every lane of
// the group.  Accumulates in the value type.
// With few lanes per row each lane requests U of its entries (and their
// gathers) before the first product; entries past the row re-read its last
// entry (in bounds) and are left out, so every lane still adds its products
// in entry order.  Wide groups (long rows) keep one entry per step, which
// measured faster there.
template <int G, typename VT, typename XF>
__device__ __forceinline__ VT row_sum(int rb, int re, int lane, const int32_t *__restrict__ col,
                                      const VT *__restrict__ val, XF xf) {
    constexpr int U = G <= 8 ? 4 : 1;
    VT s = VT(0);
    for (int k0 = rb + lane; k0 < re; k0 += U * G) {
        int c[U];
        VT v[U], x[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * G < re ? k0 + u * G : re - 1;
            c[u] = ldnt(col + k);
            v[u] = ldnt(val + k);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = xf(c[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * G < re) s += v[u] * x[u];
    }
    return group_sum<G>(s);
}

// Two block partials summed at once (fixed order), valid in thread 0.
template <int BLOCK>
__device__ __forceinline__ double2 block_sum2(double a, double b) {
    __shared__ double ws[2][BLOCK / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        ws[0][wid] = a;
        ws[1][wid] = b;
    }
    __syncthreads();
    double2 s = make_double2(0.0, 0.0);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) {
            s.x += ws[0][w];
            s.y += ws[1][w];
        }
    }
    __syncthreads();
    return s;
}

// Grid sum of two values: as grid_sum_last, with partials[2*b], partials[2*b+1].
template <int BLOCK>
__device__ __forceinline__ bool grid_sum2_last(double2 bp, double *partials, unsigned *counter, double2 *total) {
    __shared__ bool am_last;
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = bp.x;
        partials[2 * blockIdx.x + 1] = bp.y;
        __threadfence();
        unsigned t = atomicAdd(counter, 1u);
        am_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!am_last) return false;
    __threadfence();
    double a = 0.0, b = 0.0;
    for (unsigned k = threadIdx.x; k < gridDim.x; k += BLOCK) {
        a += __hip_atomic_load(&partials[2 * k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        b += __hip_atomic_load(&partials[2 * k + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    double2 s = block_sum2<BLOCK>(a, b);
    if (threadIdx.x == 0) {
        *total = s;
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return true;
}

// Block partials of a grid reduction: thread 0 stores the block's value
// (valid in thread 0) with a plain store; a one-block finalize kernel
// launched next on the stream sums them in block order.  (A last-block
// epilogue would need an agent-scope release fence in every block, which
// writes back the XCD's L2 each time.)
__device__ __forceinline__ void store_partial(double v, double *partials) {
    if (threadIdx.x == 0) partials[blockIdx.x] = v;
}
__device__ __forceinline__ void store_partial2(double2 v, double *partials) {
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = v.x;
        partials[2 * blockIdx.x + 1] = v.y;
    }
}

// Sum of nb partials in a fixed order (one block of kBlock threads; result
// valid in thread 0).
template <int BLOCK>
__device__ __forceinline__ double sum_partials(const double *partials, unsigned nb, int stride = 1, int off = 0) {
    // four independent loads in flight per thread
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    unsigned b = threadIdx.x;
    for (; b + 3 * BLOCK < nb; b += 4 * BLOCK) {
#pragma unroll
        for (int u = 0; u < 4; ++u) s[u] += partials[(size_t)(b + u * BLOCK) * stride + off];
    }
    for (; b < nb; b += BLOCK) s[0] += partials[(size_t)b * stride + off];
    return block_sum<BLOCK>((s[0] + s[1]) + (s[2] + s[3]));
}

}  // namespace dev

// The V-cycle's first smoothing step from zero, y = a D^-1 r, in the
// hierarchy's precision: written by the kernels that produce r, so that the
// first pass of the cycle gathers this vector (4 bytes per entry in mixed
// precision) instead of rebuilding a d_j r_j from r and d for every matrix
// entry.  y == nullptr: not wanted.
template <typename YT>
struct FirstStep {
    YT *y;
    const YT *d;
    YT a;
    __device__ __forceinline__ void put(size_t e, int row, double r) const {
        if (y) y[e] = a * d[row] * (YT)r;
    }
};

namespace dev {
// After r.z of the new preconditioned residual is known (thread 0 of the
// last block): beta = rz / gamma, gamma = rz; first call records gamma0; the
// preconditioned stop test and the breakdown test live here.
__device__ __forceinline__ void cg_after_precond(CgScalars *cg, double rz) {
    if (cg->iter == 0) cg->gamma0 = rz;
    if (!(rz > 0.0) || !isfinite(rz)) {
        cg->flag = (rz == 0.0 && cg->rr == 0.0) ? 1 : 2;
        cg->beta = 0.0;
        return;
    }
    cg->beta = (cg->iter == 0) ? 0.0 : rz / cg->gamma;
    cg->gamma_prev = cg->gamma;
    cg->gamma = rz;
    cg->rz_new = rz;
    if (cg->stop_mode == OCP_STOP_PRECOND) {
        if (cg->iter == 0) cg->tol2 = cg->tol2 * rz;   // tol2 held rtol^2 until now
        else if (rz <= cg->tol2) cg->flag = 1;
    }
}

}  // namespace dev
#endif
}  // namespace ocp

// ------------------------------------------------------------ sliced ELL
// Fine-level copy of a CSR matrix in sliced ELLPACK with slices of 64 rows
// (one wavefront): entry j of row 64*s + lane sits at ptr[s] + 64*j + lane,
// slice s has width w[s] = its longest row, shorter rows are padded with
// value 0 and column = the row itself.  A thread owns a row; each load
// instruction of a wavefront reads 64 consecutive entries, and a thread
// issues the loads of a whole chunk of its row before consuming them.
namespace ocp {

constexpr int kFinBlock = 1024;   // one-block finalize kernels over the partials of a SELL pass
constexpr int kSellC = 64;
constexpr int kSellDict = 16;     // column offsets per slice that 4-bit codes can name
namespace dev {
// Column codes of one slice from its entries' offsets d[j] = col - row (j <
// w, the slice width; every lane of the wavefront takes part).  The distinct
// offsets are found smallest first (a wavefront minimum over the entries not
// yet named, repeated), so the dictionary is ascending; more than kSellDict
// of them sets *overflow and leaves the slice uncoded.  d is overwritten with
// the codes.
template <int MAXW>
__device__ __forceinline__ void sell_code_regs(int64_t s, int w, int lane, int (&d)[MAXW],
                                               const int32_t *__restrict__ cp, uint32_t *__restrict__ code,
                                               int32_t *__restrict__ dict, int32_t *overflow) {
    uint32_t done = 0;   // entries already named
    int nd = 0, mine = 0;
    for (;;) {
        int m = INT_MAX;
#pragma unroll
        for (int j = 0; j < MAXW; ++j)
            if (j < w && !((done >> j) & 1u) && d[j] < m) m = d[j];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int v = __shfl_xor(m, o, 64);
            m = v < m ? v : m;
        }
        if (m == INT_MAX) break;   // every entry named
        if (nd == kSellDict) {
            if (lane == 0) atomicOr(overflow, 1);
            return;
        }
        if (lane == nd) mine = m;
#pragma unroll
        for (int j = 0; j < MAXW; ++j)
            if (j < w && !((done >> j) & 1u) && d[j] == m) {
                done |= 1u << j;
                d[j] = nd;   // the entry's code from here on
            }
        ++nd;
    }
    if (lane < kSellDict) dict[s * kSellDict + lane] = lane < nd ? mine : 0;
    const int64_t cb = cp[s] + lane;
#pragma unroll
    for (int q = 0; q < (MAXW + 7) / 8; ++q) {
        if (q * 8 >= w) break;
        uint32_t word = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int j = q * 8 + u;
            if (j < w) word |= (uint32_t)d[j] << (4 * u);
        }
        code[cb + (int64_t)q * kSellC] = word;
    }
}
}  // namespace dev

namespace dev {
// bitonic sort of 16 (key, value) register pairs by key; unused keys are INT_MAX
__device__ __forceinline__ void sort_slots(int (&keys)[16], double (&acc)[16]) {
    constexpr int S = 16;
#pragma unroll
    for (int kk = 2; kk <= S; kk <<= 1)
#pragma unroll
        for (int jj = kk >> 1; jj > 0; jj >>= 1)
#pragma unroll
            for (int q = 0; q < S; ++q) {
                const int l = q ^ jj;
                if (l > q) {
                    const bool up = (q & kk) == 0;
                    const bool sw = up ? (keys[q] > keys[l]) : (keys[q] < keys[l]);
                    const int tk = keys[q];
                    const double tv = acc[q];
                    keys[q] = sw ? keys[l] : keys[q];
                    acc[q] = sw ? acc[l] : acc[q];
                    keys[l] = sw ? tk : keys[l];
                    acc[l] = sw ? tv : acc[l];
                }
            }
}
}  // namespace dev

constexpr int kSellMinRows = 1 << 16;   // coarse levels from this size get a sliced-ELL copy
constexpr int kSellChunk = 16;
static_assert(kSellChunk == 16, "the coded row reads two code words per chunk");

struct SellLaunch {
    unsigned blocks;
    int slices_per_block;   // multiple of kBlock / kSellC
};

// One slice per wavefront while the grid stays within the partial slots of
// a reduction (kRedBlocks - 1 blocks; the last slot may hold the total):
// short per-wave work keeps the most independent loads in flight.
inline SellLaunch sell_launch(int64_t nslices) {
    constexpr int WPB = kBlock / kSellC;
    const int64_t max_blocks = kRedBlocks - 1;
    int64_t spb = (nslices + max_blocks - 1) / max_blocks;
    spb = ((spb + WPB - 1) / WPB) * WPB;
    if (spb < WPB) spb = WPB;
    SellLaunch L;
    L.slices_per_block = (int)spb;
    int64_t b = (nslices + spb - 1) / spb;
    L.blocks = (unsigned)(b < 1 ? 1 : b);
    return L;
}

#ifdef __HIPCC__
namespace dev {

// sum_j val * xf(col) over the row held by this lane of slice (base = its
// offset); w is the slice width (uniform over the wavefront).  A chunk's
// loads and gathers are all issued before its first product: entries past w
// re-read entry w-1 (cached, in bounds) and are left out of the sum, which
// adds the products in entry order.
template <typename VT, typename XF>
__device__ __forceinline__ VT sell_row(const int32_t *__restrict__ col, const VT *__restrict__ val, int64_t base,
                                       int w, XF xf) {
    w = __builtin_amdgcn_readfirstlane(w);
    VT acc = VT(0);
    for (int j0 = 0; j0 < w; j0 += kSellChunk) {
        int c[kSellChunk];
        VT v[kSellChunk], x[kSellChunk];
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) {
            const int jj = j0 + j < w ? j0 + j : w - 1;
            c[j] = ldnt(col + base + (int64_t)jj * kSellC);
            v[j] = ldnt(val + base + (int64_t)jj * kSellC);
        }
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) x[j] = xf(c[j]);
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j)
            if (j0 + j < w) acc += v[j] * x[j];
    }
    return acc;
}

// sell_row over either column source; the coded form adds the same terms in
// the same order (the same result bits) and reads half a byte per entry
// instead of four.  w is uniform over the wavefront, so every lane takes
// part in each shuffle.
template <typename VT, typename XF>
__device__ __forceinline__ VT sell_row_c(const SellCols &C, int64_t slice, int row, int n,
                                         const VT *__restrict__ val, int64_t base, int w, XF xf) {
    if (!C.code) return sell_row(C.col, val, base, w, xf);
    w = __builtin_amdgcn_readfirstlane(w);
    const int lane = threadIdx.x & 63;
    const int rr = row < n ? row : 0;   // lanes past the last row hold offset 0 from row 0
    const int dl = C.dict[slice * kSellDict + (lane & (kSellDict - 1))];
    const int64_t cb = C.cp[slice] + lane;
    VT acc = VT(0);
    for (int j0 = 0; j0 < w; j0 += kSellChunk) {
        uint32_t cw[kSellChunk / 8];
        VT v[kSellChunk], x[kSellChunk];
#pragma unroll
        for (int q = 0; q < kSellChunk / 8; ++q) {
            const int qq = j0 + 8 * q < w ? j0 / 8 + q : (w - 1) / 8;
            cw[q] = ldnt(C.code + cb + (int64_t)qq * kSellC);
        }
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) {
            const int jj = j0 + j < w ? j0 + j : w - 1;
            v[j] = ldnt(val + base + (int64_t)jj * kSellC);
        }
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) {
            // entry j of the chunk, or past w entry w-1, which lies in this
            // (last) chunk
            const int jj = j0 + j < w ? j : w - 1 - j0;
            const uint32_t word = (jj >> 3) ? cw[1] : cw[0];
            const int c = (int)((word >> (4 * (jj & 7))) & 15u);
            x[j] = xf(rr + __shfl(dl, c, 64));
        }
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j)
            if (j0 + j < w) acc += v[j] * x[j];
    }
    return acc;
}

}  // namespace dev
#endif
}  // namespace ocp

// Loop header for SELL kernels: `row` and `base` for each slice this
// wavefront owns (slices contiguous per XCD), `lane` = lane in the slice.
#define OCP_SELL_BEGIN(nslices, spb)                                                 \
    const unsigned tile_ = ::ocp::dev::xcd_tile(blockIdx.x, gridDim.x);              \
    const int lane = threadIdx.x & 63, wv_ = threadIdx.x >> 6;                       \
    for (int s0_ = 0; s0_ < (spb); s0_ += ::ocp::kBlock / ::ocp::kSellC) {            \
        const int64_t slice = (int64_t)tile_ * (spb) + s0_ + wv_;                    \
        if (slice >= (nslices)) break;                                               \
        const int w = sw[slice];                                                     \
        const int64_t base = sp[slice] + lane;                                       \
        const int row = (int)(slice * ::ocp::kSellC) + lane;
#define OCP_SELL_END() }
