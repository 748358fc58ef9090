// Block (multi right-hand side) PCG: k independent CG recurrences that share
// one matrix and one AMG hierarchy (Section 4's PCG with one V-cycle as
// preconditioner, applied to k load vectors at once).
//
// Vectors of the block are stored row-major, entry (i, j) at i*k + j, so that
// the k values of a row are contiguous.  A row is handled by a group of KB
// lanes (KB = 8/16/32/64): in the elementwise kernels lane j owns column j;
// in the kernels that gather neighbouring rows (the SpMM and the V-cycle
// passes) each lane owns VW consecutive columns when k is a multiple of VW
// (2 in FP64, 4 in FP32), so that every gather is one 16-byte access -- a
// wavefront's load instruction costs the same address-processing time
// whatever its width, and these kernels issue one per matrix entry.  Every
// matrix entry is staged once per group and multiplies k gathered values
// that sit next to each other in memory.  The matrix stream is therefore
// read once per k right-hand sides; the vector streams are what scale with
// k.
//
// Every column has its own alpha, beta, gamma and stop flag on the device.  A
// column that has converged (or broken down, or hit the cap) is frozen: the
// CG kernels leave its X, R and P alone, so they keep their final values
// (the gather kernels still compute it, into work vectors and partial sums
// that a frozen column no longer reads).  The
// V-cycle is the same polynomial-smoother cycle as the single-vector one,
// with identical coefficients, in the hierarchy's precision; the CG
// recurrences, dot products and the final residual are double.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "kernels.h"
#include "system.h"

namespace ocp {

constexpr int kMaxCols = 64;
constexpr int kBlkMaxBlocks = 1024;

// Per-column CG scalars of the block solve (device).
struct CgBlock {
    double ff[kMaxCols];      // f_j . f_j
    double tol2[kMaxCols];    // rtol^2 * (f.f or r0.z0)
    double gamma[kMaxCols];   // r.z of the current iterate
    double gamma0[kMaxCols];  // r0.z0
    double alpha[kMaxCols], beta[kMaxCols];
    double pq[kMaxCols];      // p.Ap
    double rr[kMaxCols];      // r.r
    double xa[kMaxCols];      // alpha still to be added to X (times the current P), 0 if none
    int32_t cflag[kMaxCols];  // 0 running, 1 converged, 2 breakdown, 3 iteration cap
    int32_t citer[kMaxCols];  // iterations taken by column j
    int32_t flag;             // 1 once no column runs
    int32_t iter;             // block iterations
    int32_t k, stop_mode, maxit;
    int32_t xpend;            // some xa[j] != 0
};

// Tiling of a block launch: the k columns are cut into panels of KB columns
// (lane j of a row group owns column panel*KB + j); tile t of T takes, in
// pass it, the RPP consecutive rows starting at (it T + t) RPP.  The tiles of
// one XCD are contiguous, so the blocks an XCD runs at one time work on one
// band of consecutive rows, whose gathered neighbours (256 bytes per row for
// k = 32 double columns) mostly sit in that XCD's L2; tiles that each swept
// their own run of rows spread an XCD's gathers over many mesh planes.
// Blocks run panel-major.  Partial sums are indexed by (column, tile).
struct BlkT {
    int iters;        // row passes per block
    unsigned tiles;   // row tiles per panel
};
struct BlkLaunch {
    BlkT t;
    unsigned blocks;  // tiles * panels
};

// KB lanes per row, each owning VW consecutive columns
inline BlkLaunch blk_launch(int64_t n, int KB, int k, int VW = 1) {
    const int64_t rpp = kBlock / KB;
    int64_t iters = (n + rpp * kBlkMaxBlocks - 1) / (rpp * kBlkMaxBlocks);
    if (iters < 1) iters = 1;
    int64_t b = (n + rpp * iters - 1) / (rpp * iters);
    if (b < 1) b = 1;
    const int panels = (k + KB * VW - 1) / (KB * VW);
    return {{(int)iters, (unsigned)b}, (unsigned)b * (unsigned)panels};
}

static int lanes_for_cols(int k) {
    int g = 8;
    while (g < k) g <<= 1;
    return g;
}

#define OCP_DISPATCH_KB(kb, ...)                                        \
    switch (kb) {                                                       \
        case 8: { constexpr int KB = 8; __VA_ARGS__; } break;           \
        case 16: { constexpr int KB = 16; __VA_ARGS__; } break;         \
        case 32: { constexpr int KB = 32; __VA_ARGS__; } break;         \
        default: { constexpr int KB = 64; __VA_ARGS__; } break;         \
    }

// Row loop of a block kernel: lane j of row group grp; `on` is false for
// padding lanes and frozen columns.
#define OCP_BLK_TILE(KB)                                                  \
    constexpr int RPP = kBlock / KB;                                      \
    const unsigned gtile = dev::xcd_tile(blockIdx.x, gridDim.x);         \
    const int panel = (int)(gtile / bt.tiles);                            \
    const unsigned tile = gtile % bt.tiles;                               \
    const int iters = bt.iters;                                           \
    const int lane = (int)(threadIdx.x % KB);                             \
    const int j = panel * KB + lane;                                      \
    [[maybe_unused]] const int jg = j < k ? j : k - 1; /* valid column */ \
    const int grp = threadIdx.x / KB;                                     \
    const bool on = j < k && (cgb == nullptr || cgb->cflag[j] == 0);     \
    const int base = (int)tile * RPP;                                     \
    const int stride = (int)bt.tiles * RPP;
#define OCP_BLK_BEGIN(KB)                                                 \
    OCP_BLK_TILE(KB)                                                      \
    for (int it = 0; it < iters; ++it) {                                 \
        const int row = base + it * stride + grp;                        \
        if (on && row < n) {                                             \
            const size_t e = (size_t)row * k + j;
#define OCP_BLK_END() \
    }                 \
    }

// Lane roles of a block matrix kernel that streams its rows with blk_rows.
#define OCP_BLKGRP(KB) OCP_BLK_TILE(KB)

// Lane roles of a gather kernel whose lanes own VW consecutive columns each:
// lane `lane` of row group grp owns columns j0 .. j0+VW-1 of the panel; k is
// a multiple of VW, so a lane's columns are all below k or all past it.
// These kernels compute every column below k, frozen ones too (their outputs
// feed only work vectors and partial sums that the frozen columns no longer
// read), so the stores stay whole.
#define OCP_BLKV_TILE(KB, VW)                                             \
    constexpr int RPP = kBlock / KB;                                      \
    const unsigned gtile = dev::xcd_tile(blockIdx.x, gridDim.x);         \
    const int panel = (int)(gtile / bt.tiles);                            \
    const unsigned tile = gtile % bt.tiles;                               \
    const int iters = bt.iters;                                           \
    const int lane = (int)(threadIdx.x % KB);                             \
    const int j0 = (panel * KB + lane) * VW;                              \
    const bool on = j0 < k;                                               \
    const int jg = on ? j0 : 0; /* valid column */                        \
    const int grp = threadIdx.x / KB;                                     \
    const int base = (int)tile * RPP;                                     \
    const int stride = (int)bt.tiles * RPP;

namespace dev {
constexpr int kBlkChunk = 8;    // gathers requested together
constexpr int kBlkStage = 32;   // entries of a row staged in LDS at a time (at least)

// VW consecutive columns of one row of a block vector, loaded and stored as
// one access of VW * sizeof(T) bytes (16 for FP64 pairs and FP32 quads): the
// k values of a row are contiguous and, with k a multiple of VW, every
// lane's first column sits at a multiple of VW.
template <typename T, int VW>
struct alignas(VW * sizeof(T)) BV {
    T v[VW];
};
template <typename T, int VW>
__device__ __forceinline__ BV<T, VW> ldv(const T *p) {
    return *reinterpret_cast<const BV<T, VW> *>(p);
}
template <typename T, int VW>
__device__ __forceinline__ void stv(T *p, const BV<T, VW> &x) {
    *reinterpret_cast<BV<T, VW> *>(p) = x;
}
// s += a g, per column (the scalar form for one column per lane)
template <typename T>
__device__ __forceinline__ void bv_fma(T &s, T a, T g) {
    s += a * g;
}
template <typename T, int VW>
__device__ __forceinline__ void bv_fma(BV<T, VW> &s, T a, const BV<T, VW> &g) {
#pragma unroll
    for (int w = 0; w < VW; ++w) s.v[w] += a * g.v[w];
}

// Lane q's entries q, q + KB, ... (EPL of them) of the row range [b, e),
// indices clamped into the row (level matrices always hold their diagonal
// and restriction rows an aggregate member, so rows are not empty); the
// values past the end are zeroed when they are staged, so that the loads are
// not waited for here.
template <int KB, int EPL, typename T>
__device__ __forceinline__ void blk_entries(int b, int e, int q, const int32_t *__restrict__ col,
                                            const T *__restrict__ val, int (&c)[EPL], T (&v)[EPL]) {
    const int last = e > b ? e - 1 : b;
#pragma unroll
    for (int m = 0; m < EPL; ++m) {
        const int t = b + q + m * KB;
        const int idx = t < last ? t : last;
        c[m] = ldnt(col + idx);
        v[m] = ldnt(val + idx);
    }
}

// Streams the rows of one KB-lane group (rows base + grp + it*stride, it <
// iters).  Per row: the loads of the next row's entries, of the range of the
// row after it and of the row's epilogue operands (ld) are issued first;
// every lane then reads the row's staged entries back from the group's LDS
// slot (SE = max(KB, kBlkStage) entries, EPL per lane) with wide broadcast
// reads, all issued before one wait, and the kBlkChunk gathers of the first
// chunk go out together, unconditionally (padding entries re-gather the
// row's last column with value 0, so xf must address a valid column in
// every lane).  The wait for them therefore drains every load of the row on
// all paths; after fin the group stages the next row's entries (already
// loaded), and nothing is waited for at the top of the next row -- in
// particular not the row's stores, which complete while the next row's
// gathers are in flight.  Entries past the first SE of a long row are
// loaded and staged SE at a time.  xf(c) is the lane's gathered value of
// column c: one T, or a BV of the lane's VW columns; fin(row, s, pre)
// consumes the row product s = sum_q val_q xf(col_q), added in entry order
// as in the single-vector kernels.  Every lane of the group runs the same
// rows.
template <int KB, typename T, typename XF, typename LD, typename FIN>
__device__ __forceinline__ void blk_rows(int n, int iters, int base, int stride, int grp, int lane,
                                         const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                         const T *__restrict__ val, XF xf, LD ld, FIN fin) {
    constexpr int SE = KB > kBlkStage ? KB : kBlkStage;
    constexpr int EPL = SE / KB;
    constexpr int CH = kBlkChunk;
    constexpr int RPP = kBlock / KB;
    static_assert(SE % CH == 0 && CH % 4 == 0, "chunks of whole 16-byte LDS reads");
    constexpr int VPR = 16 / (int)sizeof(T);   // values per 16-byte read
    using G = decltype(xf(0));
    __shared__ __align__(16) int32_t s_col[RPP * SE];
    __shared__ __align__(16) T s_val[RPP * SE];
    int32_t *gcol = s_col + grp * SE;
    T *gval = s_val + grp * SE;
    int row = base + grp;
    if (iters <= 0 || row >= n) return;
    int rb = rp[row], re = rp[row + 1];
    int mc[EPL];
    T mv[EPL];
    blk_entries<KB>(rb, re, lane, col, val, mc, mv);
    int nrow = row + stride;
    bool hn = iters > 1 && nrow < n;
    int nb = 0, ne = 0;
    if (hn) {
        nb = rp[nrow];
        ne = rp[nrow + 1];
    }
    // the staged entries q0 .. q0+CH-1: their values, gathers and products
    auto chunk = [&](int q0, G &s) {
        int c[CH];
        T a[CH];
#pragma unroll
        for (int u = 0; u < CH; u += 4) {
            const int4 c4 = *reinterpret_cast<const int4 *>(gcol + q0 + u);
            c[u] = c4.x;
            c[u + 1] = c4.y;
            c[u + 2] = c4.z;
            c[u + 3] = c4.w;
        }
#pragma unroll
        for (int u = 0; u < CH; u += VPR) {
            const int4 v4 = *reinterpret_cast<const int4 *>(gval + q0 + u);
            const T *vv = reinterpret_cast<const T *>(&v4);
#pragma unroll
            for (int w = 0; w < VPR; ++w) a[u + w] = vv[w];
        }
        G g[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) g[u] = xf(c[u]);
#pragma unroll
        for (int u = 0; u < CH; ++u) bv_fma(s, a[u], g[u]);
    };
    // the first SE entries of the row [b, e) into the group's LDS slot
    auto stage = [&](int b, int e, const int (&c)[EPL], const T (&v)[EPL]) {
#pragma unroll
        for (int m = 0; m < EPL; ++m) {
            gcol[lane + m * KB] = c[m];
            gval[lane + m * KB] = b + lane + m * KB < e ? v[m] : T(0);
        }
    };
    stage(rb, re, mc, mv);
    for (int it = 0;;) {
        // prefetch: entries of the next row, range of the row after it
        int mc2[EPL] = {};
        T mv2[EPL] = {};
        if (hn) blk_entries<KB>(nb, ne, lane, col, val, mc2, mv2);
        const int nnrow = nrow + stride;
        const bool hnn = hn && it + 2 < iters && nnrow < n;
        int nnb = 0, nne = 0;
        if (hnn) {
            nnb = rp[nnrow];
            nne = rp[nnrow + 1];
        }
        const auto pre = ld(row);
        const int cnt = re - rb < SE ? re - rb : SE;
        G s{};
        chunk(0, s);
        for (int q0 = CH; q0 < cnt; q0 += CH) chunk(q0, s);
        for (int b0 = rb + SE; b0 < re; b0 += SE) {   // rows longer than SE
            int c1[EPL];
            T v1[EPL];
            blk_entries<KB>(b0, re, lane, col, val, c1, v1);
            stage(b0, re, c1, v1);
            const int cnt1 = re - b0 < SE ? re - b0 : SE;
            for (int q0 = 0; q0 < cnt1; q0 += CH) chunk(q0, s);
        }
        fin(row, s, pre);
        if (!hn) break;
        stage(nb, ne, mc2, mv2);
        ++it;
        row = nrow;
        rb = nb;
        re = ne;
        nrow = nnrow;
        hn = hnn;
        nb = nnb;
        ne = nne;
    }
}

// Per-column block sums in a fixed order: partials[j * nbs + block].
template <int KB>
__device__ __forceinline__ void blk_store_partial(double acc, double *partials, int nbs, int k, int panel,
                                                  unsigned tile) {
    constexpr int RPP = kBlock / KB;
    __shared__ double red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    const int c = panel * KB + (int)threadIdx.x;
    if (threadIdx.x < (unsigned)KB && c < k) {
        double s = 0.0;
#pragma unroll
        for (int g = 0; g < RPP; ++g) s += red[g * KB + threadIdx.x];
        partials[(size_t)c * nbs + tile] = s;
    }
}

// blk_store_partial for lanes owning VW columns each
template <int KB, int VW>
__device__ __forceinline__ void blk_store_partial_v(const BV<double, VW> &acc, double *partials, int nbs, int k,
                                                    int panel, unsigned tile) {
    constexpr int RPP = kBlock / KB;
    __shared__ double red[VW][kBlock];
#pragma unroll
    for (int w = 0; w < VW; ++w) red[w][threadIdx.x] = acc.v[w];
    __syncthreads();
    const int q = (int)threadIdx.x;   // column of the panel
    const int c = panel * KB * VW + q;
    if (q < KB * VW && c < k) {
        double s = 0.0;
#pragma unroll
        for (int g = 0; g < RPP; ++g) s += red[q % VW][g * KB + q / VW];
        partials[(size_t)c * nbs + tile] = s;
    }
}

// Sum of the nb block partials of column j by one wavefront (fixed order).
__device__ __forceinline__ double col_sum(const double *partials, int nbs, unsigned nb, int j) {
    double s = 0.0;
    for (unsigned b = threadIdx.x & 63; b < nb; b += 64) s += partials[(size_t)j * nbs + b];
    return wave_sum(s);
}

// flag = 1 once every column has stopped (one block, after a column update).
__device__ __forceinline__ void blk_update_flag(CgBlock *cgb) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int any = 0;
        for (int j = 0; j < cgb->k; ++j) any |= (cgb->cflag[j] == 0);
        cgb->flag = any ? 0 : 1;
    }
}
}  // namespace dev

#define OCP_FIN_COLUMNS(kk) for (int j = (int)(threadIdx.x >> 6); j < (kk); j += kFinBlock / 64)

// ------------------------------------------------------------ V-cycle passes
enum { kBR = 0, kBX2 = 1, kBPostA = 2, kBZ = 3 };

// One pass over a level matrix for every column: r = b - A x with x either a
// stored block (GDB false) or the first smoothing step a D^-1 b rebuilt on
// the fly (GDB true); the epilogue per MODE matches the single-vector pass.
// A lane owns VW consecutive columns.
template <typename T, typename BT, typename OT, bool GDB, int MODE, int VW>
struct BlkOps {
    const T *d;
    const BT *b;
    const T *g;
    const T *xp;
    const T *u;
    T a, c1, c2;
    OT *out1;
    T *out2;
    int k;
    using VT = dev::BV<T, VW>;
    // gathered values of row c for the lane's columns from jg: the first
    // smoothing step a d_c b_c rebuilt on the fly (GDB) or the stored block
    __device__ __forceinline__ VT gather(int c, int jg) const {
        const size_t ec = (size_t)c * k + jg;
        if constexpr (GDB) {
            const auto bb = dev::ldv<BT, VW>(b + ec);
            const T f = a * d[c];
            VT r;
#pragma unroll
            for (int w = 0; w < VW; ++w) r.v[w] = f * (T)bb.v[w];
            return r;
        } else {
            return dev::ldv<T, VW>(g + ec);
        }
    }
    // epilogue operands of row i, loaded before the row's gathers
    struct Pre {
        dev::BV<BT, VW> bi;
        T di;
        VT xpi, ui;
    };
    __device__ __forceinline__ Pre load(int i, size_t e) const {
        Pre p{};
        p.bi = dev::ldv<BT, VW>(b + e);
        if (MODE != kBR) p.di = d[i];
        if (MODE == kBPostA || MODE == kBZ) p.xpi = dev::ldv<T, VW>(xp + e);
        if (MODE == kBZ && u) p.ui = dev::ldv<T, VW>(u + e);
        return p;
    }
    // stores the row's outputs; returns b.z per column (kBZ)
    __device__ __forceinline__ dev::BV<double, VW> finish(size_t e, const VT &s, const Pre &p) const {
        dev::BV<double, VW> dot{};
        dev::BV<OT, VW> o1;
        VT o2;
#pragma unroll
        for (int w = 0; w < VW; ++w) {
            const BT bi = p.bi.v[w];
            const T r = (T)bi - s.v[w];
            if (MODE == kBR) {
                o1.v[w] = (OT)r;
            } else if (MODE == kBX2) {
                o1.v[w] = (OT)(p.di * (c1 * (T)bi + c2 * r));
            } else if (MODE == kBPostA) {
                o1.v[w] = (OT)r;
                o2.v[w] = p.xpi.v[w] + a * p.di * r;
            } else {
                T wv = c2 * r;
                if (u) wv += c1 * p.ui.v[w];
                const T z = p.xpi.v[w] + p.di * wv;
                o1.v[w] = (OT)z;
                dot.v[w] = (double)bi * (double)z;
            }
        }
        dev::stv(out1 + e, o1);
        if (MODE == kBPostA) dev::stv(out2 + e, o2);
        return dot;
    }
};

template <int KB, int VW, typename T, typename BT, typename OT, bool GDB, int MODE, bool DOT>
__global__ void __launch_bounds__(kBlock) k_blk_smooth(int32_t n, int k, BlkT bt, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col, const T *__restrict__ val,
                                                       BlkOps<T, BT, OT, GDB, MODE, VW> ops, const CgBlock *cgb,
                                                       double *partials, int nbs) {
    if (cgb && cgb->flag) return;
    dev::BV<double, VW> acc{};
    using Ops = BlkOps<T, BT, OT, GDB, MODE, VW>;
    OCP_BLKV_TILE(KB, VW)
    dev::blk_rows<KB>(
        n, iters, base, stride, grp, lane, rp, col, val, [&](int c) { return ops.gather(c, jg); },
        [&](int row) { return ops.load(row, (size_t)row * k + jg); },
        [&](int row, const typename Ops::VT &s, const typename Ops::Pre &pre) {
            if (on) {
                const auto c = ops.finish((size_t)row * k + j0, s, pre);
                if (DOT)
#pragma unroll
                    for (int w = 0; w < VW; ++w) acc.v[w] += c.v[w];
            }
        });
    if (DOT) dev::blk_store_partial_v<KB, VW>(acc, partials, nbs, k, panel, tile);
}

// y = M x for every column (restriction with R = P^T)
template <int KB, int VW, typename T>
__global__ void __launch_bounds__(kBlock) k_blk_spmv(int32_t n, int k, BlkT bt, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col, const T *__restrict__ val,
                                                     const T *__restrict__ x, T *__restrict__ y, const CgBlock *cgb) {
    if (cgb && cgb->flag) return;
    using VT = dev::BV<T, VW>;
    OCP_BLKV_TILE(KB, VW)
    dev::blk_rows<KB>(
        n, iters, base, stride, grp, lane, rp, col, val, [&](int c) { return dev::ldv<T, VW>(x + (size_t)c * k + jg); },
        [](int) { return 0; },
        [&](int row, const VT &s, int) {
            if (on) dev::stv(y + (size_t)row * k + j0, s);
        });
}

// xp = base + P xc, base = the stored pre-smoothed block (HX) or a d .* b
template <int KB, int VW, typename T, typename BT, bool HX>
__global__ void __launch_bounds__(kBlock) k_blk_prolong(int32_t n, int k, BlkT bt, const int32_t *__restrict__ rp,
                                                        const int32_t *__restrict__ col, const T *__restrict__ val,
                                                        const T *__restrict__ d, const BT *__restrict__ b,
                                                        const T *__restrict__ xs, T a, const T *__restrict__ xc,
                                                        T *__restrict__ xp, const CgBlock *cgb) {
    if (cgb && cgb->flag) return;
    using VT = dev::BV<T, VW>;
    OCP_BLKV_TILE(KB, VW)
    dev::blk_rows<KB>(
        n, iters, base, stride, grp, lane, rp, col, val, [&](int c) { return dev::ldv<T, VW>(xc + (size_t)c * k + jg); },
        [&](int row) {
            const size_t e = (size_t)row * k + jg;
            if constexpr (HX) {
                return dev::ldv<T, VW>(xs + e);
            } else {
                const auto bb = dev::ldv<BT, VW>(b + e);
                const T f = a * d[row];
                VT r;
#pragma unroll
                for (int w = 0; w < VW; ++w) r.v[w] = f * (T)bb.v[w];
                return r;
            }
        },
        [&](int row, const VT &s, const VT &base_v) {
            if (on) {
                VT o;
#pragma unroll
                for (int w = 0; w < VW; ++w) o.v[w] = base_v.v[w] + s.v[w];
                dev::stv(xp + (size_t)row * k + j0, o);
            }
        });
}

// x = Ainv b on the last level (dense inverse, row-major n x n)
template <int KB, typename T, typename BT, typename ZT>
__global__ void __launch_bounds__(kBlock) k_blk_dense(int32_t n, int k, BlkT bt, const T *__restrict__ inv,
                                                      const BT *__restrict__ b, ZT *__restrict__ x,
                                                      const CgBlock *cgb) {
    if (cgb && cgb->flag) return;
    OCP_BLK_BEGIN(KB)
    const T *ir = inv + (size_t)row * n;
    T s = T(0);
    for (int c = 0; c < n; ++c) s += ir[c] * (T)b[(size_t)c * k + j];
    x[e] = (ZT)s;
    OCP_BLK_END()
}

// x = d .* b (last level without a dense inverse)
template <int KB, typename T, typename BT, typename ZT>
__global__ void __launch_bounds__(kBlock) k_blk_diag(int32_t n, int k, BlkT bt, const T *__restrict__ d,
                                                     const BT *__restrict__ b, ZT *__restrict__ x,
                                                     const CgBlock *cgb) {
    if (cgb && cgb->flag) return;
    OCP_BLK_BEGIN(KB)
    x[e] = (ZT)(d[row] * (T)b[e]);
    OCP_BLK_END()
}

// r.z per column (single-level hierarchy)
template <int KB, typename ZT>
__global__ void __launch_bounds__(kBlock) k_blk_rz(int32_t n, int k, BlkT bt, const double *__restrict__ r,
                                                   const ZT *__restrict__ z, const CgBlock *cgb, double *partials,
                                                   int nbs) {
    if (cgb && cgb->flag) return;
    double acc = 0.0;
    OCP_BLK_BEGIN(KB)
    acc += r[e] * (double)z[e];
    OCP_BLK_END()
    dev::blk_store_partial<KB>(acc, partials, nbs, k, panel, tile);
}

// ------------------------------------------------------------- CG kernels
// X = 0, R = F, P = 0 and f.f per column; F column j of row i sits at
// F[i * fs_row + j * fs_col] (fs_col = 0: the same vector for every column).
template <int KB, typename YT>
__global__ void __launch_bounds__(kBlock) k_blk_init(int32_t n, int k, BlkT bt, const double *__restrict__ F,
                                                     int64_t fs_row, int fs_col, double *__restrict__ X,
                                                     double *__restrict__ R, float *__restrict__ R32,
                                                     double *__restrict__ P, FirstStep<YT> first, double *partials,
                                                     int nbs) {
    const CgBlock *cgb = nullptr;
    double acc = 0.0;
    OCP_BLK_BEGIN(KB)
    const double fi = F[(size_t)row * fs_row + (size_t)j * fs_col];
    X[e] = 0.0;
    R[e] = fi;
    if (R32) R32[e] = (float)fi;
    P[e] = 0.0;
    first.put(e, row, fi);
    acc += fi * fi;
    OCP_BLK_END()
    dev::blk_store_partial<KB>(acc, partials, nbs, k, panel, tile);
}

// Q = A P and p.q per column, lanes owning VW columns (k a multiple of VW)
template <int KB, int VW>
__global__ void __launch_bounds__(kBlock) k_blk_spmm_pq(int32_t n, int k, BlkT bt, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ col,
                                                          const double *__restrict__ val,
                                                          const double *__restrict__ P, double *__restrict__ Q,
                                                          const CgBlock *cgb, double *partials, int nbs) {
    if (cgb->flag) return;
    using V = dev::BV<double, VW>;
    V acc{};
    OCP_BLKV_TILE(KB, VW)
    dev::blk_rows<KB>(
        n, iters, base, stride, grp, lane, rp, col, val,
        [&](int c) { return dev::ldv<double, VW>(P + (size_t)c * k + jg); },
        [&](int row) { return dev::ldv<double, VW>(P + (size_t)row * k + jg); },
        [&](int row, const V &s, const V &pi) {
            if (on) {
                dev::stv(Q + (size_t)row * k + j0, s);
#pragma unroll
                for (int w = 0; w < VW; ++w) acc.v[w] += pi.v[w] * s.v[w];
            }
        });
    dev::blk_store_partial_v<KB, VW>(acc, partials, nbs, k, panel, tile);
}

// F - A X per column, squared norm (true residual at exit; every column)
template <int KB>
__global__ void __launch_bounds__(kBlock) k_blk_resid2(int32_t n, int k, BlkT bt, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       const double *__restrict__ val, const double *__restrict__ X,
                                                       const double *__restrict__ F, int64_t fs_row, int fs_col,
                                                       double *partials, int nbs) {
    const CgBlock *cgb = nullptr;
    double acc = 0.0;
    OCP_BLKGRP(KB)
    dev::blk_rows<KB>(
        n, iters, base, stride, grp, lane, rp, col, val, [&](int c) { return X[(size_t)c * k + jg]; },
        [&](int row) { return on ? F[(size_t)row * fs_row + (size_t)j * fs_col] : 0.0; },
        [&](int row, double s, double fi) {
            (void)row;
            if (on) {
                const double r = fi - s;
                acc += r * r;
            }
        });
    dev::blk_store_partial<KB>(acc, partials, nbs, k, panel, tile);
}

// R -= alpha Q, r.r per column; with JAC also Z = dinv R and r.z.  X += alpha P
// waits for k_blk_pupdate, which reads P anyway (8 bytes per entry fewer).
// R32 (if not null): R rounded to FP32 for an FP32 V-cycle's passes, which
// round it so on every read.
template <int KB, bool JAC, typename YT>
__global__ void __launch_bounds__(kBlock) k_blk_update(int32_t n, int k, BlkT bt, double *__restrict__ R,
                                                       float *__restrict__ R32, const double *__restrict__ Q,
                                                       const double *__restrict__ dinv,
                                                       double *__restrict__ Z, FirstStep<YT> first,
                                                       const CgBlock *cgb, double *partials, double *partials2,
                                                       int nbs) {
    if (cgb->flag) return;
    double rr = 0.0, rz = 0.0;
    OCP_BLK_BEGIN(KB)
    const double a = cgb->alpha[j];
    const double r = R[e] - a * Q[e];
    R[e] = r;
    if (R32) R32[e] = (float)r;
    first.put(e, row, r);
    rr += r * r;
    if (JAC) {
        const double z = dinv[row] * r;
        Z[e] = z;
        rz += r * z;
    }
    OCP_BLK_END()
    dev::blk_store_partial<KB>(rr, partials, nbs, k, panel, tile);
    if (JAC) {
        __syncthreads();
        dev::blk_store_partial<KB>(rz, partials2, nbs, k, panel, tile);
    }
}

// Z = dinv R and r.z (Jacobi preconditioner at the start)
template <int KB>
__global__ void __launch_bounds__(kBlock) k_blk_jacobi(int32_t n, int k, BlkT bt, const double *__restrict__ R,
                                                       const double *__restrict__ dinv, double *__restrict__ Z,
                                                       const CgBlock *cgb, double *partials, int nbs) {
    if (cgb->flag) return;
    double rz = 0.0;
    OCP_BLK_BEGIN(KB)
    const double z = dinv[row] * R[e];
    Z[e] = z;
    rz += R[e] * z;
    OCP_BLK_END()
    dev::blk_store_partial<KB>(rz, partials, nbs, k, panel, tile);
}

// X += xa P (the step of this iteration's alpha, also for a column that has
// just stopped), then P = Z + beta P for the running columns.  X gets the same
// products in the same order as when the residual update added them.  Z is
// the preconditioner's output in its own precision (FP32 from an FP32
// V-cycle: the values it computed, exactly).
template <int KB, typename ZT>
__global__ void __launch_bounds__(kBlock) k_blk_pupdate(int32_t n, int k, BlkT bt, double *__restrict__ P,
                                                        const ZT *__restrict__ Z, double *__restrict__ X,
                                                        const CgBlock *cgb) {
    if (cgb->flag && !cgb->xpend) return;
    OCP_BLK_TILE(KB)
    const double xa = j < k ? cgb->xa[j] : 0.0;
    const bool ox = xa != 0.0;
    if (!on && !ox) return;
    const double b = on ? cgb->beta[j] : 0.0;
    for (int it = 0; it < iters; ++it) {
        const int row = base + it * stride + grp;
        if (row < n) {
            const size_t e = (size_t)row * k + j;
            const double p = P[e];
            if (ox) X[e] += xa * p;
            if (on) P[e] = (double)Z[e] + b * p;
        }
    }
}

// U[v][j] = X[dof(v)][j], 0 on Gamma
__global__ void k_blk_scatter(int32_t nv, int k, const int32_t *__restrict__ dof_of_vertex,
                              const double *__restrict__ X, double *__restrict__ U) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nv * k) return;
    const int v = (int)(t / k), j = (int)(t % k);
    const int d = dof_of_vertex[v];
    U[t] = d >= 0 ? X[(size_t)d * k + j] : 0.0;
}

// ------------------------------------------------- per-column finalize kernels
__global__ void __launch_bounds__(kFinBlock) k_blk_fin_init(unsigned nb, const double *partials, int nbs,
                                                            CgBlock *cgb, int k, double rtol, int mode, int maxit) {
    OCP_FIN_COLUMNS(k) {
        const double tot = dev::col_sum(partials, nbs, nb, j);
        if ((threadIdx.x & 63) == 0) {
            cgb->ff[j] = tot;
            cgb->rr[j] = tot;
            cgb->tol2[j] = (mode == OCP_STOP_L2) ? rtol * rtol * tot : rtol * rtol;
            cgb->gamma[j] = 1.0;
            cgb->gamma0[j] = 0.0;
            cgb->alpha[j] = 0.0;
            cgb->xa[j] = 0.0;
            cgb->beta[j] = 0.0;
            cgb->pq[j] = 0.0;
            cgb->citer[j] = 0;
            cgb->cflag[j] = (tot == 0.0) ? 1 : (isfinite(tot) ? 0 : 2);
        }
    }
    if (threadIdx.x == 0) {
        cgb->k = k;
        cgb->iter = 0;
        cgb->stop_mode = mode;
        cgb->maxit = maxit;
        cgb->xpend = 0;
    }
    dev::blk_update_flag(cgb);
}

// after the preconditioner: beta = rz / gamma, gamma = rz; breakdown and the
// preconditioned stop test, per running column
__global__ void __launch_bounds__(kFinBlock) k_blk_fin_rz(unsigned nb, const double *partials, int nbs, CgBlock *cgb) {
    if (cgb->flag) return;
    const int k = cgb->k;
    OCP_FIN_COLUMNS(k) {
        if (cgb->cflag[j] != 0) continue;
        const double rz = dev::col_sum(partials, nbs, nb, j);
        if ((threadIdx.x & 63) == 0) {
            const int it = cgb->citer[j];
            if (it == 0) cgb->gamma0[j] = rz;
            if (!(rz > 0.0) || !isfinite(rz)) {
                cgb->cflag[j] = (rz == 0.0 && cgb->rr[j] == 0.0) ? 1 : 2;
                cgb->beta[j] = 0.0;
            } else {
                cgb->beta[j] = (it == 0) ? 0.0 : rz / cgb->gamma[j];
                cgb->gamma[j] = rz;
                if (cgb->stop_mode == OCP_STOP_PRECOND) {
                    if (it == 0) cgb->tol2[j] *= rz;   // tol2 held rtol^2 until now
                    else if (rz <= cgb->tol2[j]) cgb->cflag[j] = 1;
                }
            }
        }
    }
    dev::blk_update_flag(cgb);
}

// alpha = gamma / p.q per running column, also as the step xa that the next
// k_blk_pupdate adds to X; every other column's xa is cleared (the previous
// one was added by then), also once no column runs.
__global__ void __launch_bounds__(kFinBlock) k_blk_fin_alpha(unsigned nb, const double *partials, int nbs,
                                                             CgBlock *cgb) {
    const bool done = cgb->flag != 0;
    const int k = cgb->k;
    OCP_FIN_COLUMNS(k) {
        if (done || cgb->cflag[j] != 0) {
            if ((threadIdx.x & 63) == 0) cgb->xa[j] = 0.0;
            continue;
        }
        const double pq = dev::col_sum(partials, nbs, nb, j);
        if ((threadIdx.x & 63) == 0) {
            cgb->pq[j] = pq;
            if (!(pq > 0.0) || !isfinite(pq)) {
                cgb->cflag[j] = 2;
                cgb->alpha[j] = 0.0;
            } else {
                cgb->alpha[j] = cgb->gamma[j] / pq;
            }
            cgb->xa[j] = cgb->alpha[j];
        }
    }
    dev::blk_update_flag(cgb);
    if (threadIdx.x == 0) {
        int any = 0;
        for (int j = 0; j < k; ++j) any |= (cgb->xa[j] != 0.0);
        cgb->xpend = any;
    }
}

// r.r after the update: L2 stop test, breakdown, iteration cap; with JAC the
// Jacobi r.z follows as in k_blk_fin_rz
template <bool JAC>
__global__ void __launch_bounds__(kFinBlock) k_blk_fin_update(unsigned nb, const double *partials,
                                                              const double *partials2, int nbs, CgBlock *cgb) {
    if (cgb->flag) return;
    const int k = cgb->k;
    OCP_FIN_COLUMNS(k) {
        if (cgb->cflag[j] != 0) continue;
        const double rr = dev::col_sum(partials, nbs, nb, j);
        const double rz = JAC ? dev::col_sum(partials2, nbs, nb, j) : 0.0;
        if ((threadIdx.x & 63) == 0) {
            cgb->rr[j] = rr;
            const int it = cgb->citer[j] + 1;
            cgb->citer[j] = it;
            if (cgb->stop_mode == OCP_STOP_L2 && rr <= cgb->tol2[j]) {
                cgb->cflag[j] = 1;
            } else if (!isfinite(rr)) {
                cgb->cflag[j] = 2;
            } else {
                if (JAC) {
                    if (!(rz > 0.0) || !isfinite(rz)) {
                        cgb->cflag[j] = (rz == 0.0 && rr == 0.0) ? 1 : 2;
                        cgb->beta[j] = 0.0;
                    } else {
                        cgb->beta[j] = rz / cgb->gamma[j];
                        cgb->gamma[j] = rz;
                        if (cgb->stop_mode == OCP_STOP_PRECOND && rz <= cgb->tol2[j]) cgb->cflag[j] = 1;
                    }
                }
                if (cgb->cflag[j] == 0 && it >= cgb->maxit) cgb->cflag[j] = 3;
            }
        }
    }
    if (threadIdx.x == 0) cgb->iter += 1;
    dev::blk_update_flag(cgb);
}

// ---------------------------------------------------------------- V-cycle
using BlkLevelWork = VcWork::Lvl;   // work blocks of one level, [n_l][k] each

template <typename T>
struct BlkArrays {
    const T *A, *P, *R, *d, *inv;
};
template <typename T>
static BlkArrays<T> blk_arrays(const Level &L);
template <>
BlkArrays<double> blk_arrays<double>(const Level &L) {
    return {L.A_val, L.P_val.get(), L.R_val.get(), L.dinv.get(), L.dense_inv.get()};
}
template <>
BlkArrays<float> blk_arrays<float>(const Level &L) {
    return {L.A_val32.get(), L.P_val32.get(), L.R_val32.get(), L.dinv32.get(), L.dense_inv32.get()};
}

struct BlkCtx {
    int k;
    const void *y0;  // level-0 first smoothing step of R ([n][k], hierarchy precision) or null
    const void *r32; // R in FP32 for an FP32 V-cycle ([n][k]) or null
    double *part;   // [k][nbs] partials of the final r.z
    int nbs;
    CgBlock *cgb;
    std::vector<BlkLevelWork> *work;
};

// Z = B R for the k columns, Z in the hierarchy's precision T.  Returns the
// number of blocks whose r.z partials the last pass stored (0 if cgb is null).
template <int KB, int VW, typename T>
static unsigned vcycle_block_t(ocp_ctx *ctx, const ocp_hierarchy *h, const double *R, T *Z, const BlkCtx &bc) {
    const auto &lv = h->levels;
    const int L = (int)lv.size();
    const int k = bc.k;
    hipStream_t s = ctx->stream;
    CgBlock *cgb = bc.cgb;
    auto &W = *bc.work;
    auto lvec = [&](int l, DevBuf<char> BlkLevelWork::*m) { return reinterpret_cast<T *>((W[l].*m).get()); };

    if (L == 1) {
        const Level &l0 = *lv[0];
        const auto a = blk_arrays<T>(l0);
        const BlkLaunch LB = blk_launch(l0.n, KB, k);
        if (a.inv)
            k_blk_dense<KB, T, double, T><<<LB.blocks, kBlock, 0, s>>>(l0.n, k, LB.t, a.inv, R, Z, cgb);
        else
            k_blk_diag<KB, T, double, T><<<LB.blocks, kBlock, 0, s>>>(l0.n, k, LB.t, a.d, R, Z, cgb);
        OCP_LAUNCH_CHECK();
        if (!cgb) return 0;
        k_blk_rz<KB, T><<<LB.blocks, kBlock, 0, s>>>(l0.n, k, LB.t, R, Z, cgb, bc.part, bc.nbs);
        OCP_LAUNCH_CHECK();
        return LB.t.tiles;
    }

    // ---- down
    for (int l = 0; l < L - 1; ++l) {
        const Level &cur = *lv[l];
        const Level &nxt = *lv[l + 1];
        const auto a = blk_arrays<T>(cur);
        const BlkLaunch LB = blk_launch(cur.n, KB, k, VW);
        T *rres = lvec(l, &BlkLevelWork::vr);
        T *x2 = lvec(l, &BlkLevelWork::vx2);
        const T ca = (T)cur.cheb_a, c1 = (T)cur.cheb_c1, c2 = (T)cur.cheb_c2;
        auto run_down = [&](auto bptr) {
            using BT = std::remove_const_t<std::remove_pointer_t<decltype(bptr)>>;
            const T *y0 = l == 0 ? static_cast<const T *>(bc.y0) : nullptr;
            if (y0) {   // the first step is stored: plain passes gathering it
                if (cur.deg == 2) {
                    k_blk_smooth<KB, VW, T, BT, T, false, kBX2, false><<<LB.blocks, kBlock, 0, s>>>(
                        cur.n, k, LB.t, cur.A_rp, cur.A_col, a.A,
                        BlkOps<T, BT, T, false, kBX2, VW>{a.d, bptr, y0, nullptr, nullptr, ca, c1, c2, x2, nullptr, k},
                        cgb, nullptr, 0);
                    k_blk_smooth<KB, VW, T, BT, T, false, kBR, false><<<LB.blocks, kBlock, 0, s>>>(
                        cur.n, k, LB.t, cur.A_rp, cur.A_col, a.A,
                        BlkOps<T, BT, T, false, kBR, VW>{a.d, bptr, x2, nullptr, nullptr, ca, c1, c2, rres, nullptr, k},
                        cgb, nullptr, 0);
                } else {
                    k_blk_smooth<KB, VW, T, BT, T, false, kBR, false><<<LB.blocks, kBlock, 0, s>>>(
                        cur.n, k, LB.t, cur.A_rp, cur.A_col, a.A,
                        BlkOps<T, BT, T, false, kBR, VW>{a.d, bptr, y0, nullptr, nullptr, ca, c1, c2, rres, nullptr, k},
                        cgb, nullptr, 0);
                }
            } else if (cur.deg == 2) {
                k_blk_smooth<KB, VW, T, BT, T, true, kBX2, false><<<LB.blocks, kBlock, 0, s>>>(
                    cur.n, k, LB.t, cur.A_rp, cur.A_col, a.A,
                    BlkOps<T, BT, T, true, kBX2, VW>{a.d, bptr, nullptr, nullptr, nullptr, ca, c1, c2, x2, nullptr, k},
                    cgb, nullptr, 0);
                k_blk_smooth<KB, VW, T, BT, T, false, kBR, false><<<LB.blocks, kBlock, 0, s>>>(
                    cur.n, k, LB.t, cur.A_rp, cur.A_col, a.A,
                    BlkOps<T, BT, T, false, kBR, VW>{a.d, bptr, x2, nullptr, nullptr, ca, c1, c2, rres, nullptr, k}, cgb,
                    nullptr, 0);
            } else {
                k_blk_smooth<KB, VW, T, BT, T, true, kBR, false><<<LB.blocks, kBlock, 0, s>>>(
                    cur.n, k, LB.t, cur.A_rp, cur.A_col, a.A,
                    BlkOps<T, BT, T, true, kBR, VW>{a.d, bptr, nullptr, nullptr, nullptr, ca, c1, c2, rres, nullptr, k},
                    cgb, nullptr, 0);
            }
            OCP_LAUNCH_CHECK();
        };
        if (l == 0 && bc.r32)
            run_down(static_cast<const T *>(bc.r32));
        else if (l == 0)
            run_down(R);
        else
            run_down(static_cast<const T *>(lvec(l, &BlkLevelWork::vb)));
        const BlkLaunch LR = blk_launch(nxt.n, KB, k, VW);
        k_blk_spmv<KB, VW, T><<<LR.blocks, kBlock, 0, s>>>(nxt.n, k, LR.t, cur.R_rp.get(), cur.R_col.get(), a.R, rres,
                                                       lvec(l + 1, &BlkLevelWork::vb), cgb);
        OCP_LAUNCH_CHECK();
    }
    // ---- coarsest
    {
        const Level &cl = *lv[L - 1];
        const auto a = blk_arrays<T>(cl);
        const BlkLaunch LB = blk_launch(cl.n, KB, k);
        const T *b = lvec(L - 1, &BlkLevelWork::vb);
        T *x = lvec(L - 1, &BlkLevelWork::vx);
        if (a.inv)
            k_blk_dense<KB, T, T, T><<<LB.blocks, kBlock, 0, s>>>(cl.n, k, LB.t, a.inv, b, x, cgb);
        else
            k_blk_diag<KB, T, T, T><<<LB.blocks, kBlock, 0, s>>>(cl.n, k, LB.t, a.d, b, x, cgb);
        OCP_LAUNCH_CHECK();
    }
    // ---- up
    unsigned fin_nb = 0;
    for (int l = L - 2; l >= 0; --l) {
        const Level &cur = *lv[l];
        const auto a = blk_arrays<T>(cur);
        const BlkLaunch LB = blk_launch(cur.n, KB, k, VW);
        const T *xc = lvec(l + 1, &BlkLevelWork::vx);
        T *xp = lvec(l, &BlkLevelWork::vxp);
        T *x2 = lvec(l, &BlkLevelWork::vx2);
        T *r0 = lvec(l, &BlkLevelWork::vr);
        T *x1 = lvec(l, &BlkLevelWork::vx1);
        const T ca = (T)cur.cheb_a, c1 = (T)cur.cheb_c1, c2 = (T)cur.cheb_c2;
        const T zero = T(0);
        // bptr: the level's right-hand side; bzptr: the same for the last
        // pass, whose b.z is taken in double (R itself on level 0)
        auto run_up = [&](auto bptr, auto bzptr, auto outptr, auto dot_tag) {
            using BT = std::remove_const_t<std::remove_pointer_t<decltype(bptr)>>;
            using BZT = std::remove_const_t<std::remove_pointer_t<decltype(bzptr)>>;
            using OT = std::remove_pointer_t<decltype(outptr)>;
            constexpr bool DOT = decltype(dot_tag)::value;
            if (cur.deg == 2)
                k_blk_prolong<KB, VW, T, BT, true><<<LB.blocks, kBlock, 0, s>>>(cur.n, k, LB.t, cur.P_rp.get(),
                                                                          cur.P_col.get(), a.P, a.d, bptr, x2, ca,
                                                                          xc, xp, cgb);
            else
                k_blk_prolong<KB, VW, T, BT, false><<<LB.blocks, kBlock, 0, s>>>(cur.n, k, LB.t, cur.P_rp.get(),
                                                                           cur.P_col.get(), a.P, a.d, bptr, nullptr,
                                                                           ca, xc, xp, cgb);
            OCP_LAUNCH_CHECK();
            if (cur.deg == 2) {
                k_blk_smooth<KB, VW, T, BT, T, false, kBPostA, false><<<LB.blocks, kBlock, 0, s>>>(
                    cur.n, k, LB.t, cur.A_rp, cur.A_col, a.A,
                    BlkOps<T, BT, T, false, kBPostA, VW>{a.d, bptr, xp, xp, nullptr, ca, c1, c2, r0, x1, k}, cgb, nullptr,
                    0);
                k_blk_smooth<KB, VW, T, BZT, OT, false, kBZ, DOT><<<LB.blocks, kBlock, 0, s>>>(
                    cur.n, k, LB.t, cur.A_rp, cur.A_col, a.A,
                    BlkOps<T, BZT, OT, false, kBZ, VW>{a.d, bzptr, x1, xp, r0, ca, c1, c2, outptr, nullptr, k}, cgb,
                    DOT ? bc.part : nullptr, bc.nbs);
            } else {
                k_blk_smooth<KB, VW, T, BZT, OT, false, kBZ, DOT><<<LB.blocks, kBlock, 0, s>>>(
                    cur.n, k, LB.t, cur.A_rp, cur.A_col, a.A,
                    BlkOps<T, BZT, OT, false, kBZ, VW>{a.d, bzptr, xp, xp, nullptr, ca, zero, ca, outptr, nullptr, k},
                    cgb, DOT ? bc.part : nullptr, bc.nbs);
            }
            OCP_LAUNCH_CHECK();
            if (DOT) fin_nb = LB.t.tiles;
        };
        if (l == 0) {
            auto up0 = [&](auto bptr) {
                if (cgb)
                    run_up(bptr, R, Z, std::true_type{});
                else
                    run_up(bptr, R, Z, std::false_type{});
            };
            if (bc.r32)
                up0(static_cast<const T *>(bc.r32));
            else
                up0(R);
        } else {
            const T *vb = lvec(l, &BlkLevelWork::vb);
            run_up(vb, vb, lvec(l, &BlkLevelWork::vx), std::false_type{});
        }
    }
    return fin_nb;
}

// Columns per lane of the block V-cycle's gather passes in precision T:
// 16-byte accesses when k allows them, else one column per lane.
template <typename T>
static int blk_vw(int k) {
    constexpr int V = 16 / (int)sizeof(T);
    return k % V == 0 ? V : 1;
}

template <typename T>
static unsigned vcycle_block(ocp_ctx *ctx, const ocp_hierarchy *h, const double *R, T *Z, const BlkCtx &bc,
                             int kb) {
    constexpr int V = 16 / (int)sizeof(T);
    unsigned nb = 0;
    if (blk_vw<T>(bc.k) == V) {
        OCP_DISPATCH_KB(kb, (nb = vcycle_block_t<KB, V, T>(ctx, h, R, Z, bc)));
    } else {
        OCP_DISPATCH_KB(kb, (nb = vcycle_block_t<KB, 1, T>(ctx, h, R, Z, bc)));
    }
    return nb;
}

// ------------------------------------------------------------------ driver
static int worst_status(const std::vector<int> &st) {
    int w = OCP_OK;
    for (int s : st) {
        if (s == OCP_ERR_BREAKDOWN) return OCP_ERR_BREAKDOWN;
        if (s == OCP_MAXIT) w = OCP_MAXIT;
    }
    return w;
}

// Panel width of the block kernels: forced by the flags, else the fastest of
// the candidates KB = 8, 16, 32, 64 (KB <= the single-panel width), timed
// once per system (SpMM) or hierarchy (V-cycle) and k, then kept, so that
// repeated solves take the same kernels and give the same bits.
static int forced_kb(int32_t flags, int kb_max) {
    const int f = (flags >> 8) & 0xff;
    if (f == 0) return 0;
    if (f != 8 && f != 16 && f != 32 && f != 64) fail(OCP_ERR_INVALID_ARG, "block tile must be 8, 16, 32 or 64");
    return f < kb_max ? f : kb_max;
}

template <typename F>
static int tune_kb(ocp_ctx *ctx, int kb_max, F launch) {
    hipEvent_t e0, e1;
    OCP_HIP(hipEventCreate(&e0));
    OCP_HIP(hipEventCreate(&e1));
    int best = kb_max;
    float best_ms = 0.f;
    for (int kb = 8; kb <= kb_max; kb <<= 1) {
        launch(kb);   // first launch of the variant (code load, caches)
        OCP_HIP(hipEventRecord(e0, ctx->stream));
        launch(kb);
        OCP_HIP(hipEventRecord(e1, ctx->stream));
        OCP_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        OCP_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (kb == 8 || ms < best_ms) {
            best_ms = ms;
            best = kb;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

static void solve_multi(ocp_ctx *ctx, ocp_system *sys, const ocp_hierarchy *h, int k, const double *F, double *U,
                        double rtol, int32_t maxit, int32_t flags, ocp_solve_info *infos, int *status) {
    const int32_t n = sys->n;
    const int KB0 = lanes_for_cols(k);   // one panel: elementwise CG kernels
    // the SpMM's lanes own column pairs (16-byte gathers) when k is even
    const int vw_mm = k % 2 == 0 ? 2 : 1;
    const int KBM = vw_mm == 2 ? lanes_for_cols(k / 2) : KB0;
    const int64_t fs_row = F ? k : 1;
    const int fs_col = F ? 1 : 0;
    const double *Fp = F ? F : sys->f.get();
    const size_t nk = (size_t)n * k;
    const int forced = forced_kb(flags, KB0);
    DevBuf<double> X(ctx, nk), R(ctx, nk), P(ctx, nk), Q(ctx, nk), Z(ctx, nk);
    const BlkLaunch LB = blk_launch(n, KB0, k);
    const int nbs = kBlkMaxBlocks;
    DevBuf<double> part0(ctx, (size_t)k * nbs), part1(ctx, (size_t)k * nbs), part2(ctx, (size_t)k * nbs);
    DevBuf<CgBlock> cgbuf(ctx, 1);
    CgBlock *cgb = cgbuf.get();
    const double *dinv = h ? nullptr : system_dinv(ctx, sys);
    const int mode = (flags & OCP_STOP_PRECOND) ? OCP_STOP_PRECOND : OCP_STOP_L2;
    VcWork vwork;
    if (h) vc_work_alloc(ctx, h, vwork, k);
    std::vector<BlkLevelWork> &work = vwork.lv;
    const bool mixed = h && h->params.precision == OCP_PREC_MIXED;
    // level-0 first smoothing step of R, written by the kernels producing R
    DevBuf<char> y0buf;
    const bool want_y0 = h && h->levels.size() > 1;
    FirstStep<float> fs32{nullptr, nullptr, 0.f};
    FirstStep<double> fs64{nullptr, nullptr, 0.0};
    if (want_y0) {
        const Level &l0 = *h->levels[0];
        y0buf.reset(ctx, nk * (mixed ? sizeof(float) : sizeof(double)));
        if (mixed)
            fs32 = {reinterpret_cast<float *>(y0buf.get()), l0.dinv32.get(), (float)l0.cheb_a};
        else
            fs64 = {reinterpret_cast<double *>(y0buf.get()), l0.dinv.get(), l0.cheb_a};
    }
    // an FP32 V-cycle leaves Z in FP32 in the first half of Z's memory and
    // reads R rounded to FP32 from the second half
    float *Z32 = reinterpret_cast<float *>(Z.get());
    float *R32 = mixed && want_y0 ? Z32 + nk : nullptr;
    BlkCtx bc{k, want_y0 ? y0buf.get() : nullptr, R32, part1.get(), nbs, cgb, &work};
    hipStream_t s = ctx->stream;
    const int32_t *rp = sys->row_ptr.get(), *ci = sys->col.get();
    const double *av = sys->val.get();
    // panel widths chosen earlier for this (system or hierarchy, k); the
    // first solve of a shape times the candidates below and publishes its
    // choice by compare-and-swap, so concurrent first solves agree on the
    // first published width and every later solve takes it
    std::atomic<int> &kb_mm_slot = const_cast<ocp_system *>(sys)->blk_kb_spmm[k];
    std::atomic<int> *kb_vc_slot = h ? &const_cast<ocp_hierarchy *>(h)->blk_kb_vc[k] : nullptr;
    auto publish = [](std::atomic<int> &slot, int kb) {
        int expected = 0;
        slot.compare_exchange_strong(expected, kb, std::memory_order_acq_rel);
        return slot.load(std::memory_order_acquire);
    };
    // lanes per row of the V-cycle's gather passes: VW columns each
    const int vw_vc = !h ? 1 : mixed ? blk_vw<float>(k) : blk_vw<double>(k);
    const int KBV = lanes_for_cols(k / vw_vc);
    int kb_vc = KBV;
    if (h) {
        const int cached = kb_vc_slot->load(std::memory_order_acquire);
        kb_vc = forced ? std::min(forced, KBV) : (cached ? cached : KBV);
    }
    const int cached_mm = kb_mm_slot.load(std::memory_order_acquire);
    int kb_mm = forced ? std::min(forced, KBM) : (cached_mm ? cached_mm : KBM);

    auto precond = [&](void) {
        if (h) {
            const unsigned nb = mixed ? vcycle_block<float>(ctx, h, R.get(), Z32, bc, kb_vc)
                                      : vcycle_block<double>(ctx, h, R.get(), Z.get(), bc, kb_vc);
            k_blk_fin_rz<<<1, kFinBlock, 0, s>>>(nb, part1.get(), nbs, cgb);
        } else {
            OCP_DISPATCH_KB(KB0, (k_blk_jacobi<KB><<<LB.blocks, kBlock, 0, s>>>(n, k, LB.t, R.get(), dinv, Z.get(),
                                                                             cgb, part1.get(), nbs)));
            k_blk_fin_rz<<<1, kFinBlock, 0, s>>>(LB.t.tiles, part1.get(), nbs, cgb);
        }
        OCP_LAUNCH_CHECK();
    };
    auto pupdate = [&](void) {
        if (h && mixed) {
            OCP_DISPATCH_KB(KB0, (k_blk_pupdate<KB, float><<<LB.blocks, kBlock, 0, s>>>(n, k, LB.t, P.get(), Z32,
                                                                                         X.get(), cgb)));
        } else {
            OCP_DISPATCH_KB(KB0, (k_blk_pupdate<KB, double><<<LB.blocks, kBlock, 0, s>>>(n, k, LB.t, P.get(), Z.get(),
                                                                                          X.get(), cgb)));
        }
        OCP_LAUNCH_CHECK();
    };
    auto spmm = [&](int kb) {
        const BlkLaunch LS = blk_launch(n, kb, k, vw_mm);
        if (vw_mm == 2) {
            OCP_DISPATCH_KB(kb, (k_blk_spmm_pq<KB, 2><<<LS.blocks, kBlock, 0, s>>>(
                                    n, k, LS.t, rp, ci, av, P.get(), Q.get(), cgb, part0.get(), nbs)));
        } else {
            OCP_DISPATCH_KB(kb, (k_blk_spmm_pq<KB, 1><<<LS.blocks, kBlock, 0, s>>>(
                                    n, k, LS.t, rp, ci, av, P.get(), Q.get(), cgb, part0.get(), nbs)));
        }
        OCP_LAUNCH_CHECK();
        return LS.t.tiles;
    };

    ctx->prof_iter = -1;
    OCP_HIP(hipEventRecord(ctx->ev0, s));
    if (mixed) {
        OCP_DISPATCH_KB(KB0, (k_blk_init<KB, float><<<LB.blocks, kBlock, 0, s>>>(
                                 n, k, LB.t, Fp, fs_row, fs_col, X.get(), R.get(), R32, P.get(), fs32, part0.get(),
                                 nbs)));
    } else {
        OCP_DISPATCH_KB(KB0, (k_blk_init<KB, double><<<LB.blocks, kBlock, 0, s>>>(
                                 n, k, LB.t, Fp, fs_row, fs_col, X.get(), R.get(), nullptr, P.get(), fs64, part0.get(),
                                 nbs)));
    }
    k_blk_fin_init<<<1, kFinBlock, 0, s>>>(LB.t.tiles, part0.get(), nbs, cgb, k, rtol, mode, maxit);
    OCP_LAUNCH_CHECK();

    struct {
        int32_t flag, iter;
    } hs{0, 0};
    read_back(ctx, &hs, &cgb->flag, sizeof(hs));
    // first solve of this shape: time the panel widths on the live data before
    // the first V-cycle (the outputs of these launches are overwritten before
    // they are read), so that every solve of the shape uses the same kernels
    if (!forced && hs.flag == 0) {
        if (!kb_mm_slot.load(std::memory_order_acquire)) publish(kb_mm_slot, tune_kb(ctx, KBM, spmm));
        kb_mm = kb_mm_slot.load(std::memory_order_acquire);
        if (h && !kb_vc_slot->load(std::memory_order_acquire)) {
            const Level &l0 = *h->levels[0];
            if (h->levels.size() > 1) {
                // one FP32 (VW 1 or 4) or FP64 (VW 1 or 2) level-0 pass per width
                auto trial = [&](int kb, auto vw_tag) {
                    constexpr int VW = decltype(vw_tag)::value;
                    OCP_DISPATCH_KB(kb, ({
                        const BlkLaunch LV = blk_launch(l0.n, KB, k, VW);
                        auto f32 = [&]() {
                            if constexpr (VW != 2) {
                                float *x2 = reinterpret_cast<float *>(work[0].vx2.get());
                                float *rr = reinterpret_cast<float *>(work[0].vr.get());
                                k_blk_smooth<KB, VW, float, float, float, false, kBR, false>
                                    <<<LV.blocks, kBlock, 0, s>>>(
                                        l0.n, k, LV.t, l0.A_rp, l0.A_col, l0.A_val32.get(),
                                        BlkOps<float, float, float, false, kBR, VW>{l0.dinv32.get(), R32, x2, nullptr,
                                                                                   nullptr, 0.f, 0.f, 0.f, rr,
                                                                                   nullptr, k},
                                        cgb, nullptr, 0);
                            }
                        };
                        auto f64 = [&]() {
                            if constexpr (VW != 4) {
                                double *x2 = reinterpret_cast<double *>(work[0].vx2.get());
                                double *rr = reinterpret_cast<double *>(work[0].vr.get());
                                k_blk_smooth<KB, VW, double, double, double, false, kBR, false>
                                    <<<LV.blocks, kBlock, 0, s>>>(
                                        l0.n, k, LV.t, l0.A_rp, l0.A_col, l0.A_val,
                                        BlkOps<double, double, double, false, kBR, VW>{l0.dinv.get(), R.get(), x2,
                                                                                       nullptr, nullptr, 0.0, 0.0,
                                                                                       0.0, rr, nullptr, k},
                                        cgb, nullptr, 0);
                            }
                        };
                        if (mixed)
                            f32();
                        else
                            f64();
                    }));
                    OCP_LAUNCH_CHECK();
                };
                publish(*kb_vc_slot, tune_kb(ctx, KBV, [&](int kb) {
                    if (vw_vc == 4)
                        trial(kb, std::integral_constant<int, 4>{});
                    else if (vw_vc == 2)
                        trial(kb, std::integral_constant<int, 2>{});
                    else
                        trial(kb, std::integral_constant<int, 1>{});
                }));
            } else {
                publish(*kb_vc_slot, KBV);
            }
        }
        if (h) kb_vc = kb_vc_slot->load(std::memory_order_acquire);
    }
    precond();
    pupdate();
    read_back(ctx, &hs, &cgb->flag, sizeof(hs));

    int chunk = 2;
    ctx->prof_iter = 0;
    for (;;) {
        if (hs.flag != 0) break;
        for (int c = 0; c < chunk; ++c) {
            const int pr = prof_begin(ctx, OCP_KERNEL_BLK_SPMM);
            const unsigned nbm = spmm(kb_mm);
            prof_end(ctx, pr);
            k_blk_fin_alpha<<<1, kFinBlock, 0, s>>>(nbm, part0.get(), nbs, cgb);
            if (h) {
                if (mixed) {
                    OCP_DISPATCH_KB(KB0, (k_blk_update<KB, false, float><<<LB.blocks, kBlock, 0, s>>>(
                                             n, k, LB.t, R.get(), R32, Q.get(), nullptr, nullptr, fs32,
                                             cgb, part0.get(), nullptr, nbs)));
                } else {
                    OCP_DISPATCH_KB(KB0, (k_blk_update<KB, false, double><<<LB.blocks, kBlock, 0, s>>>(
                                             n, k, LB.t, R.get(), nullptr, Q.get(), nullptr, nullptr, fs64,
                                             cgb, part0.get(), nullptr, nbs)));
                }
                k_blk_fin_update<false><<<1, kFinBlock, 0, s>>>(LB.t.tiles, part0.get(), nullptr, nbs, cgb);
                OCP_LAUNCH_CHECK();
                precond();
            } else {
                OCP_DISPATCH_KB(KB0, (k_blk_update<KB, true, float><<<LB.blocks, kBlock, 0, s>>>(
                                         n, k, LB.t, R.get(), nullptr, Q.get(), dinv, Z.get(), fs32, cgb,
                                         part0.get(), part2.get(), nbs)));
                k_blk_fin_update<true><<<1, kFinBlock, 0, s>>>(LB.t.tiles, part0.get(), part2.get(), nbs, cgb);
                OCP_LAUNCH_CHECK();
            }
            pupdate();
            ++ctx->prof_iter;
        }
        if (chunk < 8) chunk *= 2;
        read_back(ctx, &hs, &cgb->flag, sizeof(hs));
    }
    OCP_HIP(hipEventRecord(ctx->ev1, s));

    // true residuals in double, then U on all vertices
    const BlkLaunch LR = blk_launch(n, KB0, k);
    OCP_DISPATCH_KB(KB0, (k_blk_resid2<KB><<<LR.blocks, kBlock, 0, s>>>(n, k, LR.t, rp, ci, av, X.get(), Fp,
                                                                         fs_row, fs_col, part2.get(), nbs)));
    OCP_LAUNCH_CHECK();
    k_blk_scatter<<<grid_for((int64_t)sys->nv * k, 256), 256, 0, s>>>(sys->nv, k, sys->dof_of_vertex.get(), X.get(),
                                                                       U);
    OCP_LAUNCH_CHECK();
    // per-column residual partials and scalars to the host (summed there in
    // tile order)
    std::vector<double> res_part((size_t)k * nbs);
    OCP_HIP(hipMemcpyAsync(res_part.data(), part2.get(), sizeof(double) * k * nbs, hipMemcpyDeviceToHost, s));
    CgBlock hcg;
    OCP_HIP(hipMemcpyAsync(&hcg, cgb, sizeof(CgBlock), hipMemcpyDeviceToHost, s));
    sync(ctx);
    float ms = 0.f;
    OCP_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    prof_resolve(ctx, hs.iter - 1);

    std::vector<int> st((size_t)k);
    for (int j = 0; j < k; ++j) {
        double res2 = 0.0;
        for (unsigned b = 0; b < LR.t.tiles; ++b) res2 += res_part[(size_t)j * nbs + b];
        const int cf = hcg.cflag[j];
        st[j] = cf == 2 ? OCP_ERR_BREAKDOWN : cf == 3 ? OCP_MAXIT : OCP_OK;
        if (infos) {
            ocp_solve_info &in = infos[j];
            in.iterations = hcg.citer[j];
            in.status = st[j];
            in.rel_res_l2 = hcg.ff[j] > 0 ? std::sqrt(hcg.rr[j] / hcg.ff[j]) : 0.0;
            in.rel_res_precond = hcg.gamma0[j] > 0 ? std::sqrt(hcg.gamma[j] / hcg.gamma0[j]) : 0.0;
            in.true_rel_res = hcg.ff[j] > 0 ? std::sqrt(res2 / hcg.ff[j]) : 0.0;
            in.setup_ms = h ? h->setup_ms : 0.0;
            in.solve_ms = ms;
        }
    }
    *status = worst_status(st);
}

}  // namespace ocp

using namespace ocp;

extern "C" int pcg_solve_multi(ocp_ctx *ctx, const ocp_system *sys, const ocp_hierarchy *h, int32_t k,
                               const double *F, double *U, double rtol, int32_t maxit, int32_t flags,
                               ocp_solve_info *infos) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    int status = OCP_OK;
    int rc = run_guarded(ctx, [&] {
        if (!sys || !U) fail(OCP_ERR_INVALID_ARG, "system and U must not be NULL");
        if (k < 1 || k > kMaxCols) fail(OCP_ERR_INVALID_ARG, "k must lie in 1..64");
        if (!(rtol > 0.0) || !std::isfinite(rtol)) fail(OCP_ERR_INVALID_ARG, "rtol must be positive");
        if (maxit < 1) fail(OCP_ERR_INVALID_ARG, "maxit must be >= 1");
        check_hierarchy(h, sys);
        if (h && h->params.method != OCP_AMG_AGGREGATION)
            fail(OCP_ERR_UNSUPPORTED, "block solves take smoothed-aggregation hierarchies");
        solve_multi(ctx, const_cast<ocp_system *>(sys), h, k, F, U, rtol, maxit, flags, infos, &status);
    });
    if (rc != OCP_OK) {
        if (infos)
            for (int j = 0; j < std::max(0, std::min<int>(k, kMaxCols)); ++j) infos[j].status = rc;
        return rc;
    }
    if (status == OCP_ERR_BREAKDOWN) ctx->last_error = "CG breakdown in at least one column";
    return status;
}
