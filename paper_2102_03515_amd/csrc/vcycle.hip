// Application of the AMG preconditioner B: one V(1,1)-cycle with zero
// initial guess (Section 3.1: pre-smoothing, restriction with P^T, recursive
// coarse correction with zero start, prolongation with P, post-smoothing).
//
// The smoother is a polynomial in D^-1 A: Chebyshev of degree 1 or 2 on
// [lambda/ratio, lambda] (lambda a Gershgorin bound of D^-1 A, D = diag A), or
// L1-Jacobi (degree 1, D_ii = sum_j |a_ij|).  Pre- and post-smoothing apply the
// same polynomial, which is self-adjoint in the A inner product, so B is SPD.
// From a zero initial guess the smoothed iterate is a combination of vectors
// already in memory (x1 = a D^-1 b; x2 = D^-1 (c1 b + c2 r1) for degree 2), so
// each smoothing step and the following residual form one pass over A that
// rebuilds the neighbours' iterate on the fly; the iterate itself is never
// stored.  The prolongation rebuilds it once more and adds P e; post-smoothing
// takes one pass per degree.  On the fine level the last pass also forms r.z
// for CG.
//
// Values are double (FP64 hierarchy) or float (mixed precision); the CG
// vectors entering and leaving the cycle are always double.
#include <cmath>
#include <type_traits>

#include "kernels.h"
#include "system.h"

namespace ocp {

#define OCP_DISPATCH_G(g, ...)                          \
    switch (g) {                                        \
        case 4: { constexpr int G = 4; __VA_ARGS__; } break;   \
        case 8: { constexpr int G = 8; __VA_ARGS__; } break;   \
        case 16: { constexpr int G = 16; __VA_ARGS__; } break; \
        case 32: { constexpr int G = 32; __VA_ARGS__; } break; \
        default: { constexpr int G = 64; __VA_ARGS__; } break; \
    }

#define OCP_ROWS_BEGIN(G)                                              \
    constexpr int RPP = kBlock / G;                                    \
    const unsigned tile = dev::xcd_tile(blockIdx.x, gridDim.x);        \
    const int lane = threadIdx.x % G, grp = threadIdx.x / G;           \
    const int base = (int)tile * RPP * iters;                          \
    for (int it = 0; it < iters; ++it) {                               \
        const int row = base + it * RPP + grp;                         \
        if (row < n) {
#define OCP_ROWS_END() \
    }                  \
    }

// One pass over a level matrix: r_i = b_i - sum_j a_ij x_j, where the
// gathered iterate is either a stored vector (GDB = false: x_j = g_j) or the
// first smoothing step from zero, rebuilt on the fly (GDB = true:
// x_j = a d_j b_j).  The epilogue (row i only) writes, by MODE:
//   kR     out1 = r
//   kX2    out1 = d_i (c1 b_i + c2 r_i)          second pre-smoothing iterate
//   kPostA out1 = r, out2 = xp_i + a d_i r_i     post residual and first step
//   kZ     out1 = xp_i + d_i (c1 u_i + c2 r_i)   last post step (u = r0), and
//          with DOT also b.out1 for CG
// so every smoothing step of the V-cycle is one such pass and every pass
// gathers a single vector.
enum { kR = 0, kX2 = 1, kPostA = 2, kZ = 3 };

template <typename T, typename BT, typename OT, bool GDB, int MODE, bool DOT>
struct SmoothOps {
    const T *d;
    const BT *b;
    const T *g;
    const T *xp;
    const T *u;
    T a, c1, c2;
    OT *out1;
    T *out2;
    __device__ __forceinline__ T gather(int c) const {
        if (GDB) return a * d[c] * (T)b[c];
        return g[c];
    }
    // writes row i's outputs; returns its b.z contribution (DOT)
    __device__ __forceinline__ double finish(int i, T s) const {
        const BT bi = b[i];
        const T r = (T)bi - s;
        if (MODE == kR) {
            out1[i] = (OT)r;
        } else if (MODE == kX2) {
            out1[i] = (OT)(d[i] * (c1 * (T)bi + c2 * r));
        } else if (MODE == kPostA) {
            out1[i] = (OT)r;
            out2[i] = xp[i] + a * d[i] * r;
        } else {
            T w = c2 * r;
            if (u) w += c1 * u[i];
            const T z = xp[i] + d[i] * w;
            out1[i] = (OT)z;
            if (DOT) return (double)bi * (double)z;
        }
        return 0.0;
    }
};

template <int G, typename T, typename BT, typename OT, bool GDB, int MODE, bool DOT>
__global__ void __launch_bounds__(kBlock) k_smooth(int32_t n, int iters, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col, const T *__restrict__ val,
                                                   SmoothOps<T, BT, OT, GDB, MODE, DOT> ops, CgScalars *cg,
                                                   double *partials) {
    if (cg && cg->flag) return;
    double acc = 0.0;
    OCP_ROWS_BEGIN(G)
    const T s = dev::row_sum<G>(rp[row], rp[row + 1], lane, col, val, [&](int c) { return ops.gather(c); });
    if (lane == 0) acc += ops.finish(row, s);
    OCP_ROWS_END()
    if (DOT) dev::store_partial(dev::block_sum<kBlock>(acc), partials);
}

// the same pass on the sliced-ELL copy of the fine-level matrix
template <typename T, typename BT, typename OT, bool GDB, int MODE, bool DOT>
__global__ void __launch_bounds__(kBlock) k_smooth_sell(int32_t n, int64_t nslices, int spb,
                                                        const int32_t *__restrict__ sp, const int32_t *__restrict__ sw,
                                                        SellCols col, const T *__restrict__ val,
                                                        SmoothOps<T, BT, OT, GDB, MODE, DOT> ops, CgScalars *cg,
                                                        double *partials) {
    if (cg && cg->flag) return;
    double acc = 0.0;
    OCP_SELL_BEGIN(nslices, spb)
    const T s = dev::sell_row_c(col, slice, row, n, val, base, w, [&](int c) { return ops.gather(c); });
    if (row < n) acc += ops.finish(row, s);
    OCP_SELL_END()
    if (DOT) dev::store_partial(dev::block_sum<kBlock>(acc), partials);
}

// y = M x for a level matrix (restriction with R = P^T)
template <int G, typename T>
__global__ void __launch_bounds__(kBlock) k_vc_spmv(int32_t n, int iters, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ col, const T *__restrict__ val,
                                                    const T *__restrict__ x, T *__restrict__ y,
                                                    const CgScalars *cg) {
    if (cg && cg->flag) return;
    OCP_ROWS_BEGIN(G)
    const T s = dev::row_sum<G>(rp[row], rp[row + 1], lane, col, val, [&](int c) { return x[c]; });
    if (lane == 0) y[row] = s;
    OCP_ROWS_END()
}

// xp = base + P xc, base = the stored pre-smoothed iterate (HX) or a d .* b
template <int G, typename T, typename BT, bool HX>
__global__ void __launch_bounds__(kBlock) k_vc_prolong(int32_t n, int iters, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col, const T *__restrict__ val,
                                                       const T *__restrict__ d, const BT *__restrict__ b,
                                                       const T *__restrict__ xs, T a, const T *__restrict__ xc,
                                                       T *__restrict__ xp, const CgScalars *cg) {
    if (cg && cg->flag) return;
    OCP_ROWS_BEGIN(G)
    const T s = dev::row_sum<G>(rp[row], rp[row + 1], lane, col, val, [&](int c) { return xc[c]; });
    if (lane == 0) xp[row] = (HX ? xs[row] : a * d[row] * (T)b[row]) + s;
    OCP_ROWS_END()
}

// The same for P with short rows (at most kStreamRow entries): 256 rows per
// block; the block's entries are read once, consecutively, their products
// staged in LDS, and each row is summed in entry order by its own thread.
constexpr int kStreamRow = 16;
template <typename T, typename BT, bool HX>
__global__ void __launch_bounds__(kBlock) k_vc_prolong_stream(int32_t n, const int32_t *__restrict__ rp,
                                                              const int32_t *__restrict__ col,
                                                              const T *__restrict__ val, const T *__restrict__ d,
                                                              const BT *__restrict__ b, const T *__restrict__ xs, T a,
                                                              const T *__restrict__ xc, T *__restrict__ xp,
                                                              const CgScalars *cg) {
    if (cg && cg->flag) return;
    __shared__ T prod[kBlock * kStreamRow];
    const int r0 = blockIdx.x * kBlock;
    const int r1 = r0 + kBlock < n ? r0 + kBlock : n;
    const int e0 = rp[r0], e1 = rp[r1];
    constexpr int U = 4;   // entries per thread and step, all requested first
    for (int k0 = e0 + (int)threadIdx.x; k0 < e1; k0 += U * kBlock) {
        int c[U];
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * kBlock < e1 ? k0 + u * kBlock : e1 - 1;
            c[u] = dev::ldnt(col + k);
            v[u] = dev::ldnt(val + k);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * kBlock < e1) prod[k0 + u * kBlock - e0] = v[u] * xc[c[u]];
    }
    __syncthreads();
    const int row = r0 + (int)threadIdx.x;
    if (row >= n) return;
    const int kb = rp[row] - e0, ke = rp[row + 1] - e0;
    T s = T(0);
    for (int k = kb; k < ke; ++k) s += prod[k];
    xp[row] = (HX ? xs[row] : a * d[row] * (T)b[row]) + s;
}

// x = Ainv b on the last level (dense, one wavefront per row)
template <typename T, typename BT, typename ZT>
__global__ void __launch_bounds__(kBlock) k_vc_dense(int32_t n, const T *__restrict__ inv, const BT *__restrict__ b,
                                                     ZT *__restrict__ x, const CgScalars *cg) {
    if (cg && cg->flag) return;
    const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    T s = T(0);
    for (int j = lane; j < n; j += 64) s += inv[(int64_t)row * n + j] * (T)b[j];
    s = dev::wave_sum(s);
    if (lane == 0) x[row] = (ZT)s;
}

// x = d .* b (last level too large for a dense inverse: one Jacobi sweep)
template <typename T, typename BT, typename ZT>
__global__ void k_vc_diag(int32_t n, const T *__restrict__ d, const BT *__restrict__ b, ZT *__restrict__ x,
                          const CgScalars *cg) {
    if (cg && cg->flag) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = (ZT)(d[i] * (T)b[i]);
}

// r.z after a one-level "cycle"
__global__ void __launch_bounds__(kBlock) k_cg_rz(int32_t n, int iters, const double *__restrict__ r,
                                                  const double *__restrict__ z, CgScalars *cg, double *partials) {
    if (cg->flag) return;
    const unsigned tile = dev::xcd_tile(blockIdx.x, gridDim.x);
    const int base = (int)tile * kBlock * iters;
    double acc = 0.0;
    for (int it = 0; it < iters; ++it) {
        const int i = base + it * kBlock + threadIdx.x;
        if (i < n) acc += r[i] * z[i];
    }
    dev::store_partial(dev::block_sum<kBlock>(acc), partials);
}

__global__ void __launch_bounds__(kFinBlock) k_vc_fin_rz(unsigned nb, const double *partials, CgScalars *cg) {
    if (cg->flag) return;
    const double tot = dev::sum_partials<kFinBlock>(partials, nb);
    if (threadIdx.x == 0) dev::cg_after_precond(cg, tot);
}

// ------------------------------------------------------------------ driver
template <typename T>
struct LevelArrays {
    const T *A, *P, *R, *d, *inv;
};

// values of a level's sliced-ELL copy (level 0: the system's) in the
// hierarchy's precision
template <typename T>
static const T *sell_values(const Level &L, const Sell &S);
template <>
const double *sell_values<double>(const Level &L, const Sell &S) {
    (void)L;
    return S.val.get();
}
template <>
const float *sell_values<float>(const Level &L, const Sell &S) {
    (void)S;
    return L.sell_val32.get();
}

template <typename T>
static LevelArrays<T> arrays(const Level &L);
template <>
LevelArrays<double> arrays<double>(const Level &L) {
    return {L.A_val, L.P_val.get(), L.R_val.get(), L.dinv.get(), L.dense_inv.get()};
}
template <>
LevelArrays<float> arrays<float>(const Level &L) {
    return {L.A_val32.get(), L.P_val32.get(), L.R_val32.get(), L.dinv32.get(), L.dense_inv32.get()};
}

static int lanes_for(int64_t nnz, int64_t rows) {
    const double avg = rows > 0 ? (double)nnz / (double)rows : 1.0;
    int g = 4;
    while (g < 64 && g < avg) g <<= 1;
    return g;
}

template <typename T>
static void vcycle_t(ocp_ctx *ctx, const ocp_hierarchy *h, const double *r_in, double *z_out, CgScalars *cg,
                     VcWork &W) {
    const auto &lv = h->levels;
    const int L = (int)lv.size();
    hipStream_t s = ctx->stream;
    double *part = W.part ? W.part : ctx->red_partials + 3 * kRedBlocks;
    const Sell &S = system_sell(ctx, h->sys);
    const T *sval = sell_values<T>(*lv[0], S);
    const SellLaunch LSL = sell_launch(S.nslices);

    if (L == 1) {
        const Level &l0 = *lv[0];
        const auto a = arrays<T>(l0);
        if (a.inv)
            k_vc_dense<T, double, double><<<grid_for(l0.n, kBlock / 64), kBlock, 0, s>>>(l0.n, a.inv, r_in, z_out, cg);
        else
            k_vc_diag<T, double, double><<<grid_for(l0.n, 256), 256, 0, s>>>(l0.n, a.d, r_in, z_out, cg);
        OCP_LAUNCH_CHECK();
        if (cg) {
            const RowLaunch LV = vec_launch(l0.n);
            k_cg_rz<<<LV.blocks, kBlock, 0, s>>>(l0.n, LV.iters, r_in, z_out, cg, part);
            k_vc_fin_rz<<<1, kFinBlock, 0, s>>>(LV.blocks, part, cg);
            OCP_LAUNCH_CHECK();
        }
        return;
    }

    // one pass over level l's matrix (sliced ELL on level 0, CSR with G lanes
    // per row on the coarser levels)
    auto pass = [&](int l, auto ops, bool dot) {
        const Level &cur = *lv[l];
        unsigned nb;
        if (l == 0) {
            nb = LSL.blocks;
            k_smooth_sell<<<LSL.blocks, kBlock, 0, s>>>(S.n, S.nslices, LSL.slices_per_block, S.sp.get(), S.sw.get(),
                                                         sell_cols(S), sval, ops, cg, dot ? part : nullptr);
        } else if (cur.sell.col.get()) {
            const Sell &C = cur.sell;
            const SellLaunch LC = sell_launch(C.nslices);
            nb = LC.blocks;
            k_smooth_sell<<<LC.blocks, kBlock, 0, s>>>(C.n, C.nslices, LC.slices_per_block, C.sp.get(), C.sw.get(),
                                                        sell_cols(C), sell_values<T>(cur, C), ops, cg,
                                                        dot ? part : nullptr);
        } else {
            const auto a = arrays<T>(cur);
            const RowLaunch LA = row_launch(cur.n, cur.gA);
            nb = LA.blocks;
            OCP_DISPATCH_G(cur.gA, (k_smooth<G><<<LA.blocks, kBlock, 0, s>>>(cur.n, LA.iters, cur.A_rp, cur.A_col,
                                                                            a.A, ops, cg, dot ? part : nullptr)));
        }
        OCP_LAUNCH_CHECK();
        return nb;
    };

    // ---- down: pre-smoothing from zero, residual, restriction
    auto down = [&](int l, auto bptr) {
        using BT = std::remove_const_t<std::remove_pointer_t<decltype(bptr)>>;
        const Level &cur = *lv[l];
        const Level &nxt = *lv[l + 1];
        const auto a = arrays<T>(cur);
        T *rres = reinterpret_cast<T *>(W.lv[l].vr.get());
        T *x2 = reinterpret_cast<T *>(W.lv[l].vx2.get());
        const T ca = (T)cur.cheb_a, c1 = (T)cur.cheb_c1, c2 = (T)cur.cheb_c2;
        // the first step from zero, a D^-1 b, as stored by b's producer
        const T *y0 = l == 0 ? static_cast<const T *>(W.y0) : nullptr;
        if (cur.deg == 2) {
            // x2 = D^-1 (c1 b + c2 r1), r1 = b - A (a D^-1 b); then r2 = b - A x2
            const int pr = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_PRE0) : -1;
            if (y0)
                pass(l, SmoothOps<T, BT, T, false, kX2, false>{a.d, bptr, y0, nullptr, nullptr, ca, c1, c2, x2,
                                                               nullptr},
                     false);
            else
                pass(l, SmoothOps<T, BT, T, true, kX2, false>{a.d, bptr, nullptr, nullptr, nullptr, ca, c1, c2, x2,
                                                              nullptr},
                     false);
            prof_end(ctx, pr);
            const int pr2 = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_PRE0_B) : -1;
            pass(l, SmoothOps<T, BT, T, false, kR, false>{a.d, bptr, x2, nullptr, nullptr, ca, c1, c2, rres, nullptr},
                 false);
            prof_end(ctx, pr2);
        } else {
            // r1 = b - A (a D^-1 b)
            const int pr = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_PRE0) : -1;
            if (y0)
                pass(l, SmoothOps<T, BT, T, false, kR, false>{a.d, bptr, y0, nullptr, nullptr, ca, c1, c2, rres,
                                                              nullptr},
                     false);
            else
                pass(l, SmoothOps<T, BT, T, true, kR, false>{a.d, bptr, nullptr, nullptr, nullptr, ca, c1, c2, rres,
                                                             nullptr},
                     false);
            prof_end(ctx, pr);
        }
        T *bn = reinterpret_cast<T *>(W.lv[l + 1].vb.get());
        const RowLaunch LR = row_launch(nxt.n, cur.gR);
        const int prr = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_RESTRICT0) : -1;
        OCP_DISPATCH_G(cur.gR, (k_vc_spmv<G, T><<<LR.blocks, kBlock, 0, s>>>(nxt.n, LR.iters, cur.R_rp.get(),
                                                                              cur.R_col.get(), a.R, rres, bn, cg)));
        prof_end(ctx, prr);
        OCP_LAUNCH_CHECK();
    };
    for (int l = 0; l < L - 1; ++l) {
        if (l == 0)
            down(0, r_in);
        else
            down(l, reinterpret_cast<const T *>(W.lv[l].vb.get()));
    }
    // ---- coarsest
    {
        const Level &cl = *lv[L - 1];
        const auto a = arrays<T>(cl);
        const T *b = reinterpret_cast<const T *>(W.lv[L - 1].vb.get());
        T *x = reinterpret_cast<T *>(W.lv[L - 1].vx.get());
        if (a.inv)
            k_vc_dense<T, T, T><<<grid_for(cl.n, kBlock / 64), kBlock, 0, s>>>(cl.n, a.inv, b, x, cg);
        else
            k_vc_diag<T, T, T><<<grid_for(cl.n, 256), 256, 0, s>>>(cl.n, a.d, b, x, cg);
        OCP_LAUNCH_CHECK();
    }
    // ---- up: prolongation + correction, post-smoothing
    unsigned fin_nb = 0;
    auto up = [&](int l, auto bptr, auto outptr, bool dot) {
        using BT = std::remove_const_t<std::remove_pointer_t<decltype(bptr)>>;
        using OT = std::remove_pointer_t<decltype(outptr)>;
        const Level &cur = *lv[l];
        const auto a = arrays<T>(cur);
        const T *xc = reinterpret_cast<const T *>(W.lv[l + 1].vx.get());
        T *xp = reinterpret_cast<T *>(W.lv[l].vxp.get());
        T *x2 = reinterpret_cast<T *>(W.lv[l].vx2.get());
        T *r0 = reinterpret_cast<T *>(W.lv[l].vr.get());
        T *x1 = reinterpret_cast<T *>(W.lv[l].vx1.get());
        const T ca = (T)cur.cheb_a, c1 = (T)cur.cheb_c1, c2 = (T)cur.cheb_c2;
        const T zero = T(0);
        const RowLaunch LP = row_launch(cur.n, cur.gP);
        const int prp = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_PROLONG0) : -1;
        if (cur.maxP <= kStreamRow) {
            const unsigned nb = (unsigned)((cur.n + kBlock - 1) / kBlock);
            if (cur.deg == 2)
                k_vc_prolong_stream<T, BT, true><<<nb, kBlock, 0, s>>>(cur.n, cur.P_rp.get(), cur.P_col.get(), a.P,
                                                                       a.d, bptr, x2, ca, xc, xp, cg);
            else
                k_vc_prolong_stream<T, BT, false><<<nb, kBlock, 0, s>>>(cur.n, cur.P_rp.get(), cur.P_col.get(), a.P,
                                                                        a.d, bptr, nullptr, ca, xc, xp, cg);
        } else if (cur.deg == 2) {
            OCP_DISPATCH_G(cur.gP, (k_vc_prolong<G, T, BT, true><<<LP.blocks, kBlock, 0, s>>>(
                                       cur.n, LP.iters, cur.P_rp.get(), cur.P_col.get(), a.P, a.d, bptr, x2, ca, xc, xp,
                                       cg)));
        } else {
            OCP_DISPATCH_G(cur.gP, (k_vc_prolong<G, T, BT, false><<<LP.blocks, kBlock, 0, s>>>(
                                       cur.n, LP.iters, cur.P_rp.get(), cur.P_col.get(), a.P, a.d, bptr, nullptr, ca,
                                       xc, xp, cg)));
        }
        prof_end(ctx, prp);
        OCP_LAUNCH_CHECK();
        if (cur.deg == 2) {
            // r0 = b - A xp and x1 = xp + a D^-1 r0; then r1 = b - A x1 and
            // z = xp + D^-1 (c1 r0 + c2 r1)
            const int pra = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_POST0_A) : -1;
            pass(l, SmoothOps<T, BT, T, false, kPostA, false>{a.d, bptr, xp, xp, nullptr, ca, c1, c2, r0, x1}, false);
            prof_end(ctx, pra);
            const int pro = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_POST0) : -1;
            if (dot)
                fin_nb = pass(l, SmoothOps<T, BT, OT, false, kZ, true>{a.d, bptr, x1, xp, r0, ca, c1, c2, outptr,
                                                                       nullptr},
                              true);
            else
                pass(l, SmoothOps<T, BT, OT, false, kZ, false>{a.d, bptr, x1, xp, r0, ca, c1, c2, outptr, nullptr},
                     false);
            prof_end(ctx, pro);
        } else {
            // z = xp + a D^-1 (b - A xp)
            const int pro = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_POST0) : -1;
            if (dot)
                fin_nb = pass(l, SmoothOps<T, BT, OT, false, kZ, true>{a.d, bptr, xp, xp, nullptr, ca, zero, ca, outptr,
                                                                       nullptr},
                              true);
            else
                pass(l, SmoothOps<T, BT, OT, false, kZ, false>{a.d, bptr, xp, xp, nullptr, ca, zero, ca, outptr,
                                                               nullptr},
                     false);
            prof_end(ctx, pro);
        }
    };
    for (int l = L - 2; l >= 0; --l) {
        if (l == 0)
            up(0, r_in, z_out, cg != nullptr);
        else
            up(l, reinterpret_cast<const T *>(W.lv[l].vb.get()), reinterpret_cast<T *>(W.lv[l].vx.get()), false);
    }
    if (cg) {
        k_vc_fin_rz<<<1, kFinBlock, 0, s>>>(fin_nb, part, cg);
        OCP_LAUNCH_CHECK();
    }
}

// ------------------------------------------------- red-black method cycle
// Section 3.1's V(1,1)-cycle: one forward Gauss-Seidel sweep from zero
// before the coarse correction and one backward sweep after it (the
// backward sweep is the adjoint of the forward one in the A inner product,
// so the cycle is a symmetric positive definite preconditioner).  A sweep
// takes the colours of the level's colouring in order (reverse order
// backwards); rows of one colour are not coupled, so each colour is one
// launch that updates its rows from the current iterate:
//   x_i += (b_i - sum_j a_ij x_j) / a_ii.
template <int G, typename T, typename BT, typename XT>
__global__ void __launch_bounds__(kBlock) k_gs_colour(int32_t m, const int32_t *__restrict__ rows,
                                                      const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                      const T *__restrict__ val, const T *__restrict__ dinv,
                                                      const BT *__restrict__ b, XT *__restrict__ x,
                                                      const CgScalars *cg) {
    if (cg && cg->flag) return;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int r = (int)(t / G), lane = (int)(t % G);
    if (r >= m) return;
    const int i = rows[r];
    const T s = dev::row_sum<G>(rp[i], rp[i + 1], lane, col, val, [&](int c) { return (T)x[c]; });
    if (lane == 0) x[i] = (XT)((T)x[i] + ((T)b[i] - s) * dinv[i]);
}

// r = b - A x
template <int G, typename T, typename BT, typename XT>
__global__ void __launch_bounds__(kBlock) k_rb_resid(int32_t n, int iters, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col, const T *__restrict__ val,
                                                     const BT *__restrict__ b, const XT *__restrict__ x,
                                                     T *__restrict__ r, const CgScalars *cg) {
    if (cg && cg->flag) return;
    OCP_ROWS_BEGIN(G)
    const T s = dev::row_sum<G>(rp[row], rp[row + 1], lane, col, val, [&](int c) { return (T)x[c]; });
    if (lane == 0) r[row] = (T)b[row] - s;
    OCP_ROWS_END()
}

// x += P xc
template <int G, typename T, typename XT>
__global__ void __launch_bounds__(kBlock) k_rb_prolong(int32_t n, int iters, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col, const T *__restrict__ val,
                                                       const T *__restrict__ xc, XT *__restrict__ x,
                                                       const CgScalars *cg) {
    if (cg && cg->flag) return;
    OCP_ROWS_BEGIN(G)
    const T s = dev::row_sum<G>(rp[row], rp[row + 1], lane, col, val, [&](int c) { return xc[c]; });
    if (lane == 0) x[row] = (XT)((T)x[row] + s);
    OCP_ROWS_END()
}

template <typename XT>
__global__ void k_rb_zero(int32_t n, XT *__restrict__ x, const CgScalars *cg) {
    if (cg && cg->flag) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = XT(0);
}

template <typename T>
static void vcycle_rb(ocp_ctx *ctx, const ocp_hierarchy *h, const double *r_in, double *z_out, CgScalars *cg,
                      VcWork &W) {
    const auto &lv = h->levels;
    const int L = (int)lv.size();
    hipStream_t s = ctx->stream;
    double *part = W.part ? W.part : ctx->red_partials + 3 * kRedBlocks;
    // one sweep over level l's colours (forward or backward)
    auto sweep = [&](int l, auto b, auto x, bool forward) {
        const Level &cur = *lv[l];
        const auto a = arrays<T>(cur);
        for (int q = 0; q < cur.ncolors; ++q) {
            const int c = forward ? q : cur.ncolors - 1 - q;
            const int32_t r0 = cur.color_ptr[c], m = cur.color_ptr[c + 1] - r0;
            if (m <= 0) continue;
            OCP_DISPATCH_G(cur.gA, (k_gs_colour<G, T><<<grid_for((int64_t)m * G, kBlock), kBlock, 0, s>>>(
                                       m, cur.color_rows.get() + r0, cur.A_rp, cur.A_col, a.A, a.d, b, x, cg)));
        }
        OCP_LAUNCH_CHECK();
    };
    auto coarsest = [&](int l, auto b, auto x) {
        const Level &cl = *lv[l];
        const auto a = arrays<T>(cl);
        if (a.inv) {
            k_vc_dense<T><<<grid_for(cl.n, kBlock / 64), kBlock, 0, s>>>(cl.n, a.inv, b, x, cg);
            OCP_LAUNCH_CHECK();
        } else {   // too large for the dense inverse: a symmetric sweep from zero
            k_rb_zero<<<grid_for(cl.n, 256), 256, 0, s>>>(cl.n, x, cg);
            sweep(l, b, x, true);
            sweep(l, b, x, false);
        }
    };
    auto vec = [&](const DevBuf<char> &v) { return reinterpret_cast<T *>(v.get()); };
    if (L == 1) {
        coarsest(0, r_in, z_out);
    } else {
        // down: x_l = forward sweep from zero; b_{l+1} = R (b_l - A x_l)
        for (int l = 0; l < L - 1; ++l) {
            const Level &cur = *lv[l];
            const Level &nxt = *lv[l + 1];
            const auto a = arrays<T>(cur);
            T *rres = vec(W.lv[l].vr);
            T *bn = vec(W.lv[l + 1].vb);
            const RowLaunch LA = row_launch(cur.n, cur.gA);
            const RowLaunch LR = row_launch(nxt.n, cur.gR);
            auto go = [&](auto b, auto x) {
                k_rb_zero<<<grid_for(cur.n, 256), 256, 0, s>>>(cur.n, x, cg);
                sweep(l, b, x, true);
                OCP_DISPATCH_G(cur.gA, (k_rb_resid<G, T><<<LA.blocks, kBlock, 0, s>>>(cur.n, LA.iters, cur.A_rp,
                                                                                    cur.A_col, a.A, b, x, rres, cg)));
            };
            if (l == 0)
                go(r_in, z_out);
            else
                go(static_cast<const T *>(vec(W.lv[l].vb)), vec(W.lv[l].vx));
            OCP_DISPATCH_G(cur.gR, (k_vc_spmv<G, T><<<LR.blocks, kBlock, 0, s>>>(nxt.n, LR.iters, cur.R_rp.get(),
                                                                              cur.R_col.get(), a.R, rres, bn, cg)));
            OCP_LAUNCH_CHECK();
        }
        coarsest(L - 1, static_cast<const T *>(vec(W.lv[L - 1].vb)), vec(W.lv[L - 1].vx));
        // up: x_l += P x_{l+1}, then a backward sweep
        for (int l = L - 2; l >= 0; --l) {
            const Level &cur = *lv[l];
            const auto a = arrays<T>(cur);
            const RowLaunch LP = row_launch(cur.n, cur.gP);
            const T *xc = vec(W.lv[l + 1].vx);
            auto go = [&](auto b, auto x) {
                OCP_DISPATCH_G(cur.gP, (k_rb_prolong<G, T><<<LP.blocks, kBlock, 0, s>>>(
                                           cur.n, LP.iters, cur.P_rp.get(), cur.P_col.get(), a.P, xc, x, cg)));
                OCP_LAUNCH_CHECK();
                sweep(l, b, x, false);
            };
            if (l == 0)
                go(r_in, z_out);
            else
                go(static_cast<const T *>(vec(W.lv[l].vb)), vec(W.lv[l].vx));
        }
    }
    if (cg) {
        const int32_t n0 = lv[0]->n;
        const RowLaunch LV = vec_launch(n0);
        k_cg_rz<<<LV.blocks, kBlock, 0, s>>>(n0, LV.iters, r_in, z_out, cg, part);
        k_vc_fin_rz<<<1, kFinBlock, 0, s>>>(LV.blocks, part, cg);
        OCP_LAUNCH_CHECK();
    }
}

void vcycle_enqueue(ocp_ctx *ctx, const ocp_hierarchy *h, const double *r, double *z, CgScalars *cg, VcWork &w) {
    if (h->params.method == OCP_AMG_REDBLACK) {
        if (h->params.precision == OCP_PREC_MIXED)
            vcycle_rb<float>(ctx, h, r, z, cg, w);
        else
            vcycle_rb<double>(ctx, h, r, z, cg, w);
        return;
    }
    if (h->params.precision == OCP_PREC_MIXED)
        vcycle_t<float>(ctx, h, r, z, cg, w);
    else
        vcycle_t<double>(ctx, h, r, z, cg, w);
}

void vc_work_alloc(ocp_ctx *ctx, const ocp_hierarchy *h, VcWork &w, int k) {
    const size_t vs = h->params.precision == OCP_PREC_MIXED ? sizeof(float) : sizeof(double);
    const int L = (int)h->levels.size();
    w.lv.clear();
    w.lv.resize(L);
    for (int l = 0; l < L; ++l) {
        const size_t bytes = (size_t)h->levels[l]->n * k * vs;
        if (l > 0) {
            w.lv[l].vb.reset(ctx, bytes);
            w.lv[l].vx.reset(ctx, bytes);
        }
        if (l < L - 1) {
            w.lv[l].vr.reset(ctx, bytes);
            w.lv[l].vxp.reset(ctx, bytes);
            w.lv[l].vx1.reset(ctx, bytes);
            w.lv[l].vx2.reset(ctx, bytes);
        }
    }
}

int level_lanes(int64_t nnz, int64_t rows) { return lanes_for(nnz, rows); }

}  // namespace ocp

using namespace ocp;

extern "C" int amg_vcycle(ocp_ctx *ctx, const ocp_hierarchy *h, const double *r, double *z) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    return run_guarded(ctx, [&] {
        if (!h || !r || !z) fail(OCP_ERR_INVALID_ARG, "hierarchy, r and z must not be NULL");
        check_hierarchy(h, h->sys);
        VcWork w;
        vc_work_alloc(ctx, h, w);
        vcycle_enqueue(ctx, h, r, z, nullptr, w);
        sync(ctx);   // the work vectors are released on return
    });
}
