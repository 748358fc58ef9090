// Application of the AMG preconditioner B: one V(1,1)-cycle with zero
// initial guess (Section 4.1: pre-smoothing, restriction with P^T, recursive
// coarse correction with zero start, prolongation with P, post-smoothing).
//
// The smoother is L1-Jacobi, S = I - D1^{-1} A with D1_ii = sum_j |a_ij|; it
// is symmetric, so pre- and post-smoothing are adjoint and B is SPD.  With a
// zero initial guess the pre-smoothed iterate is x = D1^{-1} b, so the
// pre-smoother and the residual r = b - A D1^{-1} b form one pass over A that
// recomputes the neighbours' x on the fly; x itself is never stored.  The
// prolongation rebuilds it, xp = D1^{-1} b + P e, and the post-smoother
// x = xp + D1^{-1}(b - A xp) is the second pass over A.  On the fine level the
// post-smoother also forms r.z for CG.
//
// Values are double (FP64 hierarchy) or float (mixed precision); the CG
// vectors entering and leaving the cycle are always double.
#include <cmath>

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

// r = b - A (d .* b)
template <int G, typename T, typename BT>
__global__ void __launch_bounds__(kBlock) k_vc_pre(int32_t n, int iters, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col, const T *__restrict__ val,
                                                   const T *__restrict__ d, const BT *__restrict__ b,
                                                   T *__restrict__ r, const CgScalars *cg) {
    if (cg && cg->flag) return;
    OCP_ROWS_BEGIN(G)
    const T s = dev::row_sum<G>(rp[row], rp[row + 1], lane, col, val, [&](int c) { return d[c] * (T)b[c]; });
    if (lane == 0) r[row] = (T)b[row] - s;
    OCP_ROWS_END()
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

// xp = d .* b + P xc
template <int G, typename T, typename BT>
__global__ void __launch_bounds__(kBlock) k_vc_prolong(int32_t n, int iters, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col, const T *__restrict__ val,
                                                       const T *__restrict__ d, const BT *__restrict__ b,
                                                       const T *__restrict__ xc, T *__restrict__ xp,
                                                       const CgScalars *cg) {
    if (cg && cg->flag) return;
    OCP_ROWS_BEGIN(G)
    const T s = dev::row_sum<G>(rp[row], rp[row + 1], lane, col, val, [&](int c) { return xc[c]; });
    if (lane == 0) xp[row] = d[row] * (T)b[row] + s;
    OCP_ROWS_END()
}

// z = xp + d .* (b - A xp); with DOT also r.z -> CG scalars
template <int G, typename T, typename BT, typename ZT, bool DOT>
__global__ void __launch_bounds__(kBlock) k_vc_post(int32_t n, int iters, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ col, const T *__restrict__ val,
                                                    const T *__restrict__ d, const BT *__restrict__ b,
                                                    const T *__restrict__ xp, ZT *__restrict__ z, CgScalars *cg,
                                                    double *partials, unsigned *counter) {
    if (cg && cg->flag) return;
    double acc = 0.0;
    OCP_ROWS_BEGIN(G)
    const T s = dev::row_sum<G>(rp[row], rp[row + 1], lane, col, val, [&](int c) { return xp[c]; });
    if (lane == 0) {
        const BT bi = b[row];
        const T zi = xp[row] + d[row] * ((T)bi - s);
        z[row] = (ZT)zi;
        if (DOT) acc += (double)bi * (double)zi;
    }
    OCP_ROWS_END()
    if (DOT) {
        acc = dev::block_sum<kBlock>(acc);
        double tot;
        if (dev::grid_sum_last<kBlock>(acc, partials, counter, &tot) && threadIdx.x == 0)
            dev::cg_after_precond(cg, tot);
    }
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
                                                  const double *__restrict__ z, CgScalars *cg, double *partials,
                                                  unsigned *counter) {
    if (cg->flag) return;
    const unsigned tile = dev::xcd_tile(blockIdx.x, gridDim.x);
    const int base = (int)tile * kBlock * iters;
    double acc = 0.0;
    for (int it = 0; it < iters; ++it) {
        const int i = base + it * kBlock + threadIdx.x;
        if (i < n) acc += r[i] * z[i];
    }
    acc = dev::block_sum<kBlock>(acc);
    double tot;
    if (dev::grid_sum_last<kBlock>(acc, partials, counter, &tot) && threadIdx.x == 0) dev::cg_after_precond(cg, tot);
}

// ------------------------------------------------------------------ driver
template <typename T>
struct LevelArrays {
    const T *A, *P, *R, *d, *inv;
};

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
static void vcycle_t(ocp_ctx *ctx, const ocp_hierarchy *h, const double *r_in, double *z_out, CgScalars *cg) {
    const auto &lv = h->levels;
    const int L = (int)lv.size();
    hipStream_t s = ctx->stream;
    double *part = ctx->red_partials + 3 * kRedBlocks;
    unsigned *cnt = ctx->red_counters + 3;

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
            k_cg_rz<<<LV.blocks, kBlock, 0, s>>>(l0.n, LV.iters, r_in, z_out, cg, part, cnt);
            OCP_LAUNCH_CHECK();
        }
        return;
    }

    // ---- down
    for (int l = 0; l < L - 1; ++l) {
        const Level &cur = *lv[l];
        const Level &nxt = *lv[l + 1];
        const auto a = arrays<T>(cur);
        T *r = reinterpret_cast<T *>(cur.vr.get());
        const RowLaunch LA = row_launch(cur.n, cur.gA);
        if (l == 0) {
            const int pr = cg ? prof_begin(ctx, OCP_KERNEL_VC_PRE0) : -1;
            OCP_DISPATCH_G(cur.gA, (k_vc_pre<G, T, double><<<LA.blocks, kBlock, 0, s>>>(
                                       cur.n, LA.iters, cur.A_rp, cur.A_col, a.A, a.d, r_in, r, cg)));
            prof_end(ctx, pr);
        } else {
            const T *b = reinterpret_cast<const T *>(cur.vb.get());
            OCP_DISPATCH_G(cur.gA, (k_vc_pre<G, T, T><<<LA.blocks, kBlock, 0, s>>>(cur.n, LA.iters, cur.A_rp,
                                                                                    cur.A_col, a.A, a.d, b, r, cg)));
        }
        OCP_LAUNCH_CHECK();
        T *bn = reinterpret_cast<T *>(nxt.vb.get());
        const RowLaunch LR = row_launch(nxt.n, cur.gR);
        const int prr = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_RESTRICT0) : -1;
        OCP_DISPATCH_G(cur.gR, (k_vc_spmv<G, T><<<LR.blocks, kBlock, 0, s>>>(nxt.n, LR.iters, cur.R_rp.get(),
                                                                              cur.R_col.get(), a.R, r, bn, cg)));
        prof_end(ctx, prr);
        OCP_LAUNCH_CHECK();
    }
    // ---- coarsest
    {
        const Level &cl = *lv[L - 1];
        const auto a = arrays<T>(cl);
        const T *b = reinterpret_cast<const T *>(cl.vb.get());
        T *x = reinterpret_cast<T *>(cl.vx.get());
        if (a.inv)
            k_vc_dense<T, T, T><<<grid_for(cl.n, kBlock / 64), kBlock, 0, s>>>(cl.n, a.inv, b, x, cg);
        else
            k_vc_diag<T, T, T><<<grid_for(cl.n, 256), 256, 0, s>>>(cl.n, a.d, b, x, cg);
        OCP_LAUNCH_CHECK();
    }
    // ---- up
    for (int l = L - 2; l >= 0; --l) {
        const Level &cur = *lv[l];
        const Level &nxt = *lv[l + 1];
        const auto a = arrays<T>(cur);
        const T *xc = reinterpret_cast<const T *>(nxt.vx.get());
        T *xp = reinterpret_cast<T *>(cur.vxp.get());
        const RowLaunch LP = row_launch(cur.n, cur.gP);
        const RowLaunch LA = row_launch(cur.n, cur.gA);
        if (l == 0) {
            const int prp = cg ? prof_begin(ctx, OCP_KERNEL_VC_PROLONG0) : -1;
            OCP_DISPATCH_G(cur.gP, (k_vc_prolong<G, T, double><<<LP.blocks, kBlock, 0, s>>>(
                                       cur.n, LP.iters, cur.P_rp.get(), cur.P_col.get(), a.P, a.d, r_in, xc, xp, cg)));
            prof_end(ctx, prp);
            OCP_LAUNCH_CHECK();
            if (cg) {
                const int pro = prof_begin(ctx, OCP_KERNEL_VC_POST0);
                OCP_DISPATCH_G(cur.gA, (k_vc_post<G, T, double, double, true><<<LA.blocks, kBlock, 0, s>>>(
                                           cur.n, LA.iters, cur.A_rp, cur.A_col, a.A, a.d, r_in, xp, z_out, cg, part,
                                           cnt)));
                prof_end(ctx, pro);
            } else {
                OCP_DISPATCH_G(cur.gA, (k_vc_post<G, T, double, double, false><<<LA.blocks, kBlock, 0, s>>>(
                                           cur.n, LA.iters, cur.A_rp, cur.A_col, a.A, a.d, r_in, xp, z_out, nullptr,
                                           nullptr, nullptr)));
            }
        } else {
            const T *b = reinterpret_cast<const T *>(cur.vb.get());
            T *x = reinterpret_cast<T *>(cur.vx.get());
            OCP_DISPATCH_G(cur.gP, (k_vc_prolong<G, T, T><<<LP.blocks, kBlock, 0, s>>>(
                                       cur.n, LP.iters, cur.P_rp.get(), cur.P_col.get(), a.P, a.d, b, xc, xp, cg)));
            OCP_LAUNCH_CHECK();
            OCP_DISPATCH_G(cur.gA, (k_vc_post<G, T, T, T, false><<<LA.blocks, kBlock, 0, s>>>(
                                       cur.n, LA.iters, cur.A_rp, cur.A_col, a.A, a.d, b, xp, x, cg, nullptr,
                                       nullptr)));
        }
        OCP_LAUNCH_CHECK();
    }
}

void vcycle_enqueue(ocp_ctx *ctx, const ocp_hierarchy *h, const double *r, double *z, CgScalars *cg) {
    if (h->params.precision == OCP_PREC_MIXED)
        vcycle_t<float>(ctx, h, r, z, cg);
    else
        vcycle_t<double>(ctx, h, r, z, cg);
}

int level_lanes(int64_t nnz, int64_t rows) { return lanes_for(nnz, rows); }

}  // namespace ocp

using namespace ocp;

extern "C" int amg_vcycle(ocp_ctx *ctx, const ocp_hierarchy *h, const double *r, double *z) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    return run_guarded(ctx, [&] {
        if (!h || !r || !z) fail(OCP_ERR_INVALID_ARG, "hierarchy, r and z must not be NULL");
        vcycle_enqueue(ctx, h, r, z, nullptr);
    });
}
