// Application of the AMG preconditioner B: one V(1,1)-cycle with zero
// initial guess (Section 4.1: pre-smoothing, restriction with P^T, recursive
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

// Residual with the iterate formed on the fly from vectors already in memory:
//   x_j = [X0_j] + d_j (alpha u_j [+ beta v_j]),   r_i = b_i - sum_j a_ij x_j
// MODE 0 writes r; MODE 1 writes z_i = [X0_i] + d_i (e1 u_i + e2 r_i) (and with
// DOT also accumulates b.z for CG).  Every smoothing step of the V-cycle is
// one instance of this kernel, i.e. one pass over the level matrix.
template <int G, typename T, typename BT, typename UT, typename OT, bool HX0, bool HU, bool HV, int MODE, bool DOT>
__global__ void __launch_bounds__(kBlock) k_smooth(int32_t n, int iters, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col, const T *__restrict__ val,
                                                   const T *__restrict__ d, const BT *__restrict__ b,
                                                   const T *__restrict__ x0, const UT *__restrict__ u,
                                                   const T *__restrict__ v, T alpha, T beta, T e1, T e2,
                                                   OT *__restrict__ out, CgScalars *cg, double *partials,
                                                   unsigned *counter) {
    if (cg && cg->flag) return;
    double acc = 0.0;
    OCP_ROWS_BEGIN(G)
    const T s = dev::row_sum<G>(rp[row], rp[row + 1], lane, col, val, [&](int c) {
        T x = HX0 ? x0[c] : T(0);
        if (HU) {
            T w = alpha * (T)u[c];
            if (HV) w += beta * v[c];
            x += d[c] * w;
        }
        return x;
    });
    if (lane == 0) {
        const BT bi = b[row];
        const T r = (T)bi - s;
        if (MODE == 0) {
            out[row] = (OT)r;
        } else {
            T w = e2 * r;
            if (HU) w += e1 * (T)u[row];
            const T z = (HX0 ? x0[row] : T(0)) + d[row] * w;
            out[row] = (OT)z;
            if (DOT) acc += (double)bi * (double)z;
        }
    }
    OCP_ROWS_END()
    if (DOT) {
        acc = dev::block_sum<kBlock>(acc);
        double tot;
        if (dev::grid_sum_last<kBlock>(acc, partials, counter, &tot) && threadIdx.x == 0)
            dev::cg_after_precond(cg, tot);
    }
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

// xp = d .* (alpha b [+ beta v]) + P xc: the pre-smoothed iterate rebuilt from
// the vectors that defined it, plus the coarse-grid correction
template <int G, typename T, typename BT, bool HV>
__global__ void __launch_bounds__(kBlock) k_vc_prolong(int32_t n, int iters, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col, const T *__restrict__ val,
                                                       const T *__restrict__ d, const BT *__restrict__ b,
                                                       const T *__restrict__ v, T alpha, T beta,
                                                       const T *__restrict__ xc, T *__restrict__ xp,
                                                       const CgScalars *cg) {
    if (cg && cg->flag) return;
    OCP_ROWS_BEGIN(G)
    const T s = dev::row_sum<G>(rp[row], rp[row + 1], lane, col, val, [&](int c) { return xc[c]; });
    if (lane == 0) {
        T w = alpha * (T)b[row];
        if (HV) w += beta * v[row];
        xp[row] = d[row] * w + s;
    }
    OCP_ROWS_END()
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
    const T zero = T(0);

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

    // ---- down: pre-smoothing from zero, residual, restriction
    auto down = [&](int l, auto bptr) {
        using BT = std::remove_const_t<std::remove_pointer_t<decltype(bptr)>>;
        const Level &cur = *lv[l];
        const Level &nxt = *lv[l + 1];
        const auto a = arrays<T>(cur);
        T *r1 = reinterpret_cast<T *>(cur.vr.get());
        T *r2 = reinterpret_cast<T *>(cur.vr2.get());
        const RowLaunch LA = row_launch(cur.n, cur.gA);
        const T ca = (T)cur.cheb_a, c1 = (T)cur.cheb_c1, c2 = (T)cur.cheb_c2;
        const int pr = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_PRE0) : -1;
        OCP_DISPATCH_G(cur.gA, (k_smooth<G, T, BT, BT, T, false, true, false, 0, false><<<LA.blocks, kBlock, 0, s>>>(
                                   cur.n, LA.iters, cur.A_rp, cur.A_col, a.A, a.d, bptr, nullptr, bptr, nullptr, ca,
                                   zero, zero, zero, r1, cg, nullptr, nullptr)));
        prof_end(ctx, pr);
        OCP_LAUNCH_CHECK();
        const T *rr = r1;
        if (cur.deg == 2) {
            const int pr2 = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_PRE0_B) : -1;
            OCP_DISPATCH_G(cur.gA, (k_smooth<G, T, BT, BT, T, false, true, true, 0, false><<<LA.blocks, kBlock, 0, s>>>(
                                       cur.n, LA.iters, cur.A_rp, cur.A_col, a.A, a.d, bptr, nullptr, bptr, r1, c1, c2,
                                       zero, zero, r2, cg, nullptr, nullptr)));
            prof_end(ctx, pr2);
            OCP_LAUNCH_CHECK();
            rr = r2;
        }
        T *bn = reinterpret_cast<T *>(nxt.vb.get());
        const RowLaunch LR = row_launch(nxt.n, cur.gR);
        const int prr = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_RESTRICT0) : -1;
        OCP_DISPATCH_G(cur.gR, (k_vc_spmv<G, T><<<LR.blocks, kBlock, 0, s>>>(nxt.n, LR.iters, cur.R_rp.get(),
                                                                              cur.R_col.get(), a.R, rr, bn, cg)));
        prof_end(ctx, prr);
        OCP_LAUNCH_CHECK();
    };
    for (int l = 0; l < L - 1; ++l) {
        if (l == 0)
            down(0, r_in);
        else
            down(l, reinterpret_cast<const T *>(lv[l]->vb.get()));
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
    // ---- up: prolongation + correction, post-smoothing
    auto up = [&](int l, auto bptr, auto outptr, bool dot) {
        using BT = std::remove_const_t<std::remove_pointer_t<decltype(bptr)>>;
        using OT = std::remove_pointer_t<decltype(outptr)>;
        const Level &cur = *lv[l];
        const Level &nxt = *lv[l + 1];
        const auto a = arrays<T>(cur);
        const T *xc = reinterpret_cast<const T *>(nxt.vx.get());
        T *xp = reinterpret_cast<T *>(cur.vxp.get());
        T *r1 = reinterpret_cast<T *>(cur.vr.get());
        T *r0 = reinterpret_cast<T *>(cur.vr2.get());
        const T ca = (T)cur.cheb_a, c1 = (T)cur.cheb_c1, c2 = (T)cur.cheb_c2;
        const RowLaunch LP = row_launch(cur.n, cur.gP);
        const RowLaunch LA = row_launch(cur.n, cur.gA);
        const int prp = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_PROLONG0) : -1;
        if (cur.deg == 2) {
            OCP_DISPATCH_G(cur.gP, (k_vc_prolong<G, T, BT, true><<<LP.blocks, kBlock, 0, s>>>(
                                       cur.n, LP.iters, cur.P_rp.get(), cur.P_col.get(), a.P, a.d, bptr, r1, c1, c2,
                                       xc, xp, cg)));
        } else {
            OCP_DISPATCH_G(cur.gP, (k_vc_prolong<G, T, BT, false><<<LP.blocks, kBlock, 0, s>>>(
                                       cur.n, LP.iters, cur.P_rp.get(), cur.P_col.get(), a.P, a.d, bptr, nullptr, ca,
                                       zero, xc, xp, cg)));
        }
        prof_end(ctx, prp);
        OCP_LAUNCH_CHECK();
        int pro = -1;
        if (cur.deg == 2) {
            // r0 = b - A xp, then z = xp + D^-1 (c1 r0 + c2 r1) with r1 = b - A (xp + a D^-1 r0)
            const int pra = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_POST0_A) : -1;
            OCP_DISPATCH_G(cur.gA, (k_smooth<G, T, BT, T, T, true, false, false, 0, false><<<LA.blocks, kBlock, 0, s>>>(
                                       cur.n, LA.iters, cur.A_rp, cur.A_col, a.A, a.d, bptr, xp, nullptr, nullptr,
                                       zero, zero, zero, zero, r0, cg, nullptr, nullptr)));
            prof_end(ctx, pra);
            OCP_LAUNCH_CHECK();
            pro = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_POST0) : -1;
            if (dot) {
                OCP_DISPATCH_G(cur.gA, (k_smooth<G, T, BT, T, OT, true, true, false, 1, true><<<LA.blocks, kBlock, 0, s>>>(
                                           cur.n, LA.iters, cur.A_rp, cur.A_col, a.A, a.d, bptr, xp, r0, nullptr, ca,
                                           zero, c1, c2, outptr, cg, part, cnt)));
            } else {
                OCP_DISPATCH_G(cur.gA, (k_smooth<G, T, BT, T, OT, true, true, false, 1, false><<<LA.blocks, kBlock, 0, s>>>(
                                           cur.n, LA.iters, cur.A_rp, cur.A_col, a.A, a.d, bptr, xp, r0, nullptr, ca,
                                           zero, c1, c2, outptr, cg, nullptr, nullptr)));
            }
        } else {
            // z = xp + a D^-1 (b - A xp)
            pro = (cg && l == 0) ? prof_begin(ctx, OCP_KERNEL_VC_POST0) : -1;
            if (dot) {
                OCP_DISPATCH_G(cur.gA, (k_smooth<G, T, BT, T, OT, true, false, false, 1, true><<<LA.blocks, kBlock, 0, s>>>(
                                           cur.n, LA.iters, cur.A_rp, cur.A_col, a.A, a.d, bptr, xp, nullptr, nullptr,
                                           zero, zero, zero, ca, outptr, cg, part, cnt)));
            } else {
                OCP_DISPATCH_G(cur.gA, (k_smooth<G, T, BT, T, OT, true, false, false, 1, false><<<LA.blocks, kBlock, 0, s>>>(
                                           cur.n, LA.iters, cur.A_rp, cur.A_col, a.A, a.d, bptr, xp, nullptr, nullptr,
                                           zero, zero, zero, ca, outptr, cg, nullptr, nullptr)));
            }
        }
        prof_end(ctx, pro);
        OCP_LAUNCH_CHECK();
    };
    for (int l = L - 2; l >= 0; --l) {
        if (l == 0)
            up(0, r_in, z_out, cg != nullptr);
        else
            up(l, reinterpret_cast<const T *>(lv[l]->vb.get()), reinterpret_cast<T *>(lv[l]->vx.get()), false);
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
