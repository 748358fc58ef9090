// Preconditioned conjugate gradients for A u = f (Section 4: PCG with the
// AMG V-cycle as preconditioner, stopped at a relative residual tolerance).
//
// All scalars (alpha, beta, gamma, residual norms, the stop flag) live on the
// device: the last block of each reducing kernel finishes the reduction in a
// fixed order and updates them, so an iteration is a chain of kernels with no
// host round trip.  The host enqueues a few iterations at a time and then
// reads the flag; kernels enqueued after convergence return immediately.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.h"
#include "system.h"

namespace ocp {


// ------------------------------------------------------------------ SpMV
// y = A x on the sliced-ELL copy
__global__ void __launch_bounds__(kBlock) k_spmv_sell(int32_t n, int64_t nslices, int spb, const int32_t *__restrict__ sp,
                                                      const int32_t *__restrict__ sw, SellCols col,
                                                      const double *__restrict__ val, const double *__restrict__ x,
                                                      double *__restrict__ y) {
    OCP_SELL_BEGIN(nslices, spb)
    const double s = dev::sell_row_c(col, slice, row, n, val, base, w, [&](int c) { return x[c]; });
    if (row < n) y[row] = s;
    OCP_SELL_END()
}

// q = A p and alpha = gamma / (p.q), sliced-ELL fine matrix
__global__ void __launch_bounds__(kBlock) k_cg_spmv_pq_sell(int32_t n, int64_t nslices, int spb,
                                                            const int32_t *__restrict__ sp,
                                                            const int32_t *__restrict__ sw, SellCols col,
                                                            const double *__restrict__ val,
                                                            const double *__restrict__ p, double *__restrict__ q,
                                                            CgScalars *cg, double *partials) {
    if (cg->flag) return;
    double acc = 0.0;
    OCP_SELL_BEGIN(nslices, spb)
    const double s = dev::sell_row_c(col, slice, row, n, val, base, w, [&](int c) { return p[c]; });
    if (row < n) {
        q[row] = s;
        acc += s * p[row];
    }
    OCP_SELL_END()
    acc = dev::block_sum<kBlock>(acc);
    dev::store_partial(acc, partials);
}

// alpha = gamma / (p.q) from the partials of k_cg_spmv_pq_sell
__global__ void __launch_bounds__(kFinBlock) k_fin_alpha(unsigned nb, const double *partials, CgScalars *cg) {
    if (cg->flag) return;
    const double tot = dev::sum_partials<kFinBlock>(partials, nb);
    if (threadIdx.x == 0) {
        cg->pq = tot;
        if (!(tot > 0.0) || !isfinite(tot)) {
            cg->flag = 2;
            cg->alpha = 0.0;
        } else {
            cg->alpha = cg->gamma / tot;
        }
    }
}

// sum_i (f_i - (A x)_i)^2 on the sliced-ELL copy
__global__ void __launch_bounds__(kBlock) k_resid2_sell(int32_t n, int64_t nslices, int spb, const int32_t *__restrict__ sp,
                                                        const int32_t *__restrict__ sw, SellCols col,
                                                        const double *__restrict__ val, const double *__restrict__ x,
                                                        const double *__restrict__ f, double *partials) {
    double acc = 0.0;
    OCP_SELL_BEGIN(nslices, spb)
    const double s = dev::sell_row_c(col, slice, row, n, val, base, w, [&](int c) { return x[c]; });
    if (row < n) {
        const double d = f[row] - s;
        acc += d * d;
    }
    OCP_SELL_END()
    acc = dev::block_sum<kBlock>(acc);
    dev::store_partial(acc, partials);
}

__global__ void __launch_bounds__(kFinBlock) k_fin_store(unsigned nb, const double *partials, double *out) {
    const double tot = dev::sum_partials<kFinBlock>(partials, nb);
    if (threadIdx.x == 0) *out = tot;
}

// x += alpha p, r -= alpha q, r.r; with JAC also z = dinv r and r.z.
template <bool JAC, typename YT>
__global__ void __launch_bounds__(kBlock) k_cg_update(int32_t n, int iters, double *__restrict__ x,
                                                      double *__restrict__ r, const double *__restrict__ p,
                                                      const double *__restrict__ q, const double *__restrict__ dinv,
                                                      double *__restrict__ z, FirstStep<YT> first, CgScalars *cg,
                                                      double *partials) {
    if (cg->flag) return;
    const double alpha = cg->alpha;
    const unsigned tile = dev::xcd_tile(blockIdx.x, gridDim.x);
    const int base = (int)tile * kBlock * iters;
    double rr = 0.0, rz = 0.0;
    for (int it = 0; it < iters; ++it) {
        const int i = base + it * kBlock + threadIdx.x;
        if (i < n) {
            x[i] += alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            r[i] = ri;
            first.put(i, i, ri);
            rr += ri * ri;
            if (JAC) {
                const double zi = dinv[i] * ri;
                z[i] = zi;
                rz += ri * zi;
            }
        }
    }
    double2 bs = dev::block_sum2<kBlock>(rr, rz);
    dev::store_partial2(bs, partials);
}

// r.r (and r.z with JAC) from the partials of k_cg_update: stop tests
template <bool JAC>
__global__ void __launch_bounds__(kBlock) k_fin_update(unsigned nb, const double *partials, CgScalars *cg) {
    if (cg->flag) return;
    const double rr = dev::sum_partials<kBlock>(partials, nb, 2, 0);
    const double rz = JAC ? dev::sum_partials<kBlock>(partials, nb, 2, 1) : 0.0;
    if (threadIdx.x == 0) {
        const double2 tot = make_double2(rr, rz);
        cg->rr = tot.x;
        cg->iter += 1;
        if (cg->stop_mode == OCP_STOP_L2 && tot.x <= cg->tol2) {
            cg->flag = 1;
        } else if (!isfinite(tot.x)) {
            cg->flag = 2;
        } else {
            if (JAC) dev::cg_after_precond(cg, tot.y);
            if (cg->flag == 0 && cg->iter >= cg->maxit) cg->flag = 3;
        }
    }
}

// p = z + beta p
__global__ void __launch_bounds__(kBlock) k_cg_pupdate(int32_t n, double *__restrict__ p, const double *__restrict__ z,
                                                       const CgScalars *cg) {
    if (cg->flag) return;
    const double beta = cg->beta;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = z[i] + beta * p[i];
}

// Flexible (Polak-Ribiere) beta = r'.(z' - z) / (r.z): the partials of
// r'.z with the previous z, then beta -= r'.z / gamma_prev.  Used when the
// preconditioner is applied in lower precision and so is symmetric only to
// rounding.
__global__ void __launch_bounds__(kBlock) k_cg_rzold(int32_t n, int iters, const double *__restrict__ r,
                                                     const double *__restrict__ zold, const CgScalars *cg,
                                                     double *partials) {
    if (cg->flag) return;
    const unsigned tile = dev::xcd_tile(blockIdx.x, gridDim.x);
    const int base = (int)tile * kBlock * iters;
    double s = 0.0;
    for (int it = 0; it < iters; ++it) {
        const int i = base + it * kBlock + threadIdx.x;
        if (i < n) s += r[i] * zold[i];
    }
    dev::store_partial(dev::block_sum<kBlock>(s), partials);
}

__global__ void __launch_bounds__(kBlock) k_fin_flex(unsigned nb, const double *partials, CgScalars *cg) {
    if (cg->flag) return;
    const double tot = dev::sum_partials<kBlock>(partials, nb);
    if (threadIdx.x == 0 && cg->iter > 0) cg->beta -= tot / cg->gamma_prev;
}

// x = 0, r = f, p = 0, f.f and the initial scalars
template <typename YT>
__global__ void __launch_bounds__(kBlock) k_cg_init(int32_t n, int iters, const double *__restrict__ f,
                                                    double *__restrict__ x, double *__restrict__ r,
                                                    double *__restrict__ p, FirstStep<YT> first, double *partials) {
    const unsigned tile = dev::xcd_tile(blockIdx.x, gridDim.x);
    const int base = (int)tile * kBlock * iters;
    double ff = 0.0;
    for (int it = 0; it < iters; ++it) {
        const int i = base + it * kBlock + threadIdx.x;
        if (i < n) {
            const double fi = f[i];
            x[i] = 0.0;
            r[i] = fi;
            p[i] = 0.0;
            first.put(i, i, fi);
            ff += fi * fi;
        }
    }
    ff = dev::block_sum<kBlock>(ff);
    dev::store_partial(ff, partials);
}

__global__ void __launch_bounds__(kBlock) k_fin_init(unsigned nb, const double *partials, CgScalars *cg, double rtol,
                                                     int mode, int maxit) {
    const double tot = dev::sum_partials<kBlock>(partials, nb);
    if (threadIdx.x == 0) {
        cg->ff = tot;
        cg->rr = tot;
        cg->tol2 = (mode == OCP_STOP_L2) ? rtol * rtol * tot : rtol * rtol;
        cg->gamma = 1.0;
        cg->gamma0 = 0.0;
        cg->alpha = 0.0;
        cg->beta = 0.0;
        cg->pq = 0.0;
        cg->rz_new = 0.0;
        cg->gamma_prev = 1.0;
        cg->iter = 0;
        cg->stop_mode = mode;
        cg->maxit = maxit;
        cg->flag = (tot == 0.0) ? 1 : (isfinite(tot) ? 0 : 2);
    }
}

// z = dinv r and r.z (Jacobi preconditioner at the start)
__global__ void __launch_bounds__(kBlock) k_cg_jacobi(int32_t n, int iters, const double *__restrict__ r,
                                                      const double *__restrict__ dinv, double *__restrict__ z,
                                                      CgScalars *cg, double *partials) {
    if (cg->flag) return;
    const unsigned tile = dev::xcd_tile(blockIdx.x, gridDim.x);
    const int base = (int)tile * kBlock * iters;
    double rz = 0.0;
    for (int it = 0; it < iters; ++it) {
        const int i = base + it * kBlock + threadIdx.x;
        if (i < n) {
            const double zi = dinv[i] * r[i];
            z[i] = zi;
            rz += r[i] * zi;
        }
    }
    rz = dev::block_sum<kBlock>(rz);
    dev::store_partial(rz, partials);
}

// r.z from the partials of a preconditioner application
__global__ void __launch_bounds__(kBlock) k_fin_rz(unsigned nb, const double *partials, CgScalars *cg) {
    if (cg->flag) return;
    const double tot = dev::sum_partials<kBlock>(partials, nb);
    if (threadIdx.x == 0) dev::cg_after_precond(cg, tot);
}

__global__ void k_scatter(int32_t nv, const int32_t *__restrict__ dof_of_vertex, const double *__restrict__ x,
                          double *__restrict__ u) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const int d = dof_of_vertex[v];
    u[v] = d >= 0 ? x[d] : 0.0;
}

__global__ void k_diag_inv(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const double *__restrict__ val, double *__restrict__ dinv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k)
        if (col[k] == i) d = val[k];
    dinv[i] = 1.0 / d;
}

// --------------------------------------------------------------- host side
bool hierarchy_fits(const ocp_hierarchy *h, const ocp_system *sys) {
    const ocp_system *o = h->sys;
    if (o == sys) return true;
    return o && sys && o->nv == sys->nv && o->n == sys->n && o->nt == sys->nt && o->nnz == sys->nnz &&
           o->tets_ref == sys->tets_ref;
}

void check_hierarchy(const ocp_hierarchy *h, const ocp_system *sys) {
    if (!h) return;
    if (!hierarchy_fits(h, sys)) fail(OCP_ERR_INVALID_ARG, "hierarchy is for a system on another mesh or pattern");
    if (h->sys->generation.load(std::memory_order_acquire) != h->sys_generation)
        fail(OCP_ERR_INVALID_ARG, "hierarchy is stale: fe_set_rho changed its system after amg_setup; rebuild it");
}

const Sell &system_sell(ocp_ctx *, const ocp_system *sys) {
    if (!sys->sell.val.get()) fail(OCP_ERR_INVALID_ARG, "system has no solve-phase matrix copy");
    return sys->sell;
}

const double *system_dinv(ocp_ctx *ctx, const ocp_system *csys) {
    ocp_system *sys = const_cast<ocp_system *>(csys);   // derived data only, under the system's lock
    if (!sys->dinv_ready.load(std::memory_order_acquire)) {
        std::lock_guard<std::mutex> lock(sys->derived_mu);
        if (!sys->dinv_ready.load(std::memory_order_relaxed)) {
            // allocated through the system's own context (it lives as long as
            // the system), filled on the caller's stream and waited for before
            // any other context may see it
            sys->dinv.reset(sys->ctx, (size_t)sys->n);
            k_diag_inv<<<grid_for(sys->n, 256), 256, 0, ctx->stream>>>(sys->n, sys->row_ptr.get(), sys->col.get(),
                                                                       sys->val.get(), sys->dinv.get());
            OCP_LAUNCH_CHECK();
            sync(ctx);
            sys->dinv_ready.store(true, std::memory_order_release);
        }
    }
    return sys->dinv.get();
}

// One PCG solve in progress: its vectors, its device scalars and its
// reduction partials (its own, so several solves can be enqueued on one
// stream, as the packed batch does).
struct SolveState {
    ocp_ctx *ctx = nullptr;
    ocp_system *sys = nullptr;
    const ocp_hierarchy *h = nullptr;
    const double *f = nullptr;
    const double *dinv = nullptr;
    DevBuf<double> x, r, p, q, z, z2;
    DevBuf<double> own_dinv;   // Jacobi diagonal of an allocation-free solve (not published)
    DevBuf<char> y0;         // level 0's first smoothing step of r (hierarchies of 2+ levels)
    bool flexible = false;   // Polak-Ribiere beta with the previous z (AMG only)
    int zsel = 0;            // which of z / z2 receives the next preconditioned residual
    VcWork vw;           // V-cycle work vectors of this solve
    DevBuf<CgScalars> cgbuf;
    DevBuf<double> partbuf;   // [4][kRedBlocks]: p.q, r.r / r.z, residual, V-cycle r.z
    CgScalars *cg = nullptr;
    double *part = nullptr;
    int mode = OCP_STOP_L2;
    int32_t maxit = 0;
    double rtol = 0.0;
    int host_iter = 0;   // iterations enqueued (host count)
};

// Call fn with the FirstStep that the kernels producing r fill for the
// V-cycle (y = a D0^-1 r in the hierarchy's precision), or an empty one.
template <typename Fn>
static void with_first_step(const SolveState &S, Fn &&fn) {
    if (!S.y0.get()) {
        fn(FirstStep<float>{nullptr, nullptr, 0.f});
        return;
    }
    const Level &l0 = *S.h->levels[0];
    if (S.h->params.precision == OCP_PREC_MIXED)
        fn(FirstStep<float>{reinterpret_cast<float *>(S.y0.get()), l0.dinv32.get(), (float)l0.cheb_a});
    else
        fn(FirstStep<double>{reinterpret_cast<double *>(S.y0.get()), l0.dinv.get(), l0.cheb_a});
}

// Allocate and enqueue x = 0, r = f, the first preconditioner application
// and p = z (no host synchronization).
static void solve_begin(SolveState &S, ocp_ctx *ctx, ocp_system *sys, const ocp_hierarchy *h, const double *f_in,
                        double rtol, int32_t maxit, int32_t flags) {
    S.ctx = ctx;
    S.sys = sys;
    S.h = h;
    S.rtol = rtol;
    S.maxit = maxit;
    const int32_t n = sys->n;
    S.f = f_in ? f_in : sys->f.get();
    S.x.reset(ctx, n);
    S.r.reset(ctx, n);
    S.p.reset(ctx, n);
    S.q.reset(ctx, n);
    S.z.reset(ctx, n);
    S.flexible = h && (flags & OCP_FLEXIBLE);
    if (S.flexible) S.z2.reset(ctx, n);
    S.zsel = 0;
    if (h) {
        S.dinv = nullptr;
    } else if (ctx->bump_base && !sys->dinv_ready.load(std::memory_order_acquire)) {
        // allocation-free solve before any Jacobi solve built the system's
        // diagonal: a private copy in the scratch region
        S.own_dinv.reset(ctx, n);
        k_diag_inv<<<grid_for(n, 256), 256, 0, ctx->stream>>>(n, sys->row_ptr.get(), sys->col.get(), sys->val.get(),
                                                               S.own_dinv.get());
        OCP_LAUNCH_CHECK();
        S.dinv = S.own_dinv.get();
    } else {
        S.dinv = system_dinv(ctx, sys);
    }
    S.cgbuf.reset(ctx, 1);
    S.partbuf.reset(ctx, (size_t)4 * kRedBlocks);
    S.cg = S.cgbuf.get();
    S.part = S.partbuf.get();
    if (h) {
        vc_work_alloc(ctx, h, S.vw);
        S.vw.part = S.part + 3 * kRedBlocks;
        if (h->levels.size() > 1 && h->params.method == OCP_AMG_AGGREGATION) {
            const size_t vs = h->params.precision == OCP_PREC_MIXED ? sizeof(float) : sizeof(double);
            S.y0.reset(ctx, (size_t)n * vs);
            S.vw.y0 = S.y0.get();
        }
    }
    S.mode = (flags & OCP_STOP_PRECOND) ? OCP_STOP_PRECOND : OCP_STOP_L2;
    CgScalars *cg = S.cg;
    double *part0 = S.part;
    double *part1 = S.part + kRedBlocks;
    system_sell(ctx, sys);
    const RowLaunch LV = vec_launch(n);
    ctx->prof_iter = -1;   // the initial preconditioner application
    OCP_HIP(hipEventRecord(ctx->ev0, ctx->stream));
    with_first_step(S, [&](auto fs) {
        k_cg_init<<<LV.blocks, kBlock, 0, ctx->stream>>>(n, LV.iters, S.f, S.x.get(), S.r.get(), S.p.get(), fs,
                                                         part0);
    });
    k_fin_init<<<1, kBlock, 0, ctx->stream>>>(LV.blocks, part0, cg, rtol, S.mode, maxit);
    OCP_LAUNCH_CHECK();
    if (h) {
        vcycle_enqueue(ctx, h, S.r.get(), S.z.get(), cg, S.vw);
    } else {
        k_cg_jacobi<<<LV.blocks, kBlock, 0, ctx->stream>>>(n, LV.iters, S.r.get(), S.dinv, S.z.get(), cg, part1);
        k_fin_rz<<<1, kBlock, 0, ctx->stream>>>(LV.blocks, part1, cg);
    }
    OCP_LAUNCH_CHECK();
    k_cg_pupdate<<<grid_for(n, kBlock), kBlock, 0, ctx->stream>>>(n, S.p.get(), S.z.get(), cg);
    OCP_LAUNCH_CHECK();
    S.zsel = 1;   // flexible: the next preconditioned residual goes to z2
    ctx->prof_iter = 0;
}

// Enqueue `iters` PCG iterations; kernels of iterations after the stop
// return at once on the device flag.
static void solve_iterate(SolveState &S, int iters) {
    ocp_ctx *ctx = S.ctx;
    const int32_t n = S.sys->n;
    CgScalars *cg = S.cg;
    double *part0 = S.part;
    double *part1 = S.part + kRedBlocks;
    const Sell &A = system_sell(ctx, S.sys);
    const SellLaunch LS = sell_launch(A.nslices);
    const RowLaunch LV = vec_launch(n);
    const unsigned gp = grid_for(n, kBlock);
    for (int k = 0; k < iters; ++k) {
        const int pr = prof_begin(ctx, OCP_KERNEL_CG_SPMV);
        k_cg_spmv_pq_sell<<<LS.blocks, kBlock, 0, ctx->stream>>>(n, A.nslices, LS.slices_per_block, A.sp.get(),
                                                                 A.sw.get(), sell_cols(A), A.val.get(), S.p.get(),
                                                                 S.q.get(), cg, part0);
        prof_end(ctx, pr);
        k_fin_alpha<<<1, kFinBlock, 0, ctx->stream>>>(LS.blocks, part0, cg);
        double *znew = S.z.get();
        if (S.h) {
            with_first_step(S, [&](auto fs) {
                k_cg_update<false><<<LV.blocks, kBlock, 0, ctx->stream>>>(
                    n, LV.iters, S.x.get(), S.r.get(), S.p.get(), S.q.get(), nullptr, nullptr, fs, cg, part1);
            });
            k_fin_update<false><<<1, kBlock, 0, ctx->stream>>>(LV.blocks, part1, cg);
            if (S.flexible) {
                znew = S.zsel ? S.z2.get() : S.z.get();
                const double *zold = S.zsel ? S.z.get() : S.z2.get();
                vcycle_enqueue(ctx, S.h, S.r.get(), znew, cg, S.vw);
                double *part2 = S.part + 2 * kRedBlocks;
                k_cg_rzold<<<LV.blocks, kBlock, 0, ctx->stream>>>(n, LV.iters, S.r.get(), zold, cg, part2);
                k_fin_flex<<<1, kBlock, 0, ctx->stream>>>(LV.blocks, part2, cg);
                S.zsel ^= 1;
            } else {
                vcycle_enqueue(ctx, S.h, S.r.get(), znew, cg, S.vw);
            }
        } else {
            k_cg_update<true><<<LV.blocks, kBlock, 0, ctx->stream>>>(n, LV.iters, S.x.get(), S.r.get(), S.p.get(),
                                                                     S.q.get(), S.dinv, S.z.get(),
                                                                     FirstStep<float>{nullptr, nullptr, 0.f}, cg, part1);
            k_fin_update<true><<<1, kBlock, 0, ctx->stream>>>(LV.blocks, part1, cg);
        }
        k_cg_pupdate<<<gp, kBlock, 0, ctx->stream>>>(n, S.p.get(), znew, cg);
        ++ctx->prof_iter;
        ++S.host_iter;
    }
    OCP_LAUNCH_CHECK();
}

// After the stop: true residual in double, u on all vertices, the info
// record; synchronizes the context stream.
static int solve_finish(SolveState &S, double *u, ocp_solve_info *info) {
    ocp_ctx *ctx = S.ctx;
    ocp_system *sys = S.sys;
    const int32_t n = sys->n;
    double *part2 = S.part + 2 * kRedBlocks;
    const Sell &A = system_sell(ctx, sys);
    const SellLaunch LS = sell_launch(A.nslices);
    OCP_HIP(hipEventRecord(ctx->ev1, ctx->stream));
    k_resid2_sell<<<LS.blocks, kBlock, 0, ctx->stream>>>(n, A.nslices, LS.slices_per_block, A.sp.get(), A.sw.get(),
                                                         sell_cols(A), A.val.get(), S.x.get(), S.f, part2);
    k_fin_store<<<1, kFinBlock, 0, ctx->stream>>>(LS.blocks, part2, part2 + kRedBlocks - 1);
    OCP_LAUNCH_CHECK();
    k_scatter<<<grid_for(sys->nv, 256), 256, 0, ctx->stream>>>(sys->nv, sys->dof_of_vertex.get(), S.x.get(), u);
    OCP_LAUNCH_CHECK();
    CgScalars hs{};
    read_back(ctx, &hs, S.cg, sizeof(hs));
    double res2 = 0.0;
    read_back(ctx, &res2, part2 + kRedBlocks - 1, sizeof(res2));
    float ms = 0.f;
    OCP_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    // every kernel of host iterations 0 .. iter-2 did its full work
    prof_resolve(ctx, hs.iter - 1);
    int st = OCP_OK;
    if (hs.flag == 2) st = OCP_ERR_BREAKDOWN;
    else if (hs.flag == 3) st = OCP_MAXIT;
    else if (hs.flag == 0) st = OCP_MAXIT;   // ended by the caller before the stop
    if (info) {
        info->iterations = hs.iter;
        info->status = st;
        info->rel_res_l2 = hs.ff > 0 ? std::sqrt(hs.rr / hs.ff) : 0.0;
        info->rel_res_precond = hs.gamma0 > 0 ? std::sqrt(hs.gamma / hs.gamma0) : 0.0;
        info->true_rel_res = hs.ff > 0 ? std::sqrt(res2 / hs.ff) : 0.0;
        info->setup_ms = S.h ? S.h->setup_ms : 0.0;
        info->solve_ms = ms;
    }
    return st;
}

static void solve(ocp_ctx *ctx, ocp_system *sys, const ocp_hierarchy *h, const double *f_in, double *u,
                  double rtol, int32_t maxit, int32_t flags, ocp_solve_info *info, int *status) {
    SolveState S;
    solve_begin(S, ctx, sys, h, f_in, rtol, maxit, flags);
    CgScalars hs{};
    int chunk = 2;
    for (;;) {
        read_back(ctx, &hs, S.cg, sizeof(hs));
        if (hs.flag != 0) break;
        solve_iterate(S, chunk);
        if (chunk < 8) chunk *= 2;
    }
    *status = solve_finish(S, u, info);
}

// ------------------------------------------------------------ packed batch
constexpr int kBatchBranches = 8;   // parallel chains of a packed batch graph

bool small_eligible(const ocp_system *sys, const ocp_hierarchy *h);
void small_batch(ocp_ctx *ctx, const std::vector<int> &idx, const ocp_system *const *systems,
                 const ocp_hierarchy *const *hs, const double *const *fs, double *const *us, double rtol,
                 int32_t maxit, int mode, ocp_solve_info *infos, std::vector<int> &st);

// Number of solves of a batch still running (one thread: m is small).
__global__ void k_batch_running(int32_t m, CgScalars *const *cgs, int32_t *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int c = 0;
    for (int i = 0; i < m; ++i) c += cgs[i]->flag == 0;
    *out = c;
}

// m independent solves packed into one graph launch per iteration: the first
// steps are enqueued normally, then one iteration of every solve (and the
// running count) is captured into a HIP graph that is replayed until all
// have stopped.  Each solve runs exactly the kernels of pcg_solve on its own
// vectors and scalars, so its result is the same bits as alone.
static void solve_batch(ocp_ctx *ctx, int m, const ocp_system *const *systems, const ocp_hierarchy *const *hs,
                        const double *const *fs, double *const *us, double rtol, int32_t maxit, int32_t flags,
                        ocp_solve_info *infos, int *status) {
    // the null stream cannot be captured: run the batch on a private stream
    // (default priority), ordered after the context's work by a sync
    struct StreamSwap {
        ocp_ctx *ctx;
        hipStream_t user, own = nullptr;
        explicit StreamSwap(ocp_ctx *c) : ctx(c), user(c->stream) {
            if (user == nullptr) {
                OCP_HIP(hipStreamSynchronize(user));
                OCP_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
                ctx->stream = own;
            }
        }
        ~StreamSwap() {
            if (own) {
                (void)hipStreamSynchronize(own);
                ctx->stream = user;
                (void)hipStreamDestroy(own);
            }
        }
    } swap(ctx);
    std::vector<SolveState> S((size_t)m);
    for (int i = 0; i < m; ++i)
        solve_begin(S[i], ctx, const_cast<ocp_system *>(systems[i]), hs ? hs[i] : nullptr, fs ? fs[i] : nullptr,
                    rtol, maxit, flags & ~OCP_FLEXIBLE);   // a captured iteration has fixed buffers
    std::vector<CgScalars *> hcg((size_t)m);
    for (int i = 0; i < m; ++i) hcg[i] = S[i].cg;
    DevBuf<CgScalars *> dcg(ctx, (size_t)m);
    DevBuf<int32_t> running(ctx, 1);
    OCP_HIP(hipMemcpyAsync(dcg.get(), hcg.data(), sizeof(CgScalars *) * m, hipMemcpyHostToDevice, ctx->stream));
    sync(ctx);

    // the solves are independent: each is captured on one of B forked branch
    // streams, so one replay of the graph holds B parallel chains that the
    // GPU can run side by side
    const int B = std::min(m, kBatchBranches);
    std::vector<hipStream_t> br((size_t)B, nullptr);
    std::vector<hipEvent_t> ev((size_t)B, nullptr);
    struct Cleanup {
        std::vector<hipStream_t> &br;
        std::vector<hipEvent_t> &ev;
        ~Cleanup() {
            for (size_t b = 1; b < br.size(); ++b)
                if (br[b]) (void)hipStreamDestroy(br[b]);
            for (auto e : ev)
                if (e) (void)hipEventDestroy(e);
        }
    } cleanup{br, ev};
    hipStream_t main = ctx->stream;
    br[0] = main;
    for (int b = 0; b < B; ++b) {
        if (b > 0) OCP_HIP(hipStreamCreateWithFlags(&br[b], hipStreamNonBlocking));
        OCP_HIP(hipEventCreateWithFlags(&ev[b], hipEventDisableTiming));
    }
    const bool prof = ctx->profile;
    ctx->profile = false;   // no event timing inside the captured graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    OCP_HIP(hipStreamBeginCapture(main, hipStreamCaptureModeThreadLocal));
    try {
        OCP_HIP(hipEventRecord(ev[0], main));
        for (int b = 1; b < B; ++b) OCP_HIP(hipStreamWaitEvent(br[b], ev[0], 0));
        for (int i = 0; i < m; ++i) {
            ctx->stream = br[i % B];
            solve_iterate(S[i], 1);
        }
        ctx->stream = main;
        for (int b = 1; b < B; ++b) {
            OCP_HIP(hipEventRecord(ev[b], br[b]));
            OCP_HIP(hipStreamWaitEvent(main, ev[b], 0));
        }
        k_batch_running<<<1, 64, 0, main>>>(m, dcg.get(), running.get());
        OCP_LAUNCH_CHECK();
    } catch (...) {
        ctx->stream = main;
        hipGraph_t g2 = nullptr;
        (void)hipStreamEndCapture(main, &g2);
        if (g2) (void)hipGraphDestroy(g2);
        ctx->profile = prof;
        throw;
    }
    ctx->profile = prof;
    OCP_HIP(hipStreamEndCapture(main, &graph));
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        fail(OCP_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    int32_t left = m;
    int chunk = 2, replays = 0;
    while (left > 0 && replays <= maxit) {
        for (int c = 0; c < chunk; ++c) OCP_HIP(hipGraphLaunch(exec, ctx->stream));
        replays += chunk;
        if (chunk < 8) chunk *= 2;
        read_back(ctx, &left, running.get(), sizeof(left));
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    std::vector<int> st((size_t)m);
    for (int i = 0; i < m; ++i) st[i] = solve_finish(S[i], us[i], infos ? &infos[i] : nullptr);
    int w = OCP_OK;
    for (int x : st) {
        if (x == OCP_ERR_BREAKDOWN) w = OCP_ERR_BREAKDOWN;
        else if (x == OCP_MAXIT && w == OCP_OK) w = OCP_MAXIT;
    }
    *status = w;
}

}  // namespace ocp

using namespace ocp;

extern "C" int pcg_solve_batch(ocp_ctx *ctx, int32_t m, const ocp_system *const *systems,
                               const ocp_hierarchy *const *hierarchies, const double *const *f, double *const *u,
                               double rtol, int32_t maxit, int32_t flags, ocp_solve_info *infos) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    int status = OCP_OK;
    int rc = run_guarded(ctx, [&] {
        if (m < 1 || m > 4096) fail(OCP_ERR_INVALID_ARG, "m must lie in 1..4096");
        if (!systems || !u) fail(OCP_ERR_INVALID_ARG, "systems and u must not be NULL");
        if (!(rtol > 0.0) || !std::isfinite(rtol)) fail(OCP_ERR_INVALID_ARG, "rtol must be positive");
        if (maxit < 1) fail(OCP_ERR_INVALID_ARG, "maxit must be >= 1");
        for (int i = 0; i < m; ++i) {
            if (!systems[i] || !u[i]) fail(OCP_ERR_INVALID_ARG, "a system or u entry is NULL");
            if (hierarchies) check_hierarchy(hierarchies[i], systems[i]);
        }
        // small problems: one workgroup each in one persistent launch; the
        // rest: packed into one graph launch per iteration
        std::vector<int> small, big;
        for (int i = 0; i < m; ++i) {
            const ocp_hierarchy *h = hierarchies ? hierarchies[i] : nullptr;
            ((flags & OCP_BATCH_GRAPH) || !small_eligible(systems[i], h) ? big : small).push_back(i);
        }
        std::vector<int> st((size_t)m, OCP_OK);
        if (!big.empty()) {
            std::vector<const ocp_system *> bs;
            std::vector<const ocp_hierarchy *> bh;
            std::vector<const double *> bf;
            std::vector<double *> bu;
            std::vector<ocp_solve_info> bi(big.size());
            for (int i : big) {
                bs.push_back(systems[i]);
                bh.push_back(hierarchies ? hierarchies[i] : nullptr);
                bf.push_back(f ? f[i] : nullptr);
                bu.push_back(u[i]);
            }
            int bst = OCP_OK;
            solve_batch(ctx, (int)big.size(), bs.data(), bh.data(), bf.data(), bu.data(), rtol, maxit, flags,
                        bi.data(), &bst);
            for (size_t t = 0; t < big.size(); ++t) {
                st[big[t]] = bi[t].status;
                if (infos) infos[big[t]] = bi[t];
            }
        }
        if (!small.empty()) {
            const int mode = (flags & OCP_STOP_PRECOND) ? OCP_STOP_PRECOND : OCP_STOP_L2;
            small_batch(ctx, small, systems, hierarchies, f, u, rtol, maxit, mode, infos, st);
        }
        for (int x : st) {
            if (x == OCP_ERR_BREAKDOWN) status = OCP_ERR_BREAKDOWN;
            else if (x == OCP_MAXIT && status == OCP_OK) status = OCP_MAXIT;
        }
    });
    if (rc != OCP_OK) {
        if (infos)
            for (int i = 0; i < std::max(0, std::min<int>(m, 4096)); ++i) infos[i].status = rc;
        return rc;
    }
    if (status == OCP_ERR_BREAKDOWN) ctx->last_error = "CG breakdown in at least one solve";
    return status;
}

extern "C" int ocp_spmv(ocp_ctx *ctx, const ocp_system *sys, const double *x, double *y) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    return run_guarded(ctx, [&] {
        if (!sys || !x || !y) fail(OCP_ERR_INVALID_ARG, "system, x and y must not be NULL");
        const Sell &A = system_sell(ctx, sys);
        const SellLaunch L = sell_launch(A.nslices);
        k_spmv_sell<<<L.blocks, kBlock, 0, ctx->stream>>>(sys->n, A.nslices, L.slices_per_block, A.sp.get(),
                                                          A.sw.get(), sell_cols(A), A.val.get(), x, y);
        OCP_LAUNCH_CHECK();
    });
}

extern "C" int pcg_solve(ocp_ctx *ctx, const ocp_system *sys, const ocp_hierarchy *h, const double *f, double *u,
                         double rtol, int32_t maxit, int32_t flags, ocp_solve_info *info) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    int status = OCP_OK;
    int rc = run_guarded(ctx, [&] {
        if (!sys || !u) fail(OCP_ERR_INVALID_ARG, "system and u must not be NULL");
        if (!(rtol > 0.0) || !std::isfinite(rtol)) fail(OCP_ERR_INVALID_ARG, "rtol must be positive");
        if (maxit < 1) fail(OCP_ERR_INVALID_ARG, "maxit must be >= 1");
        check_hierarchy(h, sys);
        solve(ctx, const_cast<ocp_system *>(sys), h, f, u, rtol, maxit, flags, info, &status);
    });
    if (rc != OCP_OK) {
        if (info) info->status = rc;
        return rc;
    }
    if (status == OCP_ERR_BREAKDOWN) ctx->last_error = "CG breakdown (p^T A p <= 0, r^T z <= 0 or non-finite)";
    return status;
}

// Scratch bytes pcg_solve_noalloc carves for a solve: exactly the buffers
// solve_begin takes (each rounded up to 256 bytes, as the carving does).
static size_t noalloc_bytes(const ocp_system *sys, const ocp_hierarchy *h, int32_t flags) {
    const size_t n = (size_t)sys->n;
    size_t t = 5 * align256(sizeof(double) * n);                                  // x, r, p, q, z
    if (h && (flags & OCP_FLEXIBLE)) t += align256(sizeof(double) * n);          // z2
    if (!h && !sys->dinv_ready.load(std::memory_order_acquire)) t += align256(sizeof(double) * n);
    t += align256(sizeof(CgScalars)) + align256(sizeof(double) * 4 * kRedBlocks);
    if (h) {
        const size_t vs = h->params.precision == OCP_PREC_MIXED ? sizeof(float) : sizeof(double);
        const size_t L = h->levels.size();
        for (size_t l = 0; l < L; ++l) {
            const size_t b = align256((size_t)h->levels[l]->n * vs);
            if (l > 0) t += 2 * b;       // vb, vx
            if (l + 1 < L) t += 4 * b;   // vr, vxp, vx1, vx2
        }
        if (L > 1 && h->params.method == OCP_AMG_AGGREGATION) t += align256(n * vs);   // y0
    }
    return t;
}

extern "C" int pcg_solve_noalloc(ocp_ctx *ctx, const ocp_system *sys, const ocp_hierarchy *h, const double *f,
                                 double *u, double rtol, int32_t maxit, int32_t flags, ocp_solve_info *info) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    int status = OCP_OK;
    int rc = run_guarded(ctx, [&] {
        if (!sys || !u) fail(OCP_ERR_INVALID_ARG, "system and u must not be NULL");
        if (!(rtol > 0.0) || !std::isfinite(rtol)) fail(OCP_ERR_INVALID_ARG, "rtol must be positive");
        if (maxit < 1) fail(OCP_ERR_INVALID_ARG, "maxit must be >= 1");
        check_hierarchy(h, sys);
        char *base = scratch_region(ctx);
        if (!base) fail(OCP_ERR_HIP, "no scratch region on this context's device");
        const size_t need = noalloc_bytes(sys, h, flags);
        if (need > kScratchBytes)
            fail(OCP_ERR_UNSUPPORTED, "pcg_solve_noalloc: this solve needs " + std::to_string(need) +
                                          " bytes of work memory, more than the " +
                                          std::to_string(kScratchBytes >> 20) + " MiB scratch region (use pcg_solve)");
        // every device buffer of the solve is carved from the scratch region;
        // kernel timing (which may create events) is off meanwhile
        struct Carve {
            ocp_ctx *c;
            bool prof;
            Carve(ocp_ctx *c_, char *b) : c(c_), prof(c_->profile) {
                c->bump_base = b;
                c->bump_cap = kScratchBytes;
                c->bump_off = 0;
                c->profile = false;
            }
            ~Carve() {
                c->bump_base = nullptr;
                c->bump_cap = c->bump_off = 0;
                c->profile = prof;
            }
        } carve(ctx, base);
        solve(ctx, const_cast<ocp_system *>(sys), h, f, u, rtol, maxit, flags, info, &status);
    });
    if (rc != OCP_OK) {
        if (info) info->status = rc;
        return rc;
    }
    if (status == OCP_ERR_BREAKDOWN) ctx->last_error = "CG breakdown (p^T A p <= 0, r^T z <= 0 or non-finite)";
    return status;
}

// ------------------------------------------------------------ step API
struct ocp_solve_handle {
    ocp::SolveState S;
    hipEvent_t ev_poll = nullptr;   // recorded after the scalar copy of the last advance
    bool polled_copy = false;
};

extern "C" int pcg_begin(ocp_ctx *ctx, const ocp_system *sys, const ocp_hierarchy *h, const double *f, double rtol,
                         int32_t maxit, int32_t flags, ocp_solve_handle **out) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    return run_guarded(ctx, [&] {
        if (!out) fail(OCP_ERR_INVALID_ARG, "out must not be NULL");
        *out = nullptr;
        if (!sys) fail(OCP_ERR_INVALID_ARG, "system must not be NULL");
        if (!(rtol > 0.0) || !std::isfinite(rtol)) fail(OCP_ERR_INVALID_ARG, "rtol must be positive");
        if (maxit < 1) fail(OCP_ERR_INVALID_ARG, "maxit must be >= 1");
        check_hierarchy(h, sys);
        if (ctx->active_solve) fail(OCP_ERR_INVALID_ARG, "the context already runs a solve (one per context)");
        auto *hd = new ocp_solve_handle();
        try {
            OCP_HIP(hipEventCreateWithFlags(&hd->ev_poll, hipEventDisableTiming));
            solve_begin(hd->S, ctx, const_cast<ocp_system *>(sys), h, f, rtol, maxit, flags);
        } catch (...) {
            if (hd->ev_poll) (void)hipEventDestroy(hd->ev_poll);
            delete hd;
            throw;
        }
        ctx->active_solve = true;
        *out = hd;
    });
}

extern "C" int pcg_advance(ocp_solve_handle *hd, int32_t iters) {
    if (!hd || !hd->S.ctx) return OCP_ERR_INVALID_ARG;
    ocp_ctx *ctx = hd->S.ctx;
    return run_step(ctx, [&] {
        if (iters < 1) fail(OCP_ERR_INVALID_ARG, "iters must be >= 1");
        solve_iterate(hd->S, iters);
        // scalars to the pinned staging buffer, then a marker to poll
        OCP_HIP(hipMemcpyAsync(ctx->pinned, hd->S.cg, sizeof(CgScalars), hipMemcpyDeviceToHost, ctx->stream));
        OCP_HIP(hipEventRecord(hd->ev_poll, ctx->stream));
        hd->polled_copy = true;
    });
}

extern "C" int pcg_poll(ocp_solve_handle *hd, ocp_solve_info *info) {
    if (!hd || !hd->S.ctx) return OCP_ERR_INVALID_ARG;
    ocp_ctx *ctx = hd->S.ctx;
    if (!hd->polled_copy) return 1;   // nothing advanced yet
    const hipError_t q = hipEventQuery(hd->ev_poll);
    if (q == hipErrorNotReady) return 2;
    if (q != hipSuccess) {
        ctx->last_error = std::string("hipEventQuery: ") + hipGetErrorString(q);
        return OCP_ERR_HIP;
    }
    CgScalars hs;
    std::memcpy(&hs, ctx->pinned, sizeof(hs));
    if (info) {
        info->iterations = hs.iter;
        info->status = hs.flag == 0 ? 1 : hs.flag == 1 ? OCP_OK : hs.flag == 2 ? OCP_ERR_BREAKDOWN : OCP_MAXIT;
        info->rel_res_l2 = hs.ff > 0 ? std::sqrt(hs.rr / hs.ff) : 0.0;
        info->rel_res_precond = hs.gamma0 > 0 ? std::sqrt(hs.gamma / hs.gamma0) : 0.0;
        info->true_rel_res = 0.0;
        info->setup_ms = hd->S.h ? hd->S.h->setup_ms : 0.0;
        info->solve_ms = 0.0;
    }
    return hs.flag == 0 ? 1 : 0;
}

extern "C" int pcg_end(ocp_solve_handle *hd, double *u, ocp_solve_info *info) {
    if (!hd || !hd->S.ctx) return OCP_ERR_INVALID_ARG;
    ocp_ctx *ctx = hd->S.ctx;
    int st = OCP_OK;
    int rc = run_step(ctx, [&] {
        if (!u) fail(OCP_ERR_INVALID_ARG, "u must not be NULL");
        st = solve_finish(hd->S, u, info);
    });
    (void)hipStreamSynchronize(ctx->stream);
    if (hd->ev_poll) (void)hipEventDestroy(hd->ev_poll);
    ctx->active_solve = false;
    delete hd;
    if (rc != OCP_OK) return rc;
    if (st == OCP_ERR_BREAKDOWN) ctx->last_error = "CG breakdown (p^T A p <= 0, r^T z <= 0 or non-finite)";
    return st;
}
