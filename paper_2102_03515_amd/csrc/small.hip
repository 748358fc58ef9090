// Persistent kernel for many small solves: one workgroup runs one whole
// PCG solve (Section 4's PCG with the V(1,1)-cycle preconditioner of Section
// 4.1), every phase a loop of the workgroup's 1024 threads over the rows
// separated by barriers, the scalars in LDS, the stop test on the device.
// A batch of m small problems is one launch of m workgroups, where the
// kernel-per-step form would need some thirty dispatches per iteration per
// problem, each only microseconds of work at these sizes.
//
// The arithmetic is that of pcg_solve and its V-cycle (the same smoother
// polynomial, coefficients, transfers and coarse solve); only the order of
// the additions inside the dot products differs (one workgroup instead of a
// grid reduction), so results agree with pcg_solve to rounding.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.h"
#include "system.h"

namespace ocp {

constexpr int kSmallThreads = 1024;
constexpr int kSmallMaxLevels = 12;
constexpr int32_t kSmallMaxRows = 1 << 18;   // problems up to this size run one per workgroup

template <typename T>
struct SmallLevel {
    int32_t n = 0, deg = 1;
    const int32_t *A_rp = nullptr, *A_col = nullptr;
    const T *A_val = nullptr;
    const int32_t *P_rp = nullptr, *P_col = nullptr;
    const T *P_val = nullptr;
    const int32_t *R_rp = nullptr, *R_col = nullptr;
    const T *R_val = nullptr;
    const T *d = nullptr, *inv = nullptr;
    T a = T(1), c1 = T(0), c2 = T(0);
    T *vb = nullptr, *vr = nullptr, *vx = nullptr, *vxp = nullptr, *vx1 = nullptr, *vx2 = nullptr;
};

template <typename T>
struct SmallDesc {
    int32_t n = 0, nv = 0, nlev = 0, maxit = 0, mode = 0;
    double rtol = 0.0;
    const int32_t *rp = nullptr, *col = nullptr;   // FP64 system CSR
    const double *val = nullptr;
    const double *f = nullptr, *dinv = nullptr;     // dinv: Jacobi (no hierarchy)
    double *x = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr;
    const int32_t *dof_of_vertex = nullptr;
    double *u = nullptr;
    SmallLevel<T> lev[kSmallMaxLevels];
};

struct SmallOut {
    int32_t iter, flag;
    double ff, rr, gamma, gamma0, res2;
};

namespace dev {
// Workgroup sum (fixed order), the total in every thread.
__device__ __forceinline__ double wg_sum(double v, double *red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kSmallThreads / 64; ++w) s += red[w];
    return s;
}

// sum_k val[k] xf(col[k]) over row i, in entry order; the column indices,
// values and gathers of 8 entries are issued before any is used, so a
// thread keeps 8 gathers in flight (one workgroup per problem has few waves
// to hide memory latency with).
template <typename VT, typename XF>
__device__ __forceinline__ VT csr_row(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                      const VT *__restrict__ val, int i, XF xf) {
    constexpr int U = 8;
    VT s = VT(0);
    int k = rp[i];
    const int e = rp[i + 1];
    for (; k + U <= e; k += U) {
        int c[U];
        VT v[U], g[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = col[k + u];
            v[u] = val[k + u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) g[u] = xf(c[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u] * g[u];
    }
    for (; k < e; ++k) s += val[k] * xf(col[k]);
    return s;
}
}  // namespace dev

// z = B r for one solve, by its workgroup: down sweep (pre-smoothing from
// zero fused with the residual, restriction), coarse solve, up sweep
// (prolongation and correction, post-smoothing).  The same passes as the
// multi-kernel V-cycle.
template <typename T>
__device__ void small_vcycle(const SmallDesc<T> &D, const double *__restrict__ r0, double *__restrict__ z0) {
    const int tid = threadIdx.x;
    const int L = D.nlev;
    for (int l = 0; l < L - 1; ++l) {
        const SmallLevel<T> &c = D.lev[l];
        const SmallLevel<T> &nx = D.lev[l + 1];
        auto bval = [&](int i) -> T { return l == 0 ? (T)r0[i] : c.vb[i]; };
        if (c.deg == 2) {
            // x2 = d (c1 b + c2 (b - A (a d b)))
            for (int i = tid; i < c.n; i += kSmallThreads) {
                const T s = dev::csr_row(c.A_rp, c.A_col, c.A_val, i, [&](int j) { return c.a * c.d[j] * bval(j); });
                const T bi = bval(i);
                c.vx2[i] = c.d[i] * (c.c1 * bi + c.c2 * (bi - s));
            }
            __syncthreads();
            for (int i = tid; i < c.n; i += kSmallThreads) {
                const T s = dev::csr_row(c.A_rp, c.A_col, c.A_val, i, [&](int j) { return c.vx2[j]; });
                c.vr[i] = bval(i) - s;
            }
        } else {
            for (int i = tid; i < c.n; i += kSmallThreads) {
                const T s = dev::csr_row(c.A_rp, c.A_col, c.A_val, i, [&](int j) { return c.a * c.d[j] * bval(j); });
                c.vr[i] = bval(i) - s;
            }
        }
        __syncthreads();
        for (int i = tid; i < nx.n; i += kSmallThreads)
            nx.vb[i] = dev::csr_row(c.R_rp, c.R_col, c.R_val, i, [&](int j) { return c.vr[j]; });
        __syncthreads();
    }
    // coarsest level
    {
        const SmallLevel<T> &c = D.lev[L - 1];
        auto bval = [&](int i) -> T { return L == 1 ? (T)r0[i] : c.vb[i]; };
        for (int i = tid; i < c.n; i += kSmallThreads) {
            T s;
            if (c.inv) {
                s = T(0);
                const T *ir = c.inv + (size_t)i * c.n;
                for (int j = 0; j < c.n; ++j) s += ir[j] * bval(j);
            } else {
                s = c.d[i] * bval(i);
            }
            if (L == 1)
                z0[i] = (double)s;
            else
                c.vx[i] = s;
        }
        __syncthreads();
    }
    for (int l = L - 2; l >= 0; --l) {
        const SmallLevel<T> &c = D.lev[l];
        const SmallLevel<T> &nx = D.lev[l + 1];
        auto bval = [&](int i) -> T { return l == 0 ? (T)r0[i] : c.vb[i]; };
        auto put = [&](int i, T v) {
            if (l == 0)
                z0[i] = (double)v;
            else
                c.vx[i] = v;
        };
        for (int i = tid; i < c.n; i += kSmallThreads) {
            const T s = dev::csr_row(c.P_rp, c.P_col, c.P_val, i, [&](int j) { return nx.vx[j]; });
            c.vxp[i] = (c.deg == 2 ? c.vx2[i] : c.a * c.d[i] * bval(i)) + s;
        }
        __syncthreads();
        if (c.deg == 2) {
            for (int i = tid; i < c.n; i += kSmallThreads) {
                const T s = dev::csr_row(c.A_rp, c.A_col, c.A_val, i, [&](int j) { return c.vxp[j]; });
                const T rr = bval(i) - s;
                c.vr[i] = rr;
                c.vx1[i] = c.vxp[i] + c.a * c.d[i] * rr;
            }
            __syncthreads();
            for (int i = tid; i < c.n; i += kSmallThreads) {
                const T s = dev::csr_row(c.A_rp, c.A_col, c.A_val, i, [&](int j) { return c.vx1[j]; });
                const T rr = bval(i) - s;
                put(i, c.vxp[i] + c.d[i] * (c.c1 * c.vr[i] + c.c2 * rr));
            }
        } else {
            for (int i = tid; i < c.n; i += kSmallThreads) {
                const T s = dev::csr_row(c.A_rp, c.A_col, c.A_val, i, [&](int j) { return c.vxp[j]; });
                put(i, c.vxp[i] + c.d[i] * (c.a * (bval(i) - s)));
            }
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void __launch_bounds__(kSmallThreads) k_small_pcg(const SmallDesc<T> *__restrict__ descs,
                                                             SmallOut *__restrict__ outs) {
    __shared__ double red[kSmallThreads / 64];
    const SmallDesc<T> &D = descs[blockIdx.x];
    const int tid = threadIdx.x, n = D.n;
    const bool amg = D.nlev > 0;
    auto precond = [&]() {
        if (amg) {
            small_vcycle<T>(D, D.r, D.z);
        } else {
            for (int i = tid; i < n; i += kSmallThreads) D.z[i] = D.dinv[i] * D.r[i];
            __syncthreads();
        }
        double rz = 0.0;
        for (int i = tid; i < n; i += kSmallThreads) rz += D.r[i] * D.z[i];
        return dev::wg_sum(rz, red);
    };
    // x = 0, r = f, p = 0
    double ff = 0.0;
    for (int i = tid; i < n; i += kSmallThreads) {
        const double fi = D.f[i];
        D.x[i] = 0.0;
        D.r[i] = fi;
        D.p[i] = 0.0;
        ff += fi * fi;
    }
    ff = dev::wg_sum(ff, red);
    double tol2 = D.mode == OCP_STOP_L2 ? D.rtol * D.rtol * ff : D.rtol * D.rtol;
    double rr = ff, gamma = 1.0, gamma0 = 0.0, beta = 0.0;
    int flag = (ff == 0.0) ? 1 : (isfinite(ff) ? 0 : 2);
    int iter = 0;
    // the first preconditioner application and p = z (the stop and
    // breakdown rules of pcg_solve)
    auto after_precond = [&](double rz) {
        if (iter == 0) gamma0 = rz;
        if (!(rz > 0.0) || !isfinite(rz)) {
            flag = (rz == 0.0 && rr == 0.0) ? 1 : 2;
            beta = 0.0;
            return;
        }
        beta = (iter == 0) ? 0.0 : rz / gamma;
        gamma = rz;
        if (D.mode == OCP_STOP_PRECOND) {
            if (iter == 0) tol2 = tol2 * rz;
            else if (rz <= tol2) flag = 1;
        }
    };
    if (flag == 0) {
        after_precond(precond());
        if (flag == 0) {
            for (int i = tid; i < n; i += kSmallThreads) D.p[i] = D.z[i] + beta * D.p[i];
            __syncthreads();
        }
    }
    while (flag == 0) {
        double pq = 0.0;
        for (int i = tid; i < n; i += kSmallThreads) {
            const double s = dev::csr_row(D.rp, D.col, D.val, i, [&](int j) { return D.p[j]; });
            D.q[i] = s;
            pq += D.p[i] * s;
        }
        pq = dev::wg_sum(pq, red);
        if (!(pq > 0.0) || !isfinite(pq)) {
            flag = 2;
            break;
        }
        const double alpha = gamma / pq;
        double r2 = 0.0;
        for (int i = tid; i < n; i += kSmallThreads) {
            D.x[i] += alpha * D.p[i];
            const double ri = D.r[i] - alpha * D.q[i];
            D.r[i] = ri;
            r2 += ri * ri;
        }
        r2 = dev::wg_sum(r2, red);
        rr = r2;
        iter += 1;
        if (D.mode == OCP_STOP_L2 && r2 <= tol2) {
            flag = 1;
            break;
        }
        if (!isfinite(r2)) {
            flag = 2;
            break;
        }
        if (iter >= D.maxit) {
            flag = 3;
            break;
        }
        after_precond(precond());
        if (flag != 0) break;
        for (int i = tid; i < n; i += kSmallThreads) D.p[i] = D.z[i] + beta * D.p[i];
        __syncthreads();
    }
    // true residual in double, then u on all vertices
    double res2 = 0.0;
    for (int i = tid; i < n; i += kSmallThreads) {
        const double s = dev::csr_row(D.rp, D.col, D.val, i, [&](int j) { return D.x[j]; });
        const double ri = D.f[i] - s;
        res2 += ri * ri;
    }
    res2 = dev::wg_sum(res2, red);
    for (int v = tid; v < D.nv; v += kSmallThreads) {
        const int d = D.dof_of_vertex[v];
        D.u[v] = d >= 0 ? D.x[d] : 0.0;
    }
    if (tid == 0) outs[blockIdx.x] = SmallOut{iter, flag, ff, rr, gamma, gamma0, res2};
}

// ------------------------------------------------------------------- host
bool small_eligible(const ocp_system *sys, const ocp_hierarchy *h) {
    if (sys->n > kSmallMaxRows) return false;
    if (h && (int)h->levels.size() > kSmallMaxLevels) return false;
    if (h && h->params.method != OCP_AMG_AGGREGATION) return false;   // the graph path runs the other methods
    return true;
}

namespace {
template <typename T>
struct LvArrays;
template <>
struct LvArrays<double> {
    static const double *A(const Level &L) { return L.A_val; }
    static const double *P(const Level &L) { return L.P_val.get(); }
    static const double *R(const Level &L) { return L.R_val.get(); }
    static const double *d(const Level &L) { return L.dinv.get(); }
    static const double *inv(const Level &L) { return L.dense_inv.get(); }
};
template <>
struct LvArrays<float> {
    static const float *A(const Level &L) { return L.A_val32.get(); }
    static const float *P(const Level &L) { return L.P_val32.get(); }
    static const float *R(const Level &L) { return L.R_val32.get(); }
    static const float *d(const Level &L) { return L.dinv32.get(); }
    static const float *inv(const Level &L) { return L.dense_inv32.get(); }
};
}  // namespace

// Runs the given solves (all of value type T, or Jacobi when T is double
// and the hierarchy is null) as one launch; returns per-solve statuses.
template <typename T>
static void run_small(ocp_ctx *ctx, const std::vector<int> &idx, const ocp_system *const *systems,
                      const ocp_hierarchy *const *hs, const double *const *fs, double *const *us, double rtol,
                      int32_t maxit, int mode, ocp_solve_info *infos, std::vector<int> &st) {
    const int m = (int)idx.size();
    if (m == 0) return;
    // arena: every solve's CG vectors and V-cycle work vectors
    std::vector<SmallDesc<T>> D((size_t)m);
    size_t total = 0;
    for (int t = 0; t < m; ++t) {
        const ocp_system *s = systems[idx[t]];
        const ocp_hierarchy *h = hs ? hs[idx[t]] : nullptr;
        total += 5 * align256(sizeof(double) * s->n);
        if (h)
            for (const auto &L : h->levels) total += 6 * align256(sizeof(T) * L->n);
    }
    DevBuf<char> arena(ctx, total);
    size_t cur = 0;
    auto take = [&](size_t bytes) {
        char *p = arena.get() + cur;
        cur += align256(bytes);
        return p;
    };
    for (int t = 0; t < m; ++t) {
        const int i = idx[t];
        ocp_system *s = const_cast<ocp_system *>(systems[i]);
        const ocp_hierarchy *h = hs ? hs[i] : nullptr;
        SmallDesc<T> &d = D[t];
        d.n = s->n;
        d.nv = s->nv;
        d.maxit = maxit;
        d.mode = mode;
        d.rtol = rtol;
        d.rp = s->row_ptr.get();
        d.col = s->col.get();
        d.val = s->val.get();
        d.f = (fs && fs[i]) ? fs[i] : s->f.get();
        d.dinv = h ? nullptr : system_dinv(ctx, s);
        d.dof_of_vertex = s->dof_of_vertex.get();
        d.u = us[i];
        d.x = reinterpret_cast<double *>(take(sizeof(double) * s->n));
        d.r = reinterpret_cast<double *>(take(sizeof(double) * s->n));
        d.p = reinterpret_cast<double *>(take(sizeof(double) * s->n));
        d.q = reinterpret_cast<double *>(take(sizeof(double) * s->n));
        d.z = reinterpret_cast<double *>(take(sizeof(double) * s->n));
        d.nlev = h ? (int)h->levels.size() : 0;
        for (int l = 0; l < d.nlev; ++l) {
            const Level &L = *h->levels[l];
            SmallLevel<T> &v = d.lev[l];
            v.n = L.n;
            v.deg = L.deg;
            v.A_rp = L.A_rp;
            v.A_col = L.A_col;
            v.A_val = LvArrays<T>::A(L);
            v.P_rp = L.P_rp.get();
            v.P_col = L.P_col.get();
            v.P_val = LvArrays<T>::P(L);
            v.R_rp = L.R_rp.get();
            v.R_col = L.R_col.get();
            v.R_val = LvArrays<T>::R(L);
            v.d = LvArrays<T>::d(L);
            v.inv = LvArrays<T>::inv(L);
            v.a = (T)L.cheb_a;
            v.c1 = (T)L.cheb_c1;
            v.c2 = (T)L.cheb_c2;
            v.vb = reinterpret_cast<T *>(take(sizeof(T) * L.n));
            v.vr = reinterpret_cast<T *>(take(sizeof(T) * L.n));
            v.vx = reinterpret_cast<T *>(take(sizeof(T) * L.n));
            v.vxp = reinterpret_cast<T *>(take(sizeof(T) * L.n));
            v.vx1 = reinterpret_cast<T *>(take(sizeof(T) * L.n));
            v.vx2 = reinterpret_cast<T *>(take(sizeof(T) * L.n));
        }
    }
    DevBuf<SmallDesc<T>> ddesc(ctx, (size_t)m);
    DevBuf<SmallOut> dout(ctx, (size_t)m);
    OCP_HIP(hipMemcpyAsync(ddesc.get(), D.data(), sizeof(SmallDesc<T>) * m, hipMemcpyHostToDevice, ctx->stream));
    k_small_pcg<T><<<m, kSmallThreads, 0, ctx->stream>>>(ddesc.get(), dout.get());
    OCP_LAUNCH_CHECK();
    std::vector<SmallOut> out((size_t)m);
    OCP_HIP(hipMemcpyAsync(out.data(), dout.get(), sizeof(SmallOut) * m, hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    for (int t = 0; t < m; ++t) {
        const SmallOut &o = out[t];
        const int s = o.flag == 2 ? OCP_ERR_BREAKDOWN : (o.flag == 3 || o.flag == 0) ? OCP_MAXIT : OCP_OK;
        st[idx[t]] = s;
        if (infos) {
            ocp_solve_info &in = infos[idx[t]];
            in.iterations = o.iter;
            in.status = s;
            in.rel_res_l2 = o.ff > 0 ? std::sqrt(o.rr / o.ff) : 0.0;
            in.rel_res_precond = o.gamma0 > 0 ? std::sqrt(o.gamma / o.gamma0) : 0.0;
            in.true_rel_res = o.ff > 0 ? std::sqrt(o.res2 / o.ff) : 0.0;
            in.setup_ms = (hs && hs[idx[t]]) ? hs[idx[t]]->setup_ms : 0.0;
            in.solve_ms = 0.0;
        }
    }
}

// Small solves of a batch, one workgroup each: mixed-precision hierarchies in
// one launch, FP64 hierarchies and Jacobi in another.
void small_batch(ocp_ctx *ctx, const std::vector<int> &idx, const ocp_system *const *systems,
                 const ocp_hierarchy *const *hs, const double *const *fs, double *const *us, double rtol,
                 int32_t maxit, int mode, ocp_solve_info *infos, std::vector<int> &st) {
    std::vector<int> i32, i64;
    for (int i : idx) {
        const ocp_hierarchy *h = hs ? hs[i] : nullptr;
        (h && h->params.precision == OCP_PREC_MIXED ? i32 : i64).push_back(i);
    }
    hipEvent_t e0, e1;
    OCP_HIP(hipEventCreate(&e0));
    OCP_HIP(hipEventCreate(&e1));
    OCP_HIP(hipEventRecord(e0, ctx->stream));
    run_small<float>(ctx, i32, systems, hs, fs, us, rtol, maxit, mode, infos, st);
    run_small<double>(ctx, i64, systems, hs, fs, us, rtol, maxit, mode, infos, st);
    OCP_HIP(hipEventRecord(e1, ctx->stream));
    OCP_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (infos)
        for (int i : idx) infos[i].solve_ms = ms;
}

}  // namespace ocp
