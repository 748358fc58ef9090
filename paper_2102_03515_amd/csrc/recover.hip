// Control and adjoint from the computed state, and error norms of the state
// against the closed-form solution, on the device.
//
// Section 1: once the state u_rho solves the reduced equation (5), the
// gradient equation (4) gives the adjoint p_rho = -rho u_rho, and the state
// equation (2) together with (5) gives the control
// z_rho = -Lap u_rho = (ubar - u_rho) / rho.  For a P1 state u_h these hold
// pointwise at the vertices: p_h = -rho u_h and z_h = (ubar(x_v) - u_h(x_v))/rho
// (the nodal interpolant of z; for a P1 target its vertex values).
//
// Section 4.1 measures ||u_rho - u_rho,h||_L2 (Table 1), the H1 seminorm
// ||grad(u_rho - u_rho,h)||_L2 (Table 2) and ||ubar - u_rho,h||_L2 (Table 3,
// squared there).  For targets that are sums of Dirichlet eigenfunctions,
// ubar = sum_m a_m prod_d sin(k_md pi x_d), eq. (5) is solved mode by mode:
// u_rho = sum_m a_m / (1 + rho pi^2 |k_m|^2) prod_d sin(k_md pi x_d).  The
// integrals are taken element by element with a collapsed (Duffy) product of
// 5-point Gauss-Legendre rules: exact for polynomials of degree 7 on a
// tetrahedron, 125 points, nodes found by Newton's method on the Legendre
// recurrence when the call starts.
#include <cmath>
#include <vector>

#include "kernels.h"
#include "system.h"

namespace ocp {

namespace {

constexpr int kGL = 5;                 // Gauss-Legendre points per direction
constexpr int kQuad = kGL * kGL * kGL;  // points of the collapsed rule
constexpr int kNormBlock = 256;
constexpr int kNormMaxBlocks = 8192;

struct RecMode {
    int32_t k[3];
    int32_t pad;
    double amp;     // target amplitude a_m
    double coef;    // a_m / (1 + rho pi^2 |k_m|^2): amplitude of the exact state
};

struct RecTarget {
    int32_t kind;
    int32_t n_modes;
    const RecMode *modes;
    double offset;
    double lo[3], hi[3];
    const double *nodal;
};

// ubar at a point (sine modes, box); NODAL targets are handled by the callers
__device__ double target_at(const RecTarget &t, const double x[3]) {
    if (t.kind == OCP_TARGET_BOX) {
        bool in = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) in = in && x[d] > t.lo[d] && x[d] < t.hi[d];
        return in ? 1.0 : 0.0;
    }
    double s = t.offset;
    for (int m = 0; m < t.n_modes; ++m) {
        const RecMode md = t.modes[m];
        s += md.amp * sinpi(md.k[0] * x[0]) * sinpi(md.k[1] * x[1]) * sinpi(md.k[2] * x[2]);
    }
    return s;
}

// value and gradient of the closed-form state of a homogeneous sine target
__device__ void exact_state(const RecTarget &t, const double x[3], double &u, double g[3]) {
    u = 0.0;
    g[0] = g[1] = g[2] = 0.0;
    for (int m = 0; m < t.n_modes; ++m) {
        const RecMode md = t.modes[m];
        double s[3], c[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) sincospi(md.k[d] * x[d], &s[d], &c[d]);
        const double a = md.coef;
        u += a * s[0] * s[1] * s[2];
        g[0] += a * M_PI * md.k[0] * c[0] * s[1] * s[2];
        g[1] += a * M_PI * md.k[1] * s[0] * c[1] * s[2];
        g[2] += a * M_PI * md.k[2] * s[0] * s[1] * c[2];
    }
}

__global__ void k_recover(int32_t nv, double rho, const double *__restrict__ xyz, const double *__restrict__ u,
                          RecTarget t, double *__restrict__ p, double *__restrict__ z) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    const double uv = u[v];
    if (p) p[v] = -rho * uv;
    if (z) {
        double ub;
        if (t.kind == OCP_TARGET_NODAL) {
            ub = t.nodal[v];
        } else {
            const double x[3] = {xyz[3 * (int64_t)v], xyz[3 * (int64_t)v + 1], xyz[3 * (int64_t)v + 2]};
            ub = target_at(t, x);
        }
        z[v] = (ub - uv) / rho;
    }
}

// Per block: sums over its tets of |det B| sum_q w_q (.)^2 for the three
// errors; one thread per tet, the quadrature points (barycentric lambda_1..3
// and weight, the same for every thread) read as uniform loads.
__global__ void __launch_bounds__(kNormBlock) k_error_norms(int64_t nt, const int4 *__restrict__ tets,
                                                             const double *__restrict__ xyz,
                                                             const double *__restrict__ u, RecTarget t,
                                                             int exact, const double4 *__restrict__ quad,
                                                             double *__restrict__ part) {
    double e2 = 0.0, g2 = 0.0, t2 = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kNormBlock + threadIdx.x; e < nt; e += (int64_t)gridDim.x * kNormBlock) {
        const int4 tv = tets[e];
        const int vid[4] = {tv.x, tv.y, tv.z, tv.w};
        double P[4][3], uh[4], ub[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
#pragma unroll
            for (int d = 0; d < 3; ++d) P[a][d] = xyz[3 * (int64_t)vid[a] + d];
            uh[a] = u[vid[a]];
            if (t.kind == OCP_TARGET_NODAL) ub[a] = t.nodal[vid[a]];
        }
        // B = [p1 - p0, p2 - p0, p3 - p0] (columns); grad lambda_a = rows of B^-1
        double B[3][3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int c = 0; c < 3; ++c) B[d][c] = P[c + 1][d] - P[0][d];
        const double C00 = B[1][1] * B[2][2] - B[1][2] * B[2][1];
        const double C01 = B[1][2] * B[2][0] - B[1][0] * B[2][2];
        const double C02 = B[1][0] * B[2][1] - B[1][1] * B[2][0];
        const double det = B[0][0] * C00 + B[0][1] * C01 + B[0][2] * C02;
        const double id = 1.0 / det;
        // rows of B^-1 (the adjugate's rows over det)
        double Gi[3][3];
        Gi[0][0] = C00 * id;
        Gi[0][1] = (B[0][2] * B[2][1] - B[0][1] * B[2][2]) * id;
        Gi[0][2] = (B[0][1] * B[1][2] - B[0][2] * B[1][1]) * id;
        Gi[1][0] = C01 * id;
        Gi[1][1] = (B[0][0] * B[2][2] - B[0][2] * B[2][0]) * id;
        Gi[1][2] = (B[0][2] * B[1][0] - B[0][0] * B[1][2]) * id;
        Gi[2][0] = C02 * id;
        Gi[2][1] = (B[0][1] * B[2][0] - B[0][0] * B[2][1]) * id;
        Gi[2][2] = (B[0][0] * B[1][1] - B[0][1] * B[1][0]) * id;
        // grad u_h = sum_a u_a grad lambda_a, grad lambda_0 = -(sum of the others)
        double gh[3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
            gh[d] = (uh[1] - uh[0]) * Gi[0][d] + (uh[2] - uh[0]) * Gi[1][d] + (uh[3] - uh[0]) * Gi[2][d];
        const double vol = fabs(det);
        double se = 0.0, sg = 0.0, st = 0.0;
        for (int q = 0; q < kQuad; ++q) {
            const double4 Q = quad[q];
            const double l1 = Q.x, l2 = Q.y, l3 = Q.z, l0 = 1.0 - l1 - l2 - l3;
            double x[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) x[d] = l0 * P[0][d] + l1 * P[1][d] + l2 * P[2][d] + l3 * P[3][d];
            const double uq = l0 * uh[0] + l1 * uh[1] + l2 * uh[2] + l3 * uh[3];
            const double tq = t.kind == OCP_TARGET_NODAL ? l0 * ub[0] + l1 * ub[1] + l2 * ub[2] + l3 * ub[3]
                                                         : target_at(t, x);
            st += Q.w * (tq - uq) * (tq - uq);
            if (exact) {
                double ue, ge[3];
                exact_state(t, x, ue, ge);
                se += Q.w * (ue - uq) * (ue - uq);
                sg += Q.w * ((ge[0] - gh[0]) * (ge[0] - gh[0]) + (ge[1] - gh[1]) * (ge[1] - gh[1]) +
                             (ge[2] - gh[2]) * (ge[2] - gh[2]));
            }
        }
        e2 += vol * se;
        g2 += vol * sg;
        t2 += vol * st;
    }
    // block sums (fixed order: wavefront shuffles, then the 4 wavefronts)
    double v3[3] = {e2, g2, t2};
    __shared__ double ws[3][kNormBlock / 64];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double s = v3[c];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if ((threadIdx.x & 63) == 0) ws[c][threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int w = 0; w < kNormBlock / 64; ++w) s += ws[threadIdx.x][w];
        part[(int64_t)threadIdx.x * kNormMaxBlocks + blockIdx.x] = s;
    }
}

// one block: the three sums of the block partials, in block order
__global__ void __launch_bounds__(64) k_error_norms_fin(unsigned nb, const double *__restrict__ part,
                                                        double *__restrict__ out) {
    if (threadIdx.x >= 3) return;
    double s = 0.0;
    for (unsigned b = 0; b < nb; ++b) s += part[(int64_t)threadIdx.x * kNormMaxBlocks + b];
    out[threadIdx.x] = s;
}

// Residual-based error indicator of the reaction-diffusion equation (5) for
// a P1 state u_h, per tetrahedron tau (the robust weighting of Verfuerth's
// estimators for singularly perturbed reaction-diffusion problems):
//   eta_tau^2 = a_tau^2 ||ubar - u_h||^2_tau
//             + 1/2 sum_{interior faces F of tau} rho^{-1/2} a_F ||[rho grad u_h . n_F]||^2_F,
//   a_S = min(1, h_S / sqrt(rho)),  h_S the longest edge of S.
// The element residual ubar + rho Lap u_h - u_h is ubar - u_h for P1; its
// square is integrated by the 4-point rule of the load vector.  The normal
// flux jump is constant on a face.  A face's neighbour is the other
// tetrahedron in the incidence list of one of its vertices that holds the
// other two; a face without one lies on the boundary and adds nothing.
__device__ void tet_grad(const double P[4][3], const double uh[4], double g[3], double &vol, double &hmax) {
    double B[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < 3; ++c) B[d][c] = P[c + 1][d] - P[0][d];
    const double C00 = B[1][1] * B[2][2] - B[1][2] * B[2][1];
    const double C01 = B[1][2] * B[2][0] - B[1][0] * B[2][2];
    const double C02 = B[1][0] * B[2][1] - B[1][1] * B[2][0];
    const double det = B[0][0] * C00 + B[0][1] * C01 + B[0][2] * C02;
    const double id = 1.0 / det;
    double Gi[3][3];
    Gi[0][0] = C00 * id;
    Gi[0][1] = (B[0][2] * B[2][1] - B[0][1] * B[2][2]) * id;
    Gi[0][2] = (B[0][1] * B[1][2] - B[0][2] * B[1][1]) * id;
    Gi[1][0] = C01 * id;
    Gi[1][1] = (B[0][0] * B[2][2] - B[0][2] * B[2][0]) * id;
    Gi[1][2] = (B[0][2] * B[1][0] - B[0][0] * B[1][2]) * id;
    Gi[2][0] = C02 * id;
    Gi[2][1] = (B[0][1] * B[2][0] - B[0][0] * B[2][1]) * id;
    Gi[2][2] = (B[0][0] * B[1][1] - B[0][1] * B[1][0]) * id;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        g[d] = (uh[1] - uh[0]) * Gi[0][d] + (uh[2] - uh[0]) * Gi[1][d] + (uh[3] - uh[0]) * Gi[2][d];
    vol = fabs(det) / 6.0;
    hmax = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a + 1; b < 4; ++b) {
            const double dx = P[a][0] - P[b][0], dy = P[a][1] - P[b][1], dz = P[a][2] - P[b][2];
            hmax = fmax(hmax, sqrt(dx * dx + dy * dy + dz * dz));
        }
}

__global__ void __launch_bounds__(256) k_error_indicator(int64_t nt, const int4 *__restrict__ tets,
                                                          const double *__restrict__ xyz,
                                                          const double *__restrict__ u, RecTarget t, double rho,
                                                          const int32_t *__restrict__ inc_ptr,
                                                          const int32_t *__restrict__ inc, double *__restrict__ eta2) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= nt) return;
    const int4 tv = tets[e];
    const int vid[4] = {tv.x, tv.y, tv.z, tv.w};
    double P[4][3], uh[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int d = 0; d < 3; ++d) P[a][d] = xyz[3 * (int64_t)vid[a] + d];
        uh[a] = u[vid[a]];
    }
    double g[3], vol, h;
    tet_grad(P, uh, g, vol, h);
    const double srho = sqrt(rho);
    // element term by the 4-point degree-2 rule (barycentric (a, b, b, b) and permutations)
    const double qa = 0.5854101966249685;   // (5 + 3 sqrt5) / 20
    const double qb = 0.1381966011250105;   // (5 - sqrt5) / 20
    double r2 = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        double x[3], uq = 0.0, tq = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double s = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a) s += (a == q ? qa : qb) * P[a][d];
            x[d] = s;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) uq += (a == q ? qa : qb) * uh[a];
        if (t.kind == OCP_TARGET_NODAL) {
#pragma unroll
            for (int a = 0; a < 4; ++a) tq += (a == q ? qa : qb) * t.nodal[vid[a]];
        } else {
            tq = target_at(t, x);
        }
        r2 += (tq - uq) * (tq - uq);
    }
    r2 *= vol / 4.0;
    const double at = fmin(1.0, h / srho);
    double eta = at * at * r2;
    // faces
#pragma unroll 1
    for (int a = 0; a < 4; ++a) {
        int f[3], p = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (b != a) f[p++] = vid[b];
        int64_t nb = -1;
        for (int q = inc_ptr[f[0]]; q < inc_ptr[f[0] + 1]; ++q) {
            const int64_t e2 = inc[q] >> 2;
            if (e2 == e) continue;
            const int4 w = tets[e2];
            const bool h1 = w.x == f[1] || w.y == f[1] || w.z == f[1] || w.w == f[1];
            const bool h2 = w.x == f[2] || w.y == f[2] || w.z == f[2] || w.w == f[2];
            if (h1 && h2) {
                nb = e2;
                break;
            }
        }
        if (nb < 0) continue;   // boundary face
        const int4 w = tets[nb];
        const int wid[4] = {w.x, w.y, w.z, w.w};
        double Q[4][3], uw[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
#pragma unroll
            for (int d = 0; d < 3; ++d) Q[b][d] = xyz[3 * (int64_t)wid[b] + d];
            uw[b] = u[wid[b]];
        }
        double g2[3], vol2, h2;
        tet_grad(Q, uw, g2, vol2, h2);
        // face normal, area and diameter
        double e1[3], e2v[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            e1[d] = xyz[3 * (int64_t)f[1] + d] - xyz[3 * (int64_t)f[0] + d];
            e2v[d] = xyz[3 * (int64_t)f[2] + d] - xyz[3 * (int64_t)f[0] + d];
        }
        const double nx = e1[1] * e2v[2] - e1[2] * e2v[1];
        const double ny = e1[2] * e2v[0] - e1[0] * e2v[2];
        const double nz = e1[0] * e2v[1] - e1[1] * e2v[0];
        const double nn = sqrt(nx * nx + ny * ny + nz * nz);
        const double area = 0.5 * nn;
        const double e3[3] = {e2v[0] - e1[0], e2v[1] - e1[1], e2v[2] - e1[2]};
        const double hf = fmax(sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]),
                               fmax(sqrt(e2v[0] * e2v[0] + e2v[1] * e2v[1] + e2v[2] * e2v[2]),
                                    sqrt(e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2])));
        const double jump = rho * ((g[0] - g2[0]) * nx + (g[1] - g2[1]) * ny + (g[2] - g2[2]) * nz) / nn;
        const double af = fmin(1.0, hf / srho);
        eta += 0.5 / srho * af * area * jump * jump;
    }
    eta2[e] = eta;
}

// n-point Gauss-Legendre nodes and weights on [0, 1] (Newton's method on the
// three-term recurrence of the Legendre polynomials)
void gauss_legendre01(int n, double *x, double *w) {
    for (int i = 0; i < n; ++i) {
        double t = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (t * p1 - p0) / (t * t - 1.0);
        x[i] = 0.5 * (1.0 + t);
        w[i] = 1.0 / ((1.0 - t * t) * dp * dp);   // 2 / ((1 - t^2) P'(t)^2), halved for [0, 1]
    }
}

// The collapsed rule: (s1, s2, s3) in [0,1]^3 maps to lambda_1 = s1,
// lambda_2 = (1 - s1) s2, lambda_3 = (1 - s1)(1 - s2) s3 with Jacobian
// (1 - s1)^2 (1 - s2); the weights sum to 1/6, the reference volume, so a
// tetrahedron's integral is |det B| sum_q w_q f(lambda_q).
std::vector<double4> collapsed_rule() {
    double x[kGL], w[kGL];
    gauss_legendre01(kGL, x, w);
    std::vector<double4> q;
    q.reserve(kQuad);
    for (int i = 0; i < kGL; ++i)
        for (int j = 0; j < kGL; ++j)
            for (int k = 0; k < kGL; ++k) {
                const double s1 = x[i], s2 = x[j], s3 = x[k];
                q.push_back(make_double4(s1, (1.0 - s1) * s2, (1.0 - s1) * (1.0 - s2) * s3,
                                         w[i] * w[j] * w[k] * (1.0 - s1) * (1.0 - s1) * (1.0 - s2)));
            }
    return q;
}

struct RecUpload {
    DevBuf<RecMode> modes;
    RecTarget dev{};
    bool homogeneous_sine = false;   // closed-form state available
};

void upload_rec_target(ocp_ctx *ctx, const ocp_target *t, int32_t nv, double rho, RecUpload &up) {
    if (!t) fail(OCP_ERR_INVALID_ARG, "target must not be NULL");
    up.dev.kind = t->kind;
    up.dev.offset = t->offset;
    for (int d = 0; d < 3; ++d) {
        up.dev.lo[d] = t->lo[d];
        up.dev.hi[d] = t->hi[d];
    }
    up.dev.nodal = t->nodal;
    if (t->kind == OCP_TARGET_SINE_MODES) {
        if (t->n_modes < 1 || t->n_modes > 4096 || !t->k || !t->amp)
            fail(OCP_ERR_INVALID_ARG, "sine target needs 1..4096 modes with wave numbers and amplitudes");
        std::vector<RecMode> md((size_t)t->n_modes);
        for (int m = 0; m < t->n_modes; ++m) {
            double k2 = 0.0;
            for (int d = 0; d < 3; ++d) {
                const int k = t->k[3 * m + d];
                if (k < 1 || k > 1024) fail(OCP_ERR_INVALID_ARG, "wave numbers must lie in 1..1024");
                md[m].k[d] = k;
                k2 += (double)k * k;
            }
            if (!std::isfinite(t->amp[m])) fail(OCP_ERR_INVALID_ARG, "amplitudes must be finite");
            md[m].pad = 0;
            md[m].amp = t->amp[m];
            md[m].coef = t->amp[m] / (1.0 + rho * M_PI * M_PI * k2);
        }
        up.modes.reset(ctx, md.size());
        OCP_HIP(hipMemcpyAsync(up.modes.get(), md.data(), sizeof(RecMode) * md.size(), hipMemcpyHostToDevice,
                               ctx->stream));
        sync(ctx);   // the staging vector is released on return
        up.dev.n_modes = t->n_modes;
        up.dev.modes = up.modes.get();
        up.homogeneous_sine = t->offset == 0.0;
    } else if (t->kind == OCP_TARGET_BOX) {
        up.dev.n_modes = 0;
    } else if (t->kind == OCP_TARGET_NODAL) {
        if (!t->nodal) fail(OCP_ERR_INVALID_ARG, "nodal target needs device values");
        up.dev.n_modes = 0;
    } else {
        fail(OCP_ERR_INVALID_ARG, "unknown target kind");
    }
    (void)nv;
}

}  // namespace

}  // namespace ocp

using namespace ocp;

extern "C" int fe_recover(ocp_ctx *ctx, const ocp_system *sys, const ocp_target *target, const double *u, double *p,
                          double *z) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    return run_guarded(ctx, [&] {
        if (!sys || !u) fail(OCP_ERR_INVALID_ARG, "system and u must not be NULL");
        if (!p && !z) return;
        RecUpload up;
        if (z) upload_rec_target(ctx, target, sys->nv, sys->rho, up);
        k_recover<<<grid_for(sys->nv, 256), 256, 0, ctx->stream>>>(sys->nv, sys->rho, sys->mesh.xyz, u, up.dev, p, z);
        OCP_LAUNCH_CHECK();
        sync(ctx);   // the uploaded modes are released on return
    });
}

extern "C" int fe_error_indicator(ocp_ctx *ctx, const ocp_system *sys, const ocp_target *target, const double *u,
                                  double *eta2) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    return run_guarded(ctx, [&] {
        if (!sys || !u || !eta2) fail(OCP_ERR_INVALID_ARG, "system, u and eta2 must not be NULL");
        RecUpload up;
        upload_rec_target(ctx, target, sys->nv, sys->rho, up);
        k_error_indicator<<<grid_for(sys->nt, 256), 256, 0, ctx->stream>>>(
            sys->nt, reinterpret_cast<const int4 *>(sys->mesh.tets), sys->mesh.xyz, u, up.dev, sys->rho,
            sys->inc_ptr.get(), sys->inc.get(), eta2);
        OCP_LAUNCH_CHECK();
        sync(ctx);   // the uploaded modes are released on return
    });
}

extern "C" int fe_error_norms(ocp_ctx *ctx, const ocp_system *sys, const ocp_target *target, const double *u,
                              double *out) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    return run_guarded(ctx, [&] {
        if (!sys || !u || !out) fail(OCP_ERR_INVALID_ARG, "system, u and out must not be NULL");
        RecUpload up;
        upload_rec_target(ctx, target, sys->nv, sys->rho, up);
        const std::vector<double4> rule = collapsed_rule();
        DevBuf<double4> quad(ctx, rule.size());
        OCP_HIP(hipMemcpyAsync(quad.get(), rule.data(), sizeof(double4) * rule.size(), hipMemcpyHostToDevice,
                               ctx->stream));
        DevBuf<double> part(ctx, (size_t)3 * kNormMaxBlocks), res(ctx, 3);
        int64_t nb = (sys->nt + kNormBlock - 1) / kNormBlock;
        if (nb > kNormMaxBlocks) nb = kNormMaxBlocks;
        if (nb < 1) nb = 1;
        k_error_norms<<<(unsigned)nb, kNormBlock, 0, ctx->stream>>>(
            sys->nt, reinterpret_cast<const int4 *>(sys->mesh.tets), sys->mesh.xyz, u, up.dev,
            up.homogeneous_sine ? 1 : 0, quad.get(), part.get());
        k_error_norms_fin<<<1, 64, 0, ctx->stream>>>((unsigned)nb, part.get(), res.get());
        OCP_LAUNCH_CHECK();
        double h[3] = {0.0, 0.0, 0.0};
        read_back(ctx, h, res.get(), sizeof(h));
        const double nan = std::nan("");
        out[0] = up.homogeneous_sine ? std::sqrt(h[0]) : nan;
        out[1] = up.homogeneous_sine ? std::sqrt(h[1]) : nan;
        out[2] = std::sqrt(h[2]);
    });
}
