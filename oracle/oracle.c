/*
 * CPU oracle for the P1 finite element system of the reduced optimality
 * equation  -rho*Lap(u) + u = ubar  in Omega, u = 0 on Gamma  (eq. (5)).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product never does.  It shares
 * no code, header or table with the GPU library.
 *
 * What it computes (Section 2, system (linsys) and the matrix entries that
 * follow it):
 *     A = rho*K + M,   K_ij = int grad(phi_j).grad(phi_i),
 *     M_ij = int phi_j phi_i,   f_i = int ubar phi_i,
 * over the nodal P1 (Courant) basis of the interior vertices (homogeneous
 * Dirichlet: boundary vertices carry no unknown, Section 2).  Everything is
 * plain double precision: element by element, row by row.
 *
 * The load integral uses the 4-point degree-2 rule with barycentric points
 * (a,b,b,b) and permutations, a = (5+3 sqrt5)/20, b = (5-sqrt5)/20, weights
 * |tau|/4 each (the paper does not state its quadrature).
 *
 * The solver is Jacobi-preconditioned CG from x0 = 0 (Section 4 uses PCG;
 * with an SPD matrix every preconditioner reaches the same discrete solution).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- targets */
/* kind 0: sine modes   ubar = offset + sum_m amp[m] prod_d sin(k[m][d] pi x_d)
 * kind 1: open box     ubar = 1 on (lo, hi), 0 elsewhere
 * kind 2: nodal        ubar = sum_v nodal[v] phi_v (P1 interpolant)           */
typedef struct {
    int kind;
    int n_modes;
    const int32_t *k;      /* [n_modes][3] */
    const double *amp;     /* [n_modes] */
    double offset;
    double lo[3], hi[3];
    const double *nodal;   /* [n_vertices] */
} orc_target;

static double target_at(const orc_target *t, const double x[3])
{
    if (t->kind == 0) {
        double s = t->offset;
        for (int m = 0; m < t->n_modes; ++m) {
            double p = t->amp[m];
            for (int d = 0; d < 3; ++d)
                p *= sin((double)t->k[3 * m + d] * M_PI * x[d]);
            s += p;
        }
        return s;
    }
    if (t->kind == 1) {
        for (int d = 0; d < 3; ++d)
            if (!(x[d] > t->lo[d] && x[d] < t->hi[d])) return 0.0;
        return 1.0;
    }
    return 0.0; /* nodal targets are handled by the caller */
}

/* ------------------------------------------------------------ one element */
/* Element data of tetrahedron (p0,p1,p2,p3):
 *   vol        = |det B| / 6 with B = [p1-p0, p2-p0, p3-p0] (columns)
 *   grad[a]    = gradient of barycentric coordinate lambda_a
 *   Ke[a][b]   = vol * grad[a].grad[b]
 *   Me[a][b]   = vol/20 * (1 + delta_ab)
 *   fe[a]      = sum_q vol/4 * ubar(x_q) * lambda_a(x_q)                     */
static int element(const double *xyz, const int32_t *tv, const orc_target *t,
                   double Ke[4][4], double Me[4][4], double fe[4], double *vol_out)
{
    const double *p[4];
    for (int a = 0; a < 4; ++a) p[a] = xyz + 3 * (int64_t)tv[a];
    double B[3][3]; /* B[r][c] = (p_{c+1} - p_0)_r */
    for (int c = 0; c < 3; ++c)
        for (int r = 0; r < 3; ++r) B[r][c] = p[c + 1][r] - p[0][r];
    double det = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1])
               - B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0])
               + B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
    if (det == 0.0) return -1;
    /* inverse of B: lambda_{c+1}(x) = (B^{-1} (x - p0))_c, so grad lambda_{c+1}
     * is row c of B^{-1}. */
    double Bi[3][3];
    Bi[0][0] = (B[1][1] * B[2][2] - B[1][2] * B[2][1]) / det;
    Bi[0][1] = (B[0][2] * B[2][1] - B[0][1] * B[2][2]) / det;
    Bi[0][2] = (B[0][1] * B[1][2] - B[0][2] * B[1][1]) / det;
    Bi[1][0] = (B[1][2] * B[2][0] - B[1][0] * B[2][2]) / det;
    Bi[1][1] = (B[0][0] * B[2][2] - B[0][2] * B[2][0]) / det;
    Bi[1][2] = (B[0][2] * B[1][0] - B[0][0] * B[1][2]) / det;
    Bi[2][0] = (B[1][0] * B[2][1] - B[1][1] * B[2][0]) / det;
    Bi[2][1] = (B[0][1] * B[2][0] - B[0][0] * B[2][1]) / det;
    Bi[2][2] = (B[0][0] * B[1][1] - B[0][1] * B[1][0]) / det;
    double g[4][3];
    for (int d = 0; d < 3; ++d) {
        g[1][d] = Bi[0][d];
        g[2][d] = Bi[1][d];
        g[3][d] = Bi[2][d];
        g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    }
    double vol = fabs(det) / 6.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            Ke[a][b] = vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
            Me[a][b] = vol / 20.0 * (a == b ? 2.0 : 1.0);
        }
    /* load vector by the 4-point degree-2 rule */
    const double qa = (5.0 + 3.0 * sqrt(5.0)) / 20.0;
    const double qb = (5.0 - sqrt(5.0)) / 20.0;
    for (int a = 0; a < 4; ++a) fe[a] = 0.0;
    for (int q = 0; q < 4; ++q) {
        double x[3];
        double lam[4];
        for (int a = 0; a < 4; ++a) lam[a] = (a == q) ? qa : qb;
        for (int d = 0; d < 3; ++d)
            x[d] = lam[0] * p[0][d] + lam[1] * p[1][d] + lam[2] * p[2][d] + lam[3] * p[3][d];
        double u;
        if (t->kind == 2) {
            u = 0.0;
            for (int a = 0; a < 4; ++a) u += lam[a] * t->nodal[tv[a]];
        } else {
            u = target_at(t, x);
        }
        for (int a = 0; a < 4; ++a) fe[a] += vol / 4.0 * u * lam[a];
    }
    *vol_out = vol;
    return 0;
}

/* exported for the element-level pins */
int orc_element(const double *xyz, const int32_t *tv, const orc_target *t,
                double *Ke, double *Me, double *fe, double *vol)
{
    double K[4][4], M[4][4], F[4];
    int rc = element(xyz, tv, t, K, M, F, vol);
    for (int a = 0; a < 4; ++a) {
        fe[a] = F[a];
        for (int b = 0; b < 4; ++b) {
            Ke[4 * a + b] = K[a][b];
            Me[4 * a + b] = M[a][b];
        }
    }
    return rc;
}

/* ---------------------------------------------------------- the assembly */
typedef struct {
    int64_t n;          /* interior unknowns */
    int64_t nnz;
    int64_t *row_ptr;   /* [n+1] */
    int32_t *col;       /* [nnz] sorted per row */
    double *val;        /* [nnz] */
    double *valK;       /* [nnz] K part (optional) */
    double *valM;       /* [nnz] M part (optional) */
    double *f;          /* [n] */
    int32_t *dof_of_vertex;  /* [nv], -1 on Gamma */
    int32_t *vertex_of_dof;  /* [n] */
} orc_system;

void orc_free(orc_system *s)
{
    if (!s) return;
    free(s->row_ptr); free(s->col); free(s->val); free(s->valK); free(s->valM);
    free(s->f); free(s->dof_of_vertex); free(s->vertex_of_dof);
    memset(s, 0, sizeof(*s));
}

/* Incidence lists vertex -> tets containing it, tets in ascending order. */
static int build_incidence(int64_t nv, int64_t nt, const int32_t *tets,
                           int64_t **ptr_out, int64_t **lst_out)
{
    int64_t *ptr = calloc((size_t)nv + 1, sizeof(int64_t));
    if (!ptr) return -3;
    for (int64_t e = 0; e < nt; ++e)
        for (int a = 0; a < 4; ++a) {
            int32_t v = tets[4 * e + a];
            if (v < 0 || v >= nv) { free(ptr); return -2; }
            ptr[v + 1]++;
        }
    for (int64_t v = 0; v < nv; ++v) ptr[v + 1] += ptr[v];
    int64_t *lst = malloc(sizeof(int64_t) * (size_t)(ptr[nv] > 0 ? ptr[nv] : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(nv > 0 ? nv : 1));
    if (!lst || !fill) { free(ptr); free(lst); free(fill); return -3; }
    for (int64_t v = 0; v < nv; ++v) fill[v] = ptr[v];
    for (int64_t e = 0; e < nt; ++e)
        for (int a = 0; a < 4; ++a) {
            int32_t v = tets[4 * e + a];
            lst[fill[v]++] = e;
        }
    free(fill);
    *ptr_out = ptr;
    *lst_out = lst;
    return 0;
}

/* Row i of A (and f_i), accumulated over the tets incident to vertex vi.
 * Columns are the interior vertices of those tets, kept sorted. */
typedef struct { int32_t col; double v, k, m; } orc_entry;

static int assemble_row(int32_t vi, const double *xyz, const int32_t *tets,
                        int64_t q0, int64_t q1, const int64_t *ilst,
                        const int32_t *dof, double rho, const orc_target *t,
                        orc_entry *buf, int cap, int *cnt_out, double *f_out)
{
    int cnt = 0;
    double fi = 0.0;
    for (int64_t q = q0; q < q1; ++q) {
        int64_t e = ilst[q];
        const int32_t *tv = tets + 4 * e;
        double Ke[4][4], Me[4][4], fe[4], vol;
        if (element(xyz, tv, t, Ke, Me, fe, &vol) != 0) return -2;
        int a = 0;
        while (tv[a] != vi) ++a;
        fi += fe[a];
        for (int b = 0; b < 4; ++b) {
            int32_t j = dof[tv[b]];
            if (j < 0) continue;
            int s = 0;
            while (s < cnt && buf[s].col != j) ++s;
            if (s == cnt) {
                if (cnt == cap) return -4;
                buf[cnt].col = j; buf[cnt].v = 0.0; buf[cnt].k = 0.0; buf[cnt].m = 0.0;
                ++cnt;
            }
            buf[s].k += Ke[a][b];
            buf[s].m += Me[a][b];
            buf[s].v += rho * Ke[a][b] + Me[a][b];
        }
    }
    /* insertion sort by column */
    for (int s = 1; s < cnt; ++s) {
        orc_entry x = buf[s];
        int r = s - 1;
        while (r >= 0 && buf[r].col > x.col) { buf[r + 1] = buf[r]; --r; }
        buf[r + 1] = x;
    }
    *cnt_out = cnt;
    *f_out = fi;
    return 0;
}

#define ORC_ROW_CAP 512

/* Assemble A = rho K + M and f on the interior vertices.
 * Returns 0, -2 (bad mesh: index out of range, zero volume, row too long),
 * -3 (out of memory). */
int orc_assemble(int64_t nv, const double *xyz, int64_t nt, const int32_t *tets,
                 const uint8_t *dirichlet, double rho, const orc_target *t,
                 int keep_km, orc_system *out)
{
    memset(out, 0, sizeof(*out));
    int64_t *iptr = NULL, *ilst = NULL;
    int rc = build_incidence(nv, nt, tets, &iptr, &ilst);
    if (rc) return rc;
    int32_t *dof = malloc(sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1));
    int64_t n = 0;
    for (int64_t v = 0; v < nv; ++v) dof[v] = dirichlet[v] ? -1 : (int32_t)(n++);
    int32_t *vod = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t v = 0; v < nv; ++v) if (dof[v] >= 0) vod[dof[v]] = (int32_t)v;
    int64_t *rp = calloc((size_t)n + 1, sizeof(int64_t));
    double *f = calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    int err = 0;
    /* pass 1: row lengths */
#pragma omp parallel
    {
        orc_entry *buf = malloc(sizeof(orc_entry) * ORC_ROW_CAP);
#pragma omp for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n; ++i) {
            int cnt = 0; double fi;
            int r = assemble_row(vod[i], xyz, tets, iptr[vod[i]], iptr[vod[i] + 1], ilst, dof, rho, t, buf,
                                 ORC_ROW_CAP, &cnt, &fi);
            if (r) {
#pragma omp atomic write
                err = r;
            }
            rp[i + 1] = cnt;
            f[i] = fi;
        }
        free(buf);
    }
    if (err) {
        free(iptr); free(ilst); free(dof); free(vod); free(rp); free(f);
        return err == -4 ? -2 : err;
    }
    for (int64_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
    int64_t nnz = rp[n];
    int32_t *col = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    double *val = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    double *vk = keep_km ? malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1)) : NULL;
    double *vm = keep_km ? malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1)) : NULL;
    /* pass 2: values */
#pragma omp parallel
    {
        orc_entry *buf = malloc(sizeof(orc_entry) * ORC_ROW_CAP);
#pragma omp for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n; ++i) {
            int cnt = 0; double fi;
            assemble_row(vod[i], xyz, tets, iptr[vod[i]], iptr[vod[i] + 1], ilst, dof, rho, t, buf,
                         ORC_ROW_CAP, &cnt, &fi);
            for (int s = 0; s < cnt; ++s) {
                col[rp[i] + s] = buf[s].col;
                val[rp[i] + s] = buf[s].v;
                if (keep_km) { vk[rp[i] + s] = buf[s].k; vm[rp[i] + s] = buf[s].m; }
            }
        }
        free(buf);
    }
    free(iptr); free(ilst);
    out->n = n; out->nnz = nnz; out->row_ptr = rp; out->col = col; out->val = val;
    out->valK = vk; out->valM = vm; out->f = f; out->dof_of_vertex = dof; out->vertex_of_dof = vod;
    return 0;
}

/* Rows of A and entries of f for a sample of interior vertices, without
 * assembling the rest of the matrix.  rows_v[s] is a vertex id; output row s
 * goes to cols[s*cap .. ], vals[s*cap ..], with cnt[s] entries, f[s].
 * Column ids are interior dof ids (interior vertices counted in vertex order). */
int orc_sample_rows(int64_t nv, const double *xyz, int64_t nt, const int32_t *tets,
                    const uint8_t *dirichlet, double rho, const orc_target *t,
                    int64_t ns, const int32_t *rows_v, int cap,
                    int32_t *cols, double *vals, int32_t *cnt, double *f)
{
    int32_t *dof = malloc(sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1));
    int64_t n = 0;
    for (int64_t v = 0; v < nv; ++v) dof[v] = dirichlet[v] ? -1 : (int32_t)(n++);
    /* incidence restricted to the sampled vertices: slot of each sampled vertex */
    int32_t *slot = malloc(sizeof(int32_t) * (size_t)(nv > 0 ? nv : 1));
    for (int64_t v = 0; v < nv; ++v) slot[v] = -1;
    for (int64_t s = 0; s < ns; ++s) slot[rows_v[s]] = (int32_t)s;
    int64_t *iptr = calloc((size_t)ns + 1, sizeof(int64_t));
    for (int64_t e = 0; e < nt; ++e)
        for (int a = 0; a < 4; ++a) {
            int32_t s = slot[tets[4 * e + a]];
            if (s >= 0) iptr[s + 1]++;
        }
    for (int64_t s = 0; s < ns; ++s) iptr[s + 1] += iptr[s];
    int64_t *ilst = malloc(sizeof(int64_t) * (size_t)(iptr[ns] > 0 ? iptr[ns] : 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(ns > 0 ? ns : 1));
    for (int64_t s = 0; s < ns; ++s) fill[s] = iptr[s];
    for (int64_t e = 0; e < nt; ++e)
        for (int a = 0; a < 4; ++a) {
            int32_t s = slot[tets[4 * e + a]];
            if (s >= 0) ilst[fill[s]++] = e;
        }
    int rc = 0;
    orc_entry *buf = malloc(sizeof(orc_entry) * ORC_ROW_CAP);
    for (int64_t s = 0; s < ns && !rc; ++s) {
        int32_t vi = rows_v[s];
        int c = 0; double fi;
        rc = assemble_row(vi, xyz, tets, iptr[s], iptr[s + 1], ilst, dof, rho, t, buf,
                          ORC_ROW_CAP, &c, &fi);
        if (rc) break;
        if (c > cap) { rc = -4; break; }
        cnt[s] = c;
        f[s] = fi;
        for (int q = 0; q < c; ++q) {
            cols[s * cap + q] = buf[q].col;
            vals[s * cap + q] = buf[q].v;
        }
    }
    free(buf); free(fill); free(ilst); free(iptr); free(slot); free(dof);
    return rc;
}

/* ------------------------------------------------------------ the solver */
void orc_spmv(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
              const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) s += val[q] * x[col[q]];
        y[i] = s;
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Jacobi-preconditioned CG from x = 0 until ||f - A x||_2 <= rtol ||f||_2
 * (recurrence residual), or maxit.  Returns iterations; *relres gets the
 * final recurrence residual ratio. */
int orc_pcg(int64_t n, const int64_t *rp, const int32_t *col, const double *val,
            const double *f, double *x, double rtol, int maxit, double *relres)
{
    double *r = malloc(sizeof(double) * (size_t)n);
    double *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n);
    double *dinv = malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
            if (col[k] == i) d = val[k];
        dinv[i] = 1.0 / d;
        x[i] = 0.0;
        r[i] = f[i];
        z[i] = dinv[i] * r[i];
        p[i] = z[i];
    }
    double ff = dot(n, f, f);
    double gamma = dot(n, r, z);
    double rr = ff;
    int it = 0;
    if (ff == 0.0) { *relres = 0.0; goto done; }
    while (it < maxit && rr > rtol * rtol * ff) {
        orc_spmv(n, rp, col, val, p, q);
        double alpha = gamma / dot(n, p, q);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            z[i] = dinv[i] * r[i];
        }
        rr = dot(n, r, r);
        double gnew = dot(n, r, z);
        double beta = gnew / gamma;
        gamma = gnew;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        ++it;
    }
    *relres = sqrt(rr / ff);
done:
    free(r); free(z); free(p); free(q); free(dinv);
    return it;
}

/* Threads used by the parallel loops from now on (n >= 1). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
