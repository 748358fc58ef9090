/* Drives the CPU oracle (oracle/oracle.c, compiled into this program) through
 * assembly, sampled rows, element matrices and Jacobi-PCG on small meshes, for
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer.  Exit status
 * 0 when every call succeeds and the solves converge. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "kuhn.h"

typedef struct {
    int kind;
    int n_modes;
    const int32_t *k;
    const double *amp;
    double offset;
    double lo[3], hi[3];
    const double *nodal;
} orc_target;
typedef struct {
    int64_t n, nnz;
    int64_t *row_ptr;
    int32_t *col;
    double *val, *valK, *valM, *f;
    int32_t *dof_of_vertex, *vertex_of_dof;
} orc_system;
int orc_assemble(int64_t nv, const double *xyz, int64_t nt, const int32_t *tets, const uint8_t *dirichlet,
                 double rho, const orc_target *t, int keep_km, orc_system *out);
int orc_sample_rows(int64_t nv, const double *xyz, int64_t nt, const int32_t *tets, const uint8_t *dirichlet,
                    double rho, const orc_target *t, int64_t ns, const int32_t *rows_v, int cap, int32_t *cols,
                    double *vals, int32_t *cnt, double *f);
int orc_element(const double *xyz, const int32_t *tv, const orc_target *t, double *Ke, double *Me, double *fe,
                double *vol);
int orc_pcg(int64_t n, const int64_t *rp, const int32_t *col, const double *val, const double *f, double *x,
            double rtol, int maxit, double *relres);
void orc_spmv(int64_t n, const int64_t *rp, const int32_t *col, const double *val, const double *x, double *y);
void orc_free(orc_system *s);

static int run(int N, double jitter, const orc_target *t, int keep_km) {
    san_mesh m = san_kuhn(N, jitter);
    orc_system s;
    int rc = orc_assemble(m.nv, m.xyz, m.nt, m.tets, m.dirichlet, 1e-2, t, keep_km, &s);
    if (rc) {
        fprintf(stderr, "assemble failed %d\n", rc);
        return 1;
    }
    double *x = (double *)calloc((size_t)s.n, sizeof(double));
    double *y = (double *)calloc((size_t)s.n, sizeof(double));
    double rr = 1.0;
    const int its = orc_pcg(s.n, s.row_ptr, s.col, s.val, s.f, x, 1e-12, 1000, &rr);
    orc_spmv(s.n, s.row_ptr, s.col, s.val, x, y);
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < s.n; ++i) {
        num += (s.f[i] - y[i]) * (s.f[i] - y[i]);
        den += s.f[i] * s.f[i];
    }
    int bad = !(its > 0) || !(sqrt(num) <= 1e-10 * sqrt(den) + 1e-300);
    /* sampled rows of the first interior vertices */
    int32_t rows_v[3];
    for (int q = 0; q < 3; ++q) rows_v[q] = s.vertex_of_dof[q * (s.n / 3)];
    int32_t cols[3 * 32], cnt[3];
    double vals[3 * 32], f3[3];
    rc = orc_sample_rows(m.nv, m.xyz, m.nt, m.tets, m.dirichlet, 1e-2, t, 3, rows_v, 32, cols, vals, cnt, f3);
    bad |= rc != 0;
    double Ke[16], Me[16], fe[4], vol;
    bad |= orc_element(m.xyz, m.tets, t, Ke, Me, fe, &vol) != 0;
    free(x);
    free(y);
    orc_free(&s);
    san_free(&m);
    return bad;
}

int main(void) {
    const int32_t k[6] = {1, 1, 1, 2, 3, 1};
    const double amp[2] = {1.0, -0.5};
    orc_target sine;
    memset(&sine, 0, sizeof(sine));
    sine.kind = 0;
    sine.n_modes = 2;
    sine.k = k;
    sine.amp = amp;
    orc_target box;
    memset(&box, 0, sizeof(box));
    box.kind = 1;
    for (int d = 0; d < 3; ++d) {
        box.lo[d] = 0.25;
        box.hi[d] = 0.75;
    }
    int bad = 0;
    bad |= run(5, 0.15, &sine, 0);
    bad |= run(6, 0.0, &box, 1);
    san_mesh m = san_kuhn(4, 0.1);
    double *nod = (double *)malloc(sizeof(double) * (size_t)m.nv);
    for (int64_t v = 0; v < m.nv; ++v) nod[v] = sin(0.3 * (double)v);
    orc_target nodal;
    memset(&nodal, 0, sizeof(nodal));
    nodal.kind = 2;
    nodal.nodal = nod;
    bad |= run(4, 0.1, &nodal, 0);
    free(nod);
    san_free(&m);
    printf(bad ? "oracle driver: FAILED\n" : "oracle driver: ok\n");
    return bad;
}
