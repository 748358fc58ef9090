/* A small Kuhn-split cube mesh for the sanitizer drivers: (N+1)^3 vertices
 * (jittered interior), 6 N^3 tets listing their vertices along a monotone
 * lattice path, Dirichlet flag on the cube's faces. */
#ifndef SANITIZE_KUHN_H
#define SANITIZE_KUHN_H
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int64_t nv, nt;
    double *xyz;
    int32_t *tets;
    uint8_t *dirichlet;
} san_mesh;

static double san_unit(uint64_t *s) {
    *s = *s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(*s >> 11) / 9007199254740992.0;
}

static san_mesh san_kuhn(int N, double jitter) {
    san_mesh m;
    const int P = N + 1;
    m.nv = (int64_t)P * P * P;
    m.nt = 6 * (int64_t)N * N * N;
    m.xyz = (double *)malloc(sizeof(double) * 3 * (size_t)m.nv);
    m.tets = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)m.nt);
    m.dirichlet = (uint8_t *)malloc((size_t)m.nv);
    uint64_t seed = 12345;
    for (int z = 0; z < P; ++z)
        for (int y = 0; y < P; ++y)
            for (int x = 0; x < P; ++x) {
                const int64_t v = ((int64_t)z * P + y) * P + x;
                const int bd = x == 0 || y == 0 || z == 0 || x == N || y == N || z == N;
                const double h = 1.0 / N;
                m.xyz[3 * v + 0] = x * h + (bd ? 0.0 : jitter * h * (san_unit(&seed) - 0.5));
                m.xyz[3 * v + 1] = y * h + (bd ? 0.0 : jitter * h * (san_unit(&seed) - 0.5));
                m.xyz[3 * v + 2] = z * h + (bd ? 0.0 : jitter * h * (san_unit(&seed) - 0.5));
                m.dirichlet[v] = (uint8_t)bd;
            }
    /* the six monotone paths from corner (0,0,0) to (1,1,1) */
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int64_t e = 0;
    for (int z = 0; z < N; ++z)
        for (int y = 0; y < N; ++y)
            for (int x = 0; x < N; ++x)
                for (int p = 0; p < 6; ++p) {
                    int c[3] = {x, y, z};
                    m.tets[4 * e] = (int32_t)(((int64_t)c[2] * P + c[1]) * P + c[0]);
                    for (int s = 0; s < 3; ++s) {
                        ++c[perm[p][s]];
                        m.tets[4 * e + s + 1] = (int32_t)(((int64_t)c[2] * P + c[1]) * P + c[0]);
                    }
                    ++e;
                }
    return m;
}

static void san_free(san_mesh *m) {
    free(m->xyz);
    free(m->tets);
    free(m->dirichlet);
}
#endif
