// Adaptive refinement of tetrahedral meshes by bisection (host side).
//
// Sections 4.2 and 4.3 solve on meshes refined adaptively, driven by a
// residual-based error indicator.  The refinement here is Maubach's
// bisection of tagged simplices: a tetrahedron (x0, x1, x2, x3) with tag
// d in {1, 2, 3} is cut at the midpoint z of its refinement edge (x0, x_d)
// into
//     (x0, ..., x_{d-1}, z, x_{d+1}, ..., x3)  and  (x1, ..., x_d, z, x_{d+1}, ..., x3),
// both with tag d - 1 (3 after 1).  Meshes whose tetrahedra list their
// vertices along paths of a reflected (Kuhn) lattice, all with tag 3 (the
// Kuhn split stores each cube's six tetrahedra that way), stay conforming if
// every tetrahedron with a bisected edge is bisected in turn until none has
// one (the closure below), and the tetrahedra fall into finitely many shape
// classes.  Marking is Doerfler's bulk criterion: the smallest set of
// tetrahedra, largest indicators first, whose squared indicators sum to at
// least theta times the total.
//
// The mesh under refinement lives in host memory (the refinement is a
// sequence of small, irregular updates; the solver then assembles on the
// device mesh uploaded from it).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ocpamg.h"

struct ocp_refiner {
    std::vector<double> xyz;                   // [nv][3]
    std::vector<std::array<int32_t, 4>> tv;    // ordered vertices of every leaf
    std::vector<int8_t> tag;                   // refinement tag of every leaf
    std::unordered_map<uint64_t, int32_t> mid; // edge (lo, hi) -> its midpoint vertex
    std::vector<uint8_t> dirichlet;            // vertices on boundary faces
    std::string err;
};

namespace {

inline uint64_t edge_key(int32_t a, int32_t b) {
    const uint32_t lo = (uint32_t)std::min(a, b), hi = (uint32_t)std::max(a, b);
    return ((uint64_t)hi << 32) | lo;
}

int32_t midpoint(ocp_refiner *r, int32_t a, int32_t b) {
    const uint64_t k = edge_key(a, b);
    auto it = r->mid.find(k);
    if (it != r->mid.end()) return it->second;
    const int32_t v = (int32_t)(r->xyz.size() / 3);
    for (int d = 0; d < 3; ++d) r->xyz.push_back(0.5 * (r->xyz[3 * (size_t)a + d] + r->xyz[3 * (size_t)b + d]));
    r->mid.emplace(k, v);
    return v;
}

// bisect leaf t: it becomes the first child, the second is appended
void bisect(ocp_refiner *r, size_t t) {
    const std::array<int32_t, 4> x = r->tv[t];
    const int d = r->tag[t];
    const int32_t z = midpoint(r, x[0], x[d]);
    std::array<int32_t, 4> c1{}, c2{};
    int p = 0;
    for (int i = 0; i < d; ++i) c1[p++] = x[i];
    c1[p++] = z;
    for (int i = d + 1; i < 4; ++i) c1[p++] = x[i];
    p = 0;
    for (int i = 1; i <= d; ++i) c2[p++] = x[i];
    c2[p++] = z;
    for (int i = d + 1; i < 4; ++i) c2[p++] = x[i];
    const int8_t nt = (int8_t)(d > 1 ? d - 1 : 3);
    r->tv[t] = c1;
    r->tag[t] = nt;
    r->tv.push_back(c2);
    r->tag.push_back(nt);
}

bool has_hanging_edge(const ocp_refiner *r, const std::array<int32_t, 4> &x) {
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b)
            if (r->mid.count(edge_key(x[a], x[b]))) return true;
    return false;
}

// Dirichlet vertices = vertices of faces that belong to one tetrahedron only
void boundary_from_faces(ocp_refiner *r) {
    const size_t nv = r->xyz.size() / 3;
    std::vector<std::array<int32_t, 3>> faces;
    faces.reserve(4 * r->tv.size());
    for (const auto &x : r->tv)
        for (int a = 0; a < 4; ++a) {
            std::array<int32_t, 3> f{};
            int p = 0;
            for (int b = 0; b < 4; ++b)
                if (b != a) f[p++] = x[b];
            std::sort(f.begin(), f.end());
            faces.push_back(f);
        }
    std::sort(faces.begin(), faces.end());
    r->dirichlet.assign(nv, 0);
    for (size_t i = 0; i < faces.size();) {
        size_t j = i + 1;
        while (j < faces.size() && faces[j] == faces[i]) ++j;
        if (j - i == 1)
            for (int32_t v : faces[i]) r->dirichlet[v] = 1;
        i = j;
    }
}

}  // namespace

extern "C" int ocp_refiner_create(const double *xyz, int32_t n_vertices, const int32_t *tets, int32_t n_tets,
                                  ocp_refiner **out) {
    if (!out) return OCP_ERR_INVALID_ARG;
    *out = nullptr;
    if (!xyz || !tets || n_vertices <= 0 || n_tets <= 0) return OCP_ERR_INVALID_ARG;
    for (int64_t i = 0; i < 4 * (int64_t)n_tets; ++i)
        if (tets[i] < 0 || tets[i] >= n_vertices) return OCP_ERR_BAD_MESH;
    ocp_refiner *r = new ocp_refiner();
    r->xyz.assign(xyz, xyz + 3 * (size_t)n_vertices);
    r->tv.resize((size_t)n_tets);
    for (int32_t e = 0; e < n_tets; ++e)
        for (int a = 0; a < 4; ++a) r->tv[e][a] = tets[4 * (size_t)e + a];
    r->tag.assign((size_t)n_tets, 3);
    boundary_from_faces(r);
    *out = r;
    return OCP_OK;
}

extern "C" void ocp_refiner_destroy(ocp_refiner *r) { delete r; }

extern "C" int ocp_refiner_refine(ocp_refiner *r, const double *eta2, double theta, int32_t *n_marked) {
    if (!r || !eta2 || !(theta > 0.0) || !(theta <= 1.0)) return OCP_ERR_INVALID_ARG;
    const size_t nt = r->tv.size();
    // Doerfler marking: largest indicators first until theta of the total
    std::vector<int32_t> order(nt);
    std::iota(order.begin(), order.end(), 0);
    double total = 0.0;
    for (size_t e = 0; e < nt; ++e) {
        if (!(eta2[e] >= 0.0) || !std::isfinite(eta2[e])) return OCP_ERR_INVALID_ARG;
        total += eta2[e];
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return eta2[a] > eta2[b]; });
    std::vector<uint8_t> mark(nt, 0);
    double acc = 0.0;
    int32_t m = 0;
    for (size_t q = 0; q < nt && (acc < theta * total || m == 0); ++q) {
        mark[order[q]] = 1;
        acc += eta2[order[q]];
        ++m;
    }
    if (n_marked) *n_marked = m;
    // bisect the marked tetrahedra, then every tetrahedron with a bisected
    // edge, until none is left
    for (size_t e = 0; e < nt; ++e)
        if (mark[e]) bisect(r, e);
    for (int pass = 0;; ++pass) {
        if (pass > 200) {
            r->err = "refinement closure did not terminate";
            return OCP_ERR_BAD_MESH;
        }
        std::vector<size_t> todo;
        for (size_t e = 0; e < r->tv.size(); ++e)
            if (has_hanging_edge(r, r->tv[e])) todo.push_back(e);
        if (todo.empty()) break;
        for (size_t e : todo) bisect(r, e);
    }
    boundary_from_faces(r);
    return OCP_OK;
}

extern "C" int ocp_refiner_sizes(const ocp_refiner *r, int32_t *n_vertices, int32_t *n_tets) {
    if (!r || !n_vertices || !n_tets) return OCP_ERR_INVALID_ARG;
    if (r->xyz.size() / 3 > (size_t)INT32_MAX || r->tv.size() > (size_t)INT32_MAX / 4) return OCP_ERR_UNSUPPORTED;
    *n_vertices = (int32_t)(r->xyz.size() / 3);
    *n_tets = (int32_t)r->tv.size();
    return OCP_OK;
}

extern "C" int ocp_refiner_get(const ocp_refiner *r, double *xyz, int32_t *tets, uint8_t *dirichlet) {
    if (!r) return OCP_ERR_INVALID_ARG;
    if (xyz) std::memcpy(xyz, r->xyz.data(), sizeof(double) * r->xyz.size());
    if (tets)
        for (size_t e = 0; e < r->tv.size(); ++e)
            for (int a = 0; a < 4; ++a) tets[4 * e + a] = r->tv[e][a];
    if (dirichlet) std::memcpy(dirichlet, r->dirichlet.data(), r->dirichlet.size());
    return OCP_OK;
}
