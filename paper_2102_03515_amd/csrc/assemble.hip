// Finite element assembly of A = rho*K + M and f = (int ubar phi_i) into CSR
// (Section 2, system (linsys) and the entries K_ij, M_ij, f_i defined there).
//
// Row-owned, atomic-free on values: every interior vertex owns its row and
// sums the element matrices and element loads of its incident tetrahedra in
// ascending tet id.  The result is bitwise deterministic (and A bitwise
// symmetric).
//
//   1. per tet: index/degeneracy checks, incidence counts   (int atomics)
//   2. scan -> incidence pointers; fill; sort each list      (vertex -> tets)
//   3. dof numbering of interior vertices (scan)
//   4. per tet: element loads by the 4-point degree-2 rule
//   5. rows of at most 16 entries: one pass per row that recomputes the
//      element matrix of every incident tet from its coordinates;
//      otherwise per tet an element record (dofs, element matrix, loads),
//      then symbolic rows (sorted union of the interior vertices of the
//      incident tets) and numeric rows (sums of the records' entries)
#include <cfloat>
#include <climits>
#include <cmath>

#include <type_traits>

#include "kernels.h"
#include "system.h"

namespace ocp {

constexpr int kAsmBlock = 64;
constexpr int kRowCap = 128;       // max entries of one assembled row
constexpr int kSineTable = 8;      // sin(k pi x) by recurrence for k <= 8

// ----------------------------------------------------------------- geometry
// Barycentric gradients g[a] and signed determinant of the edge matrix of a
// tetrahedron p[0..3].  lambda_{c+1}(x) = (B^{-1}(x - p0))_c with
// B = [p1-p0, p2-p0, p3-p0], so grad lambda_{c+1} is row c of B^{-1} and
// grad lambda_0 = -(sum of the others).  No multiply-add is fused here (nor
// in elem_values): every kernel that inlines these computes the same bits.
__device__ __forceinline__ double tet_gradients(const double p[4][3], double g[4][3]) {
#pragma clang fp contract(off)
    double e[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r) e[r][c] = p[c + 1][r] - p[0][r];
    // cofactors
    const double c00 = e[1][1] * e[2][2] - e[1][2] * e[2][1];
    const double c01 = e[1][2] * e[2][0] - e[1][0] * e[2][2];
    const double c02 = e[1][0] * e[2][1] - e[1][1] * e[2][0];
    const double det = e[0][0] * c00 + e[0][1] * c01 + e[0][2] * c02;
    const double id = 1.0 / det;
    // rows of B^{-1} = adj(B)/det, adj = cofactor^T
    g[1][0] = c00 * id;
    g[1][1] = (e[0][2] * e[2][1] - e[0][1] * e[2][2]) * id;
    g[1][2] = (e[0][1] * e[1][2] - e[0][2] * e[1][1]) * id;
    g[2][0] = c01 * id;
    g[2][1] = (e[0][0] * e[2][2] - e[0][2] * e[2][0]) * id;
    g[2][2] = (e[0][2] * e[1][0] - e[0][0] * e[1][2]) * id;
    g[3][0] = c02 * id;
    g[3][1] = (e[0][1] * e[2][0] - e[0][0] * e[2][1]) * id;
    g[3][2] = (e[0][0] * e[1][1] - e[0][1] * e[1][0]) * id;
#pragma unroll
    for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    return det;
}

__device__ __forceinline__ void load_tet(const double *__restrict__ xyz, const int4 tv,
                                         double p[4][3]) {
    const int v[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int d = 0; d < 3; ++d) p[a][d] = xyz[3 * (int64_t)v[a] + d];
}

// ------------------------------------------------------- 1. check + count
// The 4 x 256 vertex references of a block's tets are first combined in an
// LDS hash table (consecutive tets share most vertices), so each distinct
// vertex costs one global atomic per block instead of one per reference.
constexpr int kIncBlock = 256;
constexpr int kIncHash = 2048;

__device__ __forceinline__ int inc_slot(int *keys, int v) {
    int s = (int)(((uint32_t)v * 2654435761u) >> (32 - 11));
    for (;;) {
        const int prev = atomicCAS(&keys[s], -1, v);
        if (prev == -1 || prev == v) return s;
        s = (s + 1) & (kIncHash - 1);
    }
}

__global__ void __launch_bounds__(kIncBlock) k_tet_check_count(const int4 *__restrict__ tets, int64_t nt,
                                                               const double *__restrict__ xyz, int32_t nv,
                                                               int32_t *__restrict__ inc_cnt,
                                                               int32_t *__restrict__ flag) {
    __shared__ int keys[kIncHash];
    __shared__ int cnt[kIncHash];
    for (int q = threadIdx.x; q < kIncHash; q += kIncBlock) {
        keys[q] = -1;
        cnt[q] = 0;
    }
    __syncthreads();
    const int64_t e = (int64_t)blockIdx.x * kIncBlock + threadIdx.x;
    bool ok = e < nt;
    int v[4] = {0, 0, 0, 0};
    if (ok) {
        const int4 tv = tets[e];
        v[0] = tv.x;
        v[1] = tv.y;
        v[2] = tv.z;
        v[3] = tv.w;
#pragma unroll
        for (int a = 0; a < 4; ++a)
            if (v[a] < 0 || v[a] >= nv) ok = false;
        if (!ok) {
            atomicOr(flag, 1);
        } else {
            double p[4][3];
            load_tet(xyz, tv, p);
            double l2 = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = a + 1; b < 4; ++b) {
                    double s = 0.0;
#pragma unroll
                    for (int d = 0; d < 3; ++d) s += (p[a][d] - p[b][d]) * (p[a][d] - p[b][d]);
                    l2 = fmax(l2, s);
                }
            double e3[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int r = 0; r < 3; ++r) e3[r][c] = p[c + 1][r] - p[0][r];
            const double det = e3[0][0] * (e3[1][1] * e3[2][2] - e3[1][2] * e3[2][1]) -
                               e3[0][1] * (e3[1][0] * e3[2][2] - e3[1][2] * e3[2][0]) +
                               e3[0][2] * (e3[1][0] * e3[2][1] - e3[1][1] * e3[2][0]);
            if (!(fabs(det) > 1e-12 * l2 * sqrt(l2))) {
                atomicOr(flag, 2);
                ok = false;
            }
        }
    }
    if (ok) {
#pragma unroll
        for (int a = 0; a < 4; ++a) atomicAdd(&cnt[inc_slot(keys, v[a])], 1);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kIncHash; q += kIncBlock)
        if (keys[q] >= 0) atomicAdd(&inc_cnt[keys[q]], cnt[q]);
}

// ------------------------------------------------------ 2. incidence lists
// Same LDS combining: one global atomic per distinct vertex reserves the
// block's range in that vertex's list; references get local offsets.  An
// entry is the code (e << 2) | a: tet e, in which the vertex is local vertex
// a (fits in int32: at most 2^29 tets).  Codes sort like tet ids.
__global__ void __launch_bounds__(kIncBlock) k_tet_fill(const int4 *__restrict__ tets, int64_t nt,
                                                        const int32_t *__restrict__ inc_ptr,
                                                        int32_t *__restrict__ fill, int32_t *__restrict__ inc) {
    __shared__ int keys[kIncHash];
    __shared__ int cnt[kIncHash];
    __shared__ int base[kIncHash];
    for (int q = threadIdx.x; q < kIncHash; q += kIncBlock) {
        keys[q] = -1;
        cnt[q] = 0;
    }
    __syncthreads();
    const int64_t e = (int64_t)blockIdx.x * kIncBlock + threadIdx.x;
    int slot[4] = {0, 0, 0, 0}, pos[4] = {0, 0, 0, 0};
    if (e < nt) {
        const int4 tv = tets[e];
        const int v[4] = {tv.x, tv.y, tv.z, tv.w};
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            slot[a] = inc_slot(keys, v[a]);
            pos[a] = atomicAdd(&cnt[slot[a]], 1);
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kIncHash; q += kIncBlock)
        if (keys[q] >= 0) base[q] = inc_ptr[keys[q]] + atomicAdd(&fill[keys[q]], cnt[q]);
    __syncthreads();
    if (e < nt) {
#pragma unroll
        for (int a = 0; a < 4; ++a) inc[base[slot[a]] + pos[a]] = (int32_t)((e << 2) | a);
    }
}

// Sort each vertex's list of incidence codes ascending: a 32-wide sorting
// network in registers for the common case, insertion sort otherwise.  One
// wavefront per 64 consecutive vertices, whose lists are contiguous: when
// they fit kSortStage codes and none is longer than 32, the wavefront stages
// them in LDS with coalesced loads, each lane sorts its list from there, and
// the lists go back with coalesced stores (a lane reading its own list from
// global memory touched 64 lines per load).  Otherwise each lane sorts its
// list in place in global memory.
constexpr int kSortStage = 2048;
__device__ __forceinline__ void sort32(int (&r)[32]) {
    // bitonic sorting network on 32 keys
#pragma unroll
    for (int k = 2; k <= 32; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const int x = r[i], y = r[l];
                    const bool sw = up ? (x > y) : (x < y);
                    r[i] = sw ? y : x;
                    r[l] = sw ? x : y;
                }
            }
}
__global__ void __launch_bounds__(64) k_inc_sort(const int32_t *__restrict__ inc_ptr, int32_t *__restrict__ inc,
                                                 int32_t nv) {
    __shared__ int32_t stage[kSortStage];
    const int v0 = blockIdx.x * 64;
    const int v = v0 + (int)threadIdx.x;
    const int vend = v0 + 64 < nv ? v0 + 64 : nv;
    const int g0 = inc_ptr[v0], g1 = inc_ptr[vend];
    const int b = v < nv ? inc_ptr[v] : g1;
    const int len = v < nv ? inc_ptr[v + 1] - b : 0;
    const bool staged = g1 - g0 <= kSortStage && __all(len <= 32);   // uniform over the wavefront
    if (staged) {
        for (int k = (int)threadIdx.x; k < g1 - g0; k += 64) stage[k] = inc[g0 + k];
        __syncthreads();
        if (len > 1) {
            const int o = b - g0;
            int r[32];
#pragma unroll
            for (int i = 0; i < 32; ++i) r[i] = i < len ? stage[o + i] : INT_MAX;
            sort32(r);
#pragma unroll
            for (int i = 0; i < 32; ++i)
                if (i < len) stage[o + i] = r[i];
        }
        __syncthreads();
        for (int k = (int)threadIdx.x; k < g1 - g0; k += 64) inc[g0 + k] = stage[k];
        return;
    }
    if (v >= nv || len <= 1) return;
    if (len <= 32) {
        int r[32];
#pragma unroll
        for (int i = 0; i < 32; ++i) r[i] = i < len ? inc[b + i] : INT_MAX;
        sort32(r);
#pragma unroll
        for (int i = 0; i < 32; ++i)
            if (i < len) inc[b + i] = r[i];
    } else {
        for (int i = 1; i < len; ++i) {
            const int x = inc[b + i];
            int j = i - 1;
            while (j >= 0 && inc[b + j] > x) {
                inc[b + j + 1] = inc[b + j];
                --j;
            }
            inc[b + j + 1] = x;
        }
    }
}

// ----------------------------------------------------------- 3. dof maps
__global__ void k_interior_flags(const uint8_t *__restrict__ dirichlet, int32_t nv, int32_t *__restrict__ fl) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < nv) fl[v] = dirichlet[v] ? 0 : 1;
}

__global__ void k_dof_maps(const uint8_t *__restrict__ dirichlet, const int32_t *__restrict__ pos, int32_t nv,
                           int32_t *__restrict__ dof_of_vertex, int32_t *__restrict__ vertex_of_dof) {
    int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    if (dirichlet[v]) {
        dof_of_vertex[v] = -1;
    } else {
        dof_of_vertex[v] = pos[v];
        vertex_of_dof[pos[v]] = v;
    }
}

// ---------------------------------------------------- 5. symbolic rows
// pass 0: row_cnt[i] = number of distinct interior neighbours (incl. i); rows
//         of at most kPadW entries are also written, sorted, to pad[i][.]
// pass 1: write the sorted list to col[row_ptr[i] ..] (only needed when some
//         row exceeded kPadW)
constexpr int kPadW = 32;
template <int CAP>
__global__ void __launch_bounds__(kAsmBlock) k_row_symbolic(
    int pass, int32_t n, const int32_t *__restrict__ vertex_of_dof, const int32_t *__restrict__ inc_ptr,
    const int32_t *__restrict__ inc, const int4 *__restrict__ tdof, int32_t *__restrict__ row_cnt,
    const int32_t *__restrict__ row_ptr, int32_t *__restrict__ col, int32_t *__restrict__ pad,
    int32_t *__restrict__ flag) {
    __shared__ int32_t lst[CAP][kAsmBlock];
    const int t = threadIdx.x;
    // XCD x takes a contiguous run of blocks (measured faster here)
    const int i = (int)dev::xcd_tile(blockIdx.x, gridDim.x) * kAsmBlock + t;
    if (i >= n) return;
    const int vi = vertex_of_dof[i];
    int cnt = 0;
    const int qe = inc_ptr[vi + 1];
    // the dof quadruples of U incident tets are requested before any is used
    constexpr int U = 8;
    for (int q0 = inc_ptr[vi]; q0 < qe; q0 += U) {
        int4 td[U];
#pragma unroll
        for (int u = 0; u < U; ++u) td[u] = q0 + u < qe ? tdof[inc[q0 + u] >> 2] : make_int4(-1, -1, -1, -1);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int dd[4] = {td[u].x, td[u].y, td[u].z, td[u].w};
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int d = dd[a];
                if (d < 0) continue;
                // insert d into the sorted list lst[0..cnt)
                int s = cnt - 1;
                while (s >= 0 && lst[s][t] > d) --s;
                if (s >= 0 && lst[s][t] == d) continue;
                if (cnt == CAP) {
                    atomicOr(flag, CAP == kRowCap ? 4 : 128);
                    return;
                }
                for (int w = cnt - 1; w > s; --w) lst[w + 1][t] = lst[w][t];
                lst[s + 1][t] = d;
                ++cnt;
            }
        }
    }
    if (pass == 0) {
        row_cnt[i] = cnt;
        if (pad)
            for (int s = 0; s < cnt; ++s) pad[(int64_t)i * kPadW + s] = lst[s][t];
    } else {
        const int b = row_ptr[i];
        for (int s = 0; s < cnt; ++s) col[b + s] = lst[s][t];
    }
}

// copy the padded sorted lists into CSR, kPadLanes lanes per row
constexpr int kPadLanes = 16;
__global__ void k_pad_to_csr(int32_t n, const int32_t *__restrict__ pad, const int32_t *__restrict__ row_ptr,
                             int32_t *__restrict__ col) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / kPadLanes), s0 = (int)(t % kPadLanes);
    if (i >= n) return;
    const int b = row_ptr[i], len = row_ptr[i + 1] - b;
    for (int s = s0; s < len; s += kPadLanes) col[b + s] = pad[(int64_t)i * kPadW + s];
}

// --------------------------------------------- 4. element loads and records
// One sine mode as the kernel reads it: 32 bytes, so that a batch of
// kModeBatch modes is a few wide scalar loads issued together.
struct SineMode {
    int32_t k[3];
    int32_t pad;
    double amp;
    double pad2;
};
constexpr int kModeBatch = 8;   // modes are padded on the host to a multiple (amp 0)

struct TargetDev {
    int32_t kind;
    int32_t n_modes;          // padded to a multiple of kModeBatch
    const SineMode *modes;    // device [n_modes] (targets with a wave number > kSineTable)
    // targets whose wave numbers are all <= kSineTable: the amplitudes
    // summed by wave vector, dense[(k1-1) T^2 + (k2-1) T + (k3-1)] with
    // T = kSineTable, and bit (k1-1) T + (k2-1) of `pairs` set when some mode
    // has that (k1, k2)
    const double *dense;
    uint64_t pairs;
    double offset;
    double lo[3], hi[3];
    const double *nodal;      // device [n_vertices]
};
static_assert(kSineTable * kSineTable <= 64, "pairs mask holds kSineTable^2 bits");

// sin(k pi x_d) for k = 1..kSineTable from the three-term recurrence
// s_{k+1} = 2 cos(pi x) s_k - s_{k-1}, seeded with sincospi.
__device__ __forceinline__ void sine_table(double xd, double (&tab)[kSineTable]) {
    double s, c;
    sincospi(xd, &s, &c);
    double sm1 = 0.0, sk = s;
#pragma unroll
    for (int k = 0; k < kSineTable; ++k) {
        tab[k] = sk;
        const double sn = 2.0 * c * sk - sm1;
        sm1 = sk;
        sk = sn;
    }
}

// ubar(x) for sine modes with every wave number <= kSineTable, as the
// separable contraction
//   ubar = offset + sum_k1 s1[k1] sum_k2 s2[k2] sum_k3 A[k1,k2,k3] s3[k3]
// over the dense amplitude array A: every table index is a compile-time
// constant (no indexed register moves), A comes in through wide scalar
// loads, and (k1, k2) pairs that no mode uses are skipped by a uniform
// branch.  Amplitudes of equal wave vectors are summed on the host.
__device__ double eval_sine_dense(const TargetDev &t, const double x[3]) {
    double t0[kSineTable], t1[kSineTable], t2[kSineTable];
    sine_table(x[0], t0);
    sine_table(x[1], t1);
    sine_table(x[2], t2);
    double u = t.offset;
#pragma unroll
    for (int a = 0; a < kSineTable; ++a) {
        double ua = 0.0;
#pragma unroll
        for (int b = 0; b < kSineTable; ++b) {
            if ((t.pairs >> (a * kSineTable + b)) & 1) {
                const double *c = t.dense + (a * kSineTable + b) * kSineTable;
                double w = 0.0;
#pragma unroll
                for (int k = 0; k < kSineTable; ++k) w += c[k] * t2[k];
                ua += t1[b] * w;
            }
        }
        u += t0[a] * ua;
    }
    return u;
}

// ubar(x) for sine modes in general: wave numbers <= kSineTable read the
// recurrence tables (a mode's wave numbers are the same for every lane, so
// the index is uniform), larger ones call sinpi.  The modes are added in
// their given order.
__device__ double eval_sine(const TargetDev &t, const double x[3]) {
    double t0[kSineTable], t1[kSineTable], t2[kSineTable];
    sine_table(x[0], t0);
    sine_table(x[1], t1);
    sine_table(x[2], t2);
    auto factor = [&](int k, const double *tab, double xd) {
        return k <= kSineTable ? tab[k - 1] : sinpi((double)k * xd);
    };
    double u = t.offset;
    for (int m0 = 0; m0 < t.n_modes; m0 += kModeBatch) {
        SineMode md[kModeBatch];
#pragma unroll
        for (int j = 0; j < kModeBatch; ++j) md[j] = t.modes[m0 + j];
#pragma unroll
        for (int j = 0; j < kModeBatch; ++j) {
            const double f0 = factor(md[j].k[0], t0, x[0]);
            const double f1 = factor(md[j].k[1], t1, x[1]);
            const double f2 = factor(md[j].k[2], t2, x[2]);
            u += md[j].amp * f0 * f1 * f2;
        }
    }
    return u;
}

// Element records, one 128-byte line per tet:
//   ints 0..3      dof numbers of the 4 vertices (-1 on the boundary)
//   doubles 2..11  the 10 distinct entries (a <= b, packed row by row) of the
//                  symmetric element matrix rho K_e + M_e, or of K_e alone
//                  when K and M are kept apart (then |tau| goes to vol[e])
//   doubles 12..15 the element loads
// with K_e[a][b] = |tau| grad phi_a . grad phi_b and M_e[a][b] =
// |tau|/20 (1 + delta_ab).  Every entry is computed once, so the element
// matrix is exactly symmetric.
constexpr int kRecD = 16;   // doubles per record
constexpr int kRecVal = 2, kRecFe = 12;
__device__ __forceinline__ int sym_index(int a, int b) {   // packed (min, max) position
    const int i = a < b ? a : b, j = a < b ? b : a;
    return i * 4 - (i * (i - 1)) / 2 + (j - i);
}

// the 10 record values of one tet and |tau|
template <bool KM>
__device__ __forceinline__ void elem_values(const double p[4][3], double rho, double v[10], double &vol) {
#pragma clang fp contract(off)
    double g[4][3];
    const double det = tet_gradients(p, g);
    vol = fabs(det) / 6.0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) {
            const double kab = vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
            const double mab = vol / 20.0 * (b == a ? 2.0 : 1.0);
            v[sym_index(a, b)] = KM ? kab : rho * kab + mab;
        }
}

__device__ __forceinline__ double ints_as_double(int lo, int hi) {
    return __longlong_as_double((long long)(uint32_t)lo | ((long long)(uint32_t)hi << 32));
}

// One lane per quadrature point (4 lanes per tet); the 4 point contributions
// are added in a fixed order across the lanes.  REC = 0: the element loads go
// to fe[e].  REC = 1 (rho K + M) or 2 (K, with |tau| to vol[e]): the whole
// element record is written, lane q storing its doubles 4q .. 4q+3 (so a
// wavefront's store covers 16 consecutive records), and the vertex dofs also
// go to tdof[e].
constexpr int kLoadBlock = 128;
struct RecOut {
    const int32_t *dof_of_vertex;
    double rho;
    double *rec;
    double *vol;
    int4 *tdof;
};
template <bool TABLE_ONLY, int REC>
__global__ void __launch_bounds__(kLoadBlock) k_tet_load(const int4 *__restrict__ tets, int64_t nt,
                                                         const double *__restrict__ xyz, TargetDev tg,
                                                         double4 *__restrict__ fe, RecOut ro) {
    const int64_t tid = (int64_t)blockIdx.x * kLoadBlock + threadIdx.x;
    const int64_t e = tid >> 2;
    const int q = (int)(tid & 3);
    if (e >= nt) return;   // uniform over the 4 lanes of a tet
    const int4 tv = tets[e];
    double p[4][3];
    load_tet(xyz, tv, p);
    double e3[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r) e3[r][c] = p[c + 1][r] - p[0][r];
    const double det = e3[0][0] * (e3[1][1] * e3[2][2] - e3[1][2] * e3[2][1]) -
                       e3[0][1] * (e3[1][0] * e3[2][2] - e3[1][2] * e3[2][0]) +
                       e3[0][2] * (e3[1][0] * e3[2][1] - e3[1][1] * e3[2][0]);
    const double w = fabs(det) / 6.0 / 4.0;  // |tau|/4 per quadrature point
    // barycentric point q: (a,b,b,b) with a at position q
    const double qa = 0.5854101966249685;   // (5 + 3 sqrt5) / 20
    const double qb = 0.1381966011250105;   // (5 - sqrt5) / 20
    double x[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double sum = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) sum += (a == q ? qa : qb) * p[a][d];
        x[d] = sum;
    }
    double u;
    if (tg.kind == OCP_TARGET_SINE_MODES) {
        u = TABLE_ONLY ? eval_sine_dense(tg, x) : eval_sine(tg, x);
    } else if (tg.kind == OCP_TARGET_BOX) {
        u = (x[0] > tg.lo[0] && x[0] < tg.hi[0] && x[1] > tg.lo[1] && x[1] < tg.hi[1] && x[2] > tg.lo[2] &&
             x[2] < tg.hi[2])
                ? 1.0
                : 0.0;
    } else {
        const int vv[4] = {tv.x, tv.y, tv.z, tv.w};
        u = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) u += (a == q ? qa : qb) * tg.nodal[vv[a]];
    }
    const double wu = w * u;
    double f[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) f[a] = dev::group_sum<4>(wu * (a == q ? qa : qb));
    if (REC == 0) {
        if (q == 0) fe[e] = make_double4(f[0], f[1], f[2], f[3]);
        return;
    }
    double v[10], vol;
    elem_values<REC == 2>(p, ro.rho, v, vol);
    double4 out;
    if (q == 0) {
        const int4 d = make_int4(ro.dof_of_vertex[tv.x], ro.dof_of_vertex[tv.y], ro.dof_of_vertex[tv.z],
                                 ro.dof_of_vertex[tv.w]);
        ro.tdof[e] = d;
        if (REC == 2) ro.vol[e] = vol;
        out = make_double4(ints_as_double(d.x, d.y), ints_as_double(d.z, d.w), v[0], v[1]);
    } else if (q == 1) {
        out = make_double4(v[2], v[3], v[4], v[5]);
    } else if (q == 2) {
        out = make_double4(v[6], v[7], v[8], v[9]);
    } else {
        out = make_double4(f[0], f[1], f[2], f[3]);
    }
    reinterpret_cast<double4 *>(ro.rec)[4 * e + q] = out;
}

// ---------------------------------------------------------- 6. numeric rows
// One thread per row: the incident tets are visited in ascending id and the
// element values are accumulated into register slots (one per row entry,
// matched by column).  Entry (i,j) and entry (j,i) therefore add the same
// element values in the same order: the assembled A is bitwise symmetric.
// The records of U incident tets are requested before any is used.  A
// wavefront holds the 64 rows of one slice of the sliced-ELL copy, so with
// its layout given (sc) the rows are also stored there, padding included
// (column = row, value 0), by consecutive stores.
// With code given, the wavefront also builds its slice's column codes (rows
// of at most 32 entries).
struct SellOut {
    int64_t nslices = 0;
    const int32_t *sp = nullptr, *sw = nullptr;
    int32_t *col = nullptr;
    double *val = nullptr;
    const int32_t *cp = nullptr;
    uint32_t *code = nullptr;
    int32_t *dict = nullptr, *over = nullptr;
};
// Row i (lane i % 64 of slice s's wavefront) stored in the sliced-ELL copy,
// padding included (column = the row, 0 past the last row; value 0), and,
// with sc.code given, the slice's column codes built by the wavefront (every
// lane of it must be here).
template <int MAXS>
__device__ __forceinline__ void sell_store_row(const SellOut &sc, int64_t s, bool valid, int i, int len,
                                               const int (&cols)[MAXS], const double (&acc)[MAXS]) {
    const int w = sc.sw[s];   // the slice's longest row: at most MAXS
    const int64_t base = sc.sp[s] + (threadIdx.x & (kSellC - 1));
    const int pad = valid ? i : 0;
#pragma unroll
    for (int q = 0; q < MAXS; ++q)
        if (q < w) {
            sc.col[base + (int64_t)q * kSellC] = q < len ? cols[q] : pad;
            sc.val[base + (int64_t)q * kSellC] = q < len ? acc[q] : 0.0;
        }
    if constexpr (MAXS <= 32) {
        if (sc.code) {
            int d[MAXS];
#pragma unroll
            for (int q = 0; q < MAXS; ++q) d[q] = q < w ? (q < len ? cols[q] : pad) - pad : 0;
            dev::sell_code_regs<MAXS>(s, w, (int)(threadIdx.x & 63), d, sc.cp, sc.code, sc.dict, sc.over);
        }
    }
}

template <int MAXS, bool KM>
__global__ void __launch_bounds__(256) k_row_numeric(
    int32_t n, double rho, const int32_t *__restrict__ vertex_of_dof, const int32_t *__restrict__ inc_ptr,
    const int32_t *__restrict__ inc, const double *__restrict__ rec, const double *__restrict__ vol_in,
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col, double *__restrict__ val,
    double *__restrict__ valK, double *__restrict__ valM, double *__restrict__ f, SellOut sc) {
#pragma clang fp contract(off)
    const int i = blockIdx.x * 256 + (int)threadIdx.x;
    const bool valid = i < n;   // the last slice also holds padding rows
    const int64_t s = i / kSellC;
    if (!valid && (!sc.val || s >= sc.nslices)) return;
    int len = 0;
    int cols[MAXS];
    double acc[MAXS], aK[KM ? MAXS : 1], aM[KM ? MAXS : 1];
#pragma unroll
    for (int q = 0; q < MAXS; ++q) {
        cols[q] = -1;
        acc[q] = 0.0;
        if (KM) {
            aK[q] = 0.0;
            aM[q] = 0.0;
        }
    }
    if (valid) {
    const int vi = vertex_of_dof[i];
    const int rb = row_ptr[i];
    len = row_ptr[i + 1] - rb;
#pragma unroll
    for (int q = 0; q < MAXS; ++q) cols[q] = q < len ? col[rb + q] : -1;
    double fi = 0.0;
    const int qe = inc_ptr[vi + 1];
    constexpr int U = 4;
    for (int q0 = inc_ptr[vi]; q0 < qe; q0 += U) {
        int code[U];
        int4 td[U];
        double kr[U][4], vol[U], fa[U];
#pragma unroll
        for (int u = 0; u < U; ++u) code[u] = q0 + u < qe ? inc[q0 + u] : -1;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (code[u] < 0) continue;
            const int64_t e = code[u] >> 2;
            const int a = code[u] & 3;
            const double *r = rec + kRecD * e;
            td[u] = *reinterpret_cast<const int4 *>(r);
#pragma unroll
            for (int b = 0; b < 4; ++b) kr[u][b] = r[kRecVal + sym_index(a, b)];
            fa[u] = r[kRecFe + a];
            if (KM) vol[u] = vol_in[e];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (code[u] < 0) continue;
            const int a = code[u] & 3;
            fi += fa[u];
            const int dd[4] = {td[u].x, td[u].y, td[u].z, td[u].w};
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = dd[b];
                if (j < 0) continue;
                double v, kab = 0.0, mab = 0.0;
                if (KM) {
                    kab = kr[u][b];
                    mab = vol[u] / 20.0 * (b == a ? 2.0 : 1.0);
                    v = rho * kab + mab;
                } else {
                    v = kr[u][b];
                }
#pragma unroll
                for (int s2 = 0; s2 < MAXS; ++s2)
                    if (cols[s2] == j) {
                        acc[s2] += v;
                        if (KM) {
                            aK[s2] += kab;
                            aM[s2] += mab;
                        }
                    }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < MAXS; ++q)
        if (q < len) {
            val[rb + q] = acc[q];
            if (KM) {
                valK[rb + q] = aK[q];
                valM[rb + q] = aM[q];
            }
        }
    f[i] = fi;
    }
    if (sc.val) sell_store_row<MAXS>(sc, s, valid, i, len, cols, acc);
}

// Rows with at most kFuseW entries in one pass over their incident tets,
// with no element records: the row's thread recomputes, for each incident
// tet, row a of its element matrix from the vertex coordinates (a = the row's
// vertex in the tet; entry (a,b) = rho |tau| grad phi_a . grad phi_b +
// |tau|/20 (1 + delta_ab), the products and sums in the order elem_values
// uses, so the same bits), and takes the element load from fe (4 per tet;
// with fe NULL, f is zero).
// The diagonal is summed in a register; every other column gets a slot at
// its first appearance (keys in registers, sums in thread-private LDS), and
// each slot sums its values in incidence order as k_row_numeric does (so
// entry (i,j) and entry (j,i) add the same values in the same order).  The
// row is then sorted by column and written to its kFuseW-wide padded slot
// with its length.  A longer row sets bit 64 of *flag (the caller then
// assembles in separate symbolic and numeric passes).
// Reading a 128-byte element record per incident tet moved about four times
// the records' size through the L2 (each record is read by the 4 rows of its
// vertices); the tets, coordinates, dofs and loads read here are shared by
// neighbouring rows.
constexpr int kFuseW = 16;
constexpr int kFuseBlock = 256;
__global__ void __launch_bounds__(kFuseBlock) k_row_fused(int32_t n, double rho,
                                                          const int32_t *__restrict__ vertex_of_dof,
                                                          const int32_t *__restrict__ dof_of_vertex,
                                                          const int32_t *__restrict__ inc_ptr,
                                                          const int32_t *__restrict__ inc,
                                                          const int4 *__restrict__ tets,
                                                          const double *__restrict__ xyz,
                                                          const double *__restrict__ fe, int32_t *__restrict__ rlen,
                                                          int32_t *__restrict__ pcol, double *__restrict__ pval,
                                                          double *__restrict__ f, int32_t *flag) {
#pragma clang fp contract(off)
    constexpr int S = kFuseW;
    __shared__ double lacc[S][kFuseBlock];   // column s of this thread's row: lacc[s][threadIdx.x]
    const int t = (int)threadIdx.x;
    const int i = blockIdx.x * kFuseBlock + t;
    if (i >= n) return;
    const int vi = vertex_of_dof[i];
    int keys[S];   // slot 0: the diagonal (summed in dg)
    keys[0] = i;
#pragma unroll
    for (int q = 1; q < S; ++q) keys[q] = INT_MAX;
    int nk = 1;
    double fi = 0.0, dg = 0.0;
    const int qe = inc_ptr[vi + 1];
    constexpr int U = 4;   // U incident tets' data requested together
    for (int q0 = inc_ptr[vi]; q0 < qe; q0 += U) {
        int code[U];
        int4 tv[U];
        double p[U][4][3], fa[U];
        int dd[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u) code[u] = q0 + u < qe ? inc[q0 + u] : -1;
        // a missing tet (past the list's end) repeats the first one's loads
#pragma unroll
        for (int u = 0; u < U; ++u) tv[u] = tets[(code[u] < 0 ? code[0] : code[u]) >> 2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int cu = code[u] < 0 ? code[0] : code[u];
            load_tet(xyz, tv[u], p[u]);
            dd[u][0] = dof_of_vertex[tv[u].x];
            dd[u][1] = dof_of_vertex[tv[u].y];
            dd[u][2] = dof_of_vertex[tv[u].z];
            dd[u][3] = dof_of_vertex[tv[u].w];
            fa[u] = fe ? fe[4 * (int64_t)(cu >> 2) + (cu & 3)] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (code[u] < 0) continue;
            fi += fa[u];
            const int a = code[u] & 3;
            double g[4][3];
            const double det = tet_gradients(p[u], g);
            const double vol = fabs(det) / 6.0;
            double ga[3] = {g[0][0], g[0][1], g[0][2]};
#pragma unroll
            for (int a2 = 1; a2 < 4; ++a2)
                if (a == a2) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) ga[d] = g[a2][d];
                }
            double v[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const double kab = vol * (ga[0] * g[b][0] + ga[1] * g[b][1] + ga[2] * g[b][2]);
                const double mab = vol / 20.0 * (b == a ? 2.0 : 1.0);
                v[b] = rho * kab + mab;
            }
            double vd = v[0];
#pragma unroll
            for (int b = 1; b < 4; ++b)
                if (b == a) vd = v[b];
            dg += vd;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = dd[u][b];
                if (b == a || j < 0) continue;
                int idx = -1;
#pragma unroll
                for (int s2 = 1; s2 < S; ++s2) idx = keys[s2] == j ? s2 : idx;
                if (idx > 0) {
                    lacc[idx][t] += v[b];
                    continue;
                }
                if (nk == S) {
                    atomicOr(flag, 64);
                    return;
                }
#pragma unroll
                for (int s2 = 1; s2 < S; ++s2)
                    if (s2 == nk) keys[s2] = j;
                lacc[nk][t] = 0.0 + v[b];   // as the first add onto a zero slot
                ++nk;
            }
        }
    }
    double acc[S];
    acc[0] = dg;
#pragma unroll
    for (int q = 1; q < S; ++q) acc[q] = q < nk ? lacc[q][t] : 0.0;
    dev::sort_slots(keys, acc);
    // the whole slot in 16-byte stores (unused slots: INT_MAX, 0)
    const int64_t p = (int64_t)i * S;
    int4 *c4 = reinterpret_cast<int4 *>(pcol + p);
    double2 *v2 = reinterpret_cast<double2 *>(pval + p);
#pragma unroll
    for (int k = 0; k < S / 4; ++k) c4[k] = make_int4(keys[4 * k], keys[4 * k + 1], keys[4 * k + 2], keys[4 * k + 3]);
#pragma unroll
    for (int k = 0; k < S / 2; ++k) v2[k] = make_double2(acc[2 * k], acc[2 * k + 1]);
    rlen[i] = nk;
    f[i] = fi;
}

// The padded rows of k_row_fused copied to the CSR and to the sliced-ELL
// copy (with its column codes), one thread per row, a wavefront per slice.
// A wavefront's 64 rows are consecutive in the CSR: they are staged in LDS
// (columns, then values, through one buffer) and stored consecutively.
__device__ __forceinline__ void lds_wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__global__ void __launch_bounds__(256) k_row_finish(int32_t n, const int32_t *__restrict__ pcol,
                                                    const double *__restrict__ pval,
                                                    const int32_t *__restrict__ row_ptr, int32_t *__restrict__ col,
                                                    double *__restrict__ val, SellOut sc) {
    constexpr int S = kFuseW;
    __shared__ double stage[256 / kSellC][kSellC * S];
    const int i = blockIdx.x * 256 + (int)threadIdx.x;
    const bool valid = i < n;
    const int64_t s = i / kSellC;
    if (!valid && s >= sc.nslices) return;   // whole wavefronts past the last slice
    const int lane = (int)(threadIdx.x & (kSellC - 1)), wv = (int)(threadIdx.x / kSellC);
    const int i0 = i - lane;
    const int e0 = row_ptr[i0], e1 = row_ptr[i0 + kSellC < n ? i0 + kSellC : n];
    int len = 0, rb = 0, cols[S];
    double acc[S];
    if (valid) {
        rb = row_ptr[i];
        len = row_ptr[i + 1] - rb;
        // the whole padded row in 16-byte loads (slots past len are read
        // and dropped: the padded arrays hold n full rows)
        const int64_t p = (int64_t)i * S;
        const int4 *c4 = reinterpret_cast<const int4 *>(pcol + p);
        const double2 *v2 = reinterpret_cast<const double2 *>(pval + p);
        int4 cc[S / 4];
        double2 vv[S / 2];
#pragma unroll
        for (int k = 0; k < S / 4; ++k) cc[k] = c4[k];
#pragma unroll
        for (int k = 0; k < S / 2; ++k) vv[k] = v2[k];
#pragma unroll
        for (int k = 0; k < S / 4; ++k) {
            const int c[4] = {cc[k].x, cc[k].y, cc[k].z, cc[k].w};
#pragma unroll
            for (int u = 0; u < 4; ++u) cols[4 * k + u] = 4 * k + u < len ? c[u] : -1;
        }
#pragma unroll
        for (int k = 0; k < S / 2; ++k) {
            acc[2 * k] = 2 * k < len ? vv[k].x : 0.0;
            acc[2 * k + 1] = 2 * k + 1 < len ? vv[k].y : 0.0;
        }
    } else {
#pragma unroll
        for (int q = 0; q < S; ++q) {
            cols[q] = -1;
            acc[q] = 0.0;
        }
    }
    // CSR: columns, then values, staged per wavefront and stored consecutively
    int *sc32 = reinterpret_cast<int *>(&stage[wv][0]);
#pragma unroll
    for (int q = 0; q < S; ++q)
        if (q < len) sc32[rb - e0 + q] = cols[q];
    lds_wave_fence();
    for (int t = lane; t < e1 - e0; t += kSellC) col[e0 + t] = sc32[t];
    lds_wave_fence();
#pragma unroll
    for (int q = 0; q < S; ++q)
        if (q < len) stage[wv][rb - e0 + q] = acc[q];
    lds_wave_fence();
    for (int t = lane; t < e1 - e0; t += kSellC) val[e0 + t] = stage[wv][t];
    sell_store_row<S>(sc, s, valid, i, len, cols, acc);
}

template <int MAXS>
static void launch_numeric(ocp_ctx *ctx, ocp_system *sys, double rho, const double *rec, const double *vol,
                           const SellOut &sc) {
    const unsigned g = grid_for(sys->n, 256);
    if (sys->valK.get())
        k_row_numeric<MAXS, true><<<g, 256, 0, ctx->stream>>>(
            sys->n, rho, sys->vertex_of_dof.get(), sys->inc_ptr.get(), sys->inc.get(), rec, vol, sys->row_ptr.get(),
            sys->col.get(), sys->val.get(), sys->valK.get(), sys->valM.get(), sys->f.get(), sc);
    else
        k_row_numeric<MAXS, false><<<g, 256, 0, ctx->stream>>>(
            sys->n, rho, sys->vertex_of_dof.get(), sys->inc_ptr.get(), sys->inc.get(), rec, nullptr,
            sys->row_ptr.get(), sys->col.get(), sys->val.get(), nullptr, nullptr, sys->f.get(), sc);
    OCP_LAUNCH_CHECK();
}

__global__ void k_set_rho(int64_t nnz, double rho, const double *__restrict__ valK,
                          const double *__restrict__ valM, double *__restrict__ val) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s < nnz) val[s] = rho * valK[s] + valM[s];
}

// -------------------------------------------------------------- host side
static void check_target(const ocp_target *t, int32_t nv) {
    if (!t) fail(OCP_ERR_INVALID_ARG, "target is NULL");
    if (t->kind == OCP_TARGET_SINE_MODES) {
        if (t->n_modes < 1 || t->n_modes > 4096 || !t->k || !t->amp)
            fail(OCP_ERR_INVALID_ARG, "sine-mode target needs 1..4096 modes with k and amp");
        for (int m = 0; m < t->n_modes; ++m) {
            for (int d = 0; d < 3; ++d)
                if (t->k[3 * m + d] < 1 || t->k[3 * m + d] > 1024)
                    fail(OCP_ERR_INVALID_ARG, "wave numbers must lie in 1..1024");
            if (!std::isfinite(t->amp[m])) fail(OCP_ERR_INVALID_ARG, "non-finite amplitude");
        }
        if (!std::isfinite(t->offset)) fail(OCP_ERR_INVALID_ARG, "non-finite offset");
    } else if (t->kind == OCP_TARGET_BOX) {
        for (int d = 0; d < 3; ++d)
            if (!std::isfinite(t->lo[d]) || !std::isfinite(t->hi[d]))
                fail(OCP_ERR_INVALID_ARG, "non-finite box bounds");
    } else if (t->kind == OCP_TARGET_NODAL) {
        if (!t->nodal) fail(OCP_ERR_INVALID_ARG, "nodal target needs device values");
    } else {
        fail(OCP_ERR_INVALID_ARG, "unknown target kind");
    }
    (void)nv;
}

// Upload the target description; the returned buffers must outlive the launch.
struct TargetUpload {
    DevBuf<SineMode> modes;
    DevBuf<double> dense;
    bool table_only = true;   // every wave number <= kSineTable
    TargetDev dev{};
};

static void upload_target(ocp_ctx *ctx, const ocp_target *t, TargetUpload &up) {
    up.dev.kind = t->kind;
    up.dev.offset = t->offset;
    for (int d = 0; d < 3; ++d) {
        up.dev.lo[d] = t->lo[d];
        up.dev.hi[d] = t->hi[d];
    }
    up.dev.nodal = t->nodal;
    if (t->kind == OCP_TARGET_SINE_MODES) {
        const int m = t->n_modes;
        for (int q = 0; q < 3 * m; ++q) up.table_only = up.table_only && t->k[q] <= kSineTable;
        if (up.table_only) {
            constexpr int T = kSineTable;
            std::vector<double> a((size_t)T * T * T, 0.0);
            uint64_t pairs = 0;
            for (int q = 0; q < m; ++q) {
                const int k1 = t->k[3 * q] - 1, k2 = t->k[3 * q + 1] - 1, k3 = t->k[3 * q + 2] - 1;
                a[((size_t)k1 * T + k2) * T + k3] += t->amp[q];
                pairs |= uint64_t(1) << (k1 * T + k2);
            }
            up.dense.reset(ctx, a.size());
            OCP_HIP(hipMemcpyAsync(up.dense.get(), a.data(), sizeof(double) * a.size(), hipMemcpyHostToDevice,
                                   ctx->stream));
            up.dev.dense = up.dense.get();
            up.dev.pairs = pairs;
            up.dev.n_modes = 0;
            up.dev.modes = nullptr;
            sync(ctx);  // the staging vector is released when this returns
            return;
        }
        const int mp = (m + kModeBatch - 1) / kModeBatch * kModeBatch;
        std::vector<SineMode> md((size_t)mp);
        for (int q = 0; q < mp; ++q) {
            SineMode &o = md[q];
            o.pad = 0;
            o.pad2 = 0.0;
            if (q < m) {
                for (int d = 0; d < 3; ++d) o.k[d] = t->k[3 * q + d];
                o.amp = t->amp[q];
            } else {   // padding: contributes amp * (...) = 0
                o.k[0] = o.k[1] = o.k[2] = 1;
                o.amp = 0.0;
            }
        }
        up.modes.reset(ctx, (size_t)mp);
        OCP_HIP(hipMemcpyAsync(up.modes.get(), md.data(), sizeof(SineMode) * mp, hipMemcpyHostToDevice, ctx->stream));
        up.dev.n_modes = mp;
        up.dev.modes = up.modes.get();
        sync(ctx);  // the staging vector is released when this returns
    }
}

// element loads of every tet to fe[e]; with rec set (RecOut::rec), the
// element records instead (REC 1, or 2 with ro.vol for separate K and M)
static void launch_tet_load(ocp_ctx *ctx, const TargetUpload &up, const int4 *tets, int64_t nt, const double *xyz,
                            double4 *fe, const RecOut &ro = RecOut{}) {
    const unsigned g = grid_for(nt * 4, kLoadBlock);
    const int rec = ro.rec ? (ro.vol ? 2 : 1) : 0;
    auto go = [&](auto table_only) {
        constexpr bool TO = decltype(table_only)::value;
        if (rec == 0)
            k_tet_load<TO, 0><<<g, kLoadBlock, 0, ctx->stream>>>(tets, nt, xyz, up.dev, fe, ro);
        else if (rec == 1)
            k_tet_load<TO, 1><<<g, kLoadBlock, 0, ctx->stream>>>(tets, nt, xyz, up.dev, fe, ro);
        else
            k_tet_load<TO, 2><<<g, kLoadBlock, 0, ctx->stream>>>(tets, nt, xyz, up.dev, fe, ro);
    };
    if (up.table_only)
        go(std::true_type{});
    else
        go(std::false_type{});
    OCP_LAUNCH_CHECK();
}

static void compute_loads(ocp_ctx *ctx, const ocp_system *sys, const ocp_mesh *mesh, const ocp_target *t,
                          double *f_out, int64_t ld = 1) {
    TargetUpload up;
    upload_target(ctx, t, up);
    DevBuf<double4> fe(ctx, (size_t)sys->nt);
    const int4 *tets = reinterpret_cast<const int4 *>(mesh->tets);
    launch_tet_load(ctx, up, tets, sys->nt, mesh->xyz, fe.get());
    // row sums of the element loads (reuse the numeric kernel's f output
    // through a dedicated pass that only accumulates f)
    extern void row_loads(ocp_ctx *, const ocp_system *, const double4 *, double *, int64_t);
    row_loads(ctx, sys, fe.get(), f_out, ld);
    sync(ctx);
}

__global__ void __launch_bounds__(kAsmBlock) k_row_loads(int32_t n, const int32_t *__restrict__ vertex_of_dof,
                                                         const int32_t *__restrict__ inc_ptr,
                                                         const int32_t *__restrict__ inc,
                                                         const double *__restrict__ fe, double *__restrict__ f,
                                                         int64_t ld) {
    const int i = blockIdx.x * kAsmBlock + threadIdx.x;
    if (i >= n) return;
    const int vi = vertex_of_dof[i];
    double fi = 0.0;
    int q = inc_ptr[vi];
    const int qe = inc_ptr[vi + 1];
    // eight incident tets at a time: their codes, then their element loads
    // at this vertex, are all requested before any is used (the sum keeps
    // list order)
    constexpr int U = 8;
    for (; q + U <= qe; q += U) {
        int code[U];
        double fv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) code[u] = inc[q + u];
#pragma unroll
        for (int u = 0; u < U; ++u) fv[u] = fe[4 * (int64_t)(code[u] >> 2) + (code[u] & 3)];
#pragma unroll
        for (int u = 0; u < U; ++u) fi += fv[u];
    }
    for (; q < qe; ++q) {
        const int code = inc[q];
        fi += fe[4 * (int64_t)(code >> 2) + (code & 3)];
    }
    f[(int64_t)i * ld] = fi;
}

// f[i * ld] = sum over the tets of row i of their element load at its vertex
void row_loads(ocp_ctx *ctx, const ocp_system *sys, const double4 *fe, double *f, int64_t ld) {
    k_row_loads<<<grid_for(sys->n, kAsmBlock), kAsmBlock, 0, ctx->stream>>>(
        sys->n, sys->vertex_of_dof.get(), sys->inc_ptr.get(), sys->inc.get(), reinterpret_cast<const double *>(fe),
        f, ld);
    OCP_LAUNCH_CHECK();
}

__global__ void k_row_lengths(int32_t n, const int32_t *__restrict__ rp, double *__restrict__ len) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) len[i] = (double)(rp[i + 1] - rp[i]);
}

// longest row of the assembled pattern (cached on the system)
static int max_row_len(ocp_ctx *ctx, ocp_system *sys) {
    if (sys->max_row_len < 0) {
        DevBuf<double> len(ctx, (size_t)sys->n);
        k_row_lengths<<<grid_for(sys->n, 256), 256, 0, ctx->stream>>>(sys->n, sys->row_ptr.get(), len.get());
        OCP_LAUNCH_CHECK();
        sys->max_row_len = (int)reduce_max_abs(ctx, len.get(), sys->n);
    }
    return sys->max_row_len;
}

static void assemble(ocp_ctx *ctx, const ocp_mesh *mesh, double rho, const ocp_target *t, int32_t flags,
                     ocp_system *sys) {
    const int32_t nv = mesh->n_vertices;
    const int64_t nt = mesh->n_tets;
    sys->nv = nv;
    sys->nt = nt;
    sys->rho = rho;
    sys->tets_ref = mesh->tets;
    sys->mesh = *mesh;
    const int4 *tets = reinterpret_cast<const int4 *>(mesh->tets);
    if (reinterpret_cast<uintptr_t>(mesh->tets) % 16 != 0)
        fail(OCP_ERR_INVALID_ARG, "tets must be 16-byte aligned");

    // 1. checks and incidence counts
    DevBuf<int32_t> cnt(ctx, (size_t)nv + 1);
    fill_zero_bytes(ctx, cnt.get(), sizeof(int32_t) * ((size_t)nv + 1));
    fill_zero_bytes(ctx, ctx->dev_flag, sizeof(int32_t));
    k_tet_check_count<<<grid_for(nt, kIncBlock), kIncBlock, 0, ctx->stream>>>(tets, nt, mesh->xyz, nv, cnt.get(),
                                                                              ctx->dev_flag);
    OCP_LAUNCH_CHECK();
    int32_t fl = 0;
    read_back(ctx, &fl, ctx->dev_flag, sizeof(fl));
    if (fl & 1) fail(OCP_ERR_BAD_MESH, "tet vertex index out of range");
    if (fl & 2) fail(OCP_ERR_BAD_MESH, "degenerate tetrahedron (|det| <= 1e-12 * longest edge^3)");

    // 2. incidence lists
    sys->inc_ptr.reset(ctx, (size_t)nv + 1);
    const int64_t ninc = scan_exclusive(ctx, cnt.get(), sys->inc_ptr.get(), nv);
    sys->inc.reset(ctx, (size_t)ninc);
    fill_zero_bytes(ctx, cnt.get(), sizeof(int32_t) * (size_t)nv);
    k_tet_fill<<<grid_for(nt, kIncBlock), kIncBlock, 0, ctx->stream>>>(tets, nt, sys->inc_ptr.get(), cnt.get(),
                                                                       sys->inc.get());
    OCP_LAUNCH_CHECK();
    k_inc_sort<<<grid_for(nv, 64), 64, 0, ctx->stream>>>(sys->inc_ptr.get(), sys->inc.get(), nv);
    OCP_LAUNCH_CHECK();

    // 3. dof numbering
    k_interior_flags<<<grid_for(nv, 256), 256, 0, ctx->stream>>>(mesh->dirichlet, nv, cnt.get());
    OCP_LAUNCH_CHECK();
    DevBuf<int32_t> pos(ctx, (size_t)nv + 1);
    const int64_t n = scan_exclusive(ctx, cnt.get(), pos.get(), nv);
    if (n < 1) fail(OCP_ERR_BAD_MESH, "mesh has no interior vertex");
    sys->n = (int32_t)n;
    sys->dof_of_vertex.reset(ctx, (size_t)nv);
    sys->vertex_of_dof.reset(ctx, (size_t)n);
    k_dof_maps<<<grid_for(nv, 256), 256, 0, ctx->stream>>>(mesh->dirichlet, pos.get(), nv, sys->dof_of_vertex.get(),
                                                           sys->vertex_of_dof.get());
    OCP_LAUNCH_CHECK();
    pos.release();

    // 4-6. With K and M not kept apart, rows of at most kFuseW entries are
    // assembled in one pass over the tets' element loads (fe, one pass over
    // the tets) and their geometry: columns are found while the values are
    // summed.  Otherwise, or if a row is longer, every tet writes its element
    // record (dofs, element matrix, element loads), then symbolic rows and
    // numeric rows read the records.
    const bool km = (flags & OCP_KEEP_KM) != 0;
    const bool noload = (flags & OCP_NO_LOAD) != 0;
    // without loads, the record route evaluates an empty box (every load 0)
    ocp_target empty_box{};
    empty_box.kind = OCP_TARGET_BOX;
    TargetUpload up;
    upload_target(ctx, noload ? &empty_box : t, up);
    bool fused = false;
    if (!km) {
        DevBuf<double4> fe;
        if (!noload) {
            fe.reset(ctx, (size_t)nt);
            launch_tet_load(ctx, up, tets, nt, mesh->xyz, fe.get());
        }
        DevBuf<int32_t> rlen(ctx, (size_t)n + 1);
        DevBuf<int32_t> pcol(ctx, (size_t)n * kFuseW);
        DevBuf<double> pval(ctx, (size_t)n * kFuseW);
        sys->f.reset(ctx, (size_t)n);
        fill_zero_bytes(ctx, ctx->dev_flag, sizeof(int32_t));
        k_row_fused<<<grid_for(n, kFuseBlock), kFuseBlock, 0, ctx->stream>>>(
            n, rho, sys->vertex_of_dof.get(), sys->dof_of_vertex.get(), sys->inc_ptr.get(), sys->inc.get(), tets,
            mesh->xyz, noload ? nullptr : reinterpret_cast<const double *>(fe.get()), rlen.get(), pcol.get(),
            pval.get(), sys->f.get(),
            ctx->dev_flag);
        OCP_LAUNCH_CHECK();
        read_back(ctx, &fl, ctx->dev_flag, sizeof(fl));
        if (!(fl & 64)) {
            fused = true;
            fe.release();
            sys->row_ptr.reset(ctx, (size_t)n + 1);
            sys->nnz = scan_exclusive(ctx, rlen.get(), sys->row_ptr.get(), n);
            sys->col.reset(ctx, (size_t)sys->nnz);
            sys->val.reset(ctx, (size_t)sys->nnz);
            sell_layout(ctx, sys->sell, n, sys->row_ptr.get());
            sell_code_layout(ctx, sys->sell);
            SellOut sc;
            sc.nslices = sys->sell.nslices;
            sc.sp = sys->sell.sp.get();
            sc.sw = sys->sell.sw.get();
            sc.col = sys->sell.col.get();
            sc.val = sys->sell.val.get();
            sc.cp = sys->sell.cp.get();
            sc.code = sys->sell.code.get();
            sc.dict = sys->sell.dict.get();
            sc.over = ctx->dev_flag;
            k_row_finish<<<grid_for(n, 256), 256, 0, ctx->stream>>>(n, pcol.get(), pval.get(), sys->row_ptr.get(),
                                                                   sys->col.get(), sys->val.get(), sc);
            OCP_LAUNCH_CHECK();
            sell_code_finish(ctx, sys->sell);
        }
    }
    if (!fused) {
        // 4. element records and the compact vertex dofs of every tet
        DevBuf<double> rec(ctx, (size_t)kRecD * nt);
        DevBuf<double> vol;
        if (km) vol.reset(ctx, (size_t)nt);
        DevBuf<int4> tdof(ctx, (size_t)nt);
        launch_tet_load(ctx, up, tets, nt, mesh->xyz, nullptr,
                        RecOut{sys->dof_of_vertex.get(), rho, rec.get(), vol.get(), tdof.get()});
        // 5. symbolic rows: rows of up to kPadW entries in one pass into a padded
        // buffer; if any row is longer, count and fill again with kRowCap slots
        DevBuf<int32_t> rcnt(ctx, (size_t)n + 1);
        DevBuf<int32_t> pad(ctx, (size_t)n * kPadW);
        fill_zero_bytes(ctx, ctx->dev_flag, sizeof(int32_t));
        k_row_symbolic<kPadW><<<grid_for(n, kAsmBlock), kAsmBlock, 0, ctx->stream>>>(
            0, sys->n, sys->vertex_of_dof.get(), sys->inc_ptr.get(), sys->inc.get(), tdof.get(), rcnt.get(), nullptr,
            nullptr, pad.get(), ctx->dev_flag);
        OCP_LAUNCH_CHECK();
        read_back(ctx, &fl, ctx->dev_flag, sizeof(fl));
        const bool long_rows = (fl & 128) != 0;
        if (long_rows) {
            pad.release();
            fill_zero_bytes(ctx, ctx->dev_flag, sizeof(int32_t));
            k_row_symbolic<kRowCap><<<grid_for(n, kAsmBlock), kAsmBlock, 0, ctx->stream>>>(
                0, sys->n, sys->vertex_of_dof.get(), sys->inc_ptr.get(), sys->inc.get(), tdof.get(), rcnt.get(), nullptr,
                nullptr, nullptr, ctx->dev_flag);
            OCP_LAUNCH_CHECK();
            read_back(ctx, &fl, ctx->dev_flag, sizeof(fl));
            if (fl & 4) fail(OCP_ERR_UNSUPPORTED, "an assembled row has more than 128 entries");
        }
        sys->row_ptr.reset(ctx, (size_t)n + 1);
        sys->nnz = scan_exclusive(ctx, rcnt.get(), sys->row_ptr.get(), n);
        sys->col.reset(ctx, (size_t)sys->nnz);
        if (long_rows) {
            k_row_symbolic<kRowCap><<<grid_for(n, kAsmBlock), kAsmBlock, 0, ctx->stream>>>(
                1, sys->n, sys->vertex_of_dof.get(), sys->inc_ptr.get(), sys->inc.get(), tdof.get(), nullptr,
                sys->row_ptr.get(), sys->col.get(), nullptr, ctx->dev_flag);
        } else {
            k_pad_to_csr<<<grid_for((int64_t)n * kPadLanes, 256), 256, 0, ctx->stream>>>(
                sys->n, pad.get(), sys->row_ptr.get(), sys->col.get());
        }
        OCP_LAUNCH_CHECK();
        pad.release();
        const int maxlen = long_rows ? kRowCap : kPadW;
        rcnt.release();

        tdof.release();

        // 6. numeric rows
        sys->val.reset(ctx, (size_t)sys->nnz);
        sys->f.reset(ctx, (size_t)n);
        if (km) {
            sys->valK.reset(ctx, (size_t)sys->nnz);
            sys->valM.reset(ctx, (size_t)sys->nnz);
        }
        // the rows go to the CSR and to the sliced-ELL copy for the solve phase
        sell_layout(ctx, sys->sell, n, sys->row_ptr.get());
        SellOut sc;
        sc.nslices = sys->sell.nslices;
        sc.sp = sys->sell.sp.get();
        sc.sw = sys->sell.sw.get();
        sc.col = sys->sell.col.get();
        sc.val = sys->sell.val.get();
        const int ml = maxlen <= 16 ? 16 : max_row_len(ctx, sys);
        const int ms = ml <= 16 ? 16 : ml <= 32 ? 32 : ml <= 64 ? 64 : 128;
        if (ms <= 32) {   // column codes built by the same wavefronts
            sell_code_layout(ctx, sys->sell);
            sc.cp = sys->sell.cp.get();
            sc.code = sys->sell.code.get();
            sc.dict = sys->sell.dict.get();
            sc.over = ctx->dev_flag;
        }
        if (ms == 16)
            launch_numeric<16>(ctx, sys, rho, rec.get(), vol.get(), sc);
        else if (ms == 32)
            launch_numeric<32>(ctx, sys, rho, rec.get(), vol.get(), sc);
        else if (ms == 64)
            launch_numeric<64>(ctx, sys, rho, rec.get(), vol.get(), sc);
        else
            launch_numeric<128>(ctx, sys, rho, rec.get(), vol.get(), sc);
        OCP_LAUNCH_CHECK();
        if (ms <= 32)
            sell_code_finish(ctx, sys->sell);
        else
            sell_codes(ctx, sys->sell);
    }
    sync(ctx);
}

}  // namespace ocp

using namespace ocp;

extern "C" int fe_assemble(ocp_ctx *ctx, const ocp_mesh *mesh, double rho, const ocp_target *target,
                           int32_t flags, ocp_system **out) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    if (out) *out = nullptr;
    ocp_system *sys = nullptr;
    int rc = run_guarded(ctx, [&] {
        if (!mesh || !out) fail(OCP_ERR_INVALID_ARG, "mesh and out must not be NULL");
        if (mesh->n_vertices <= 0 || mesh->n_tets <= 0 || !mesh->xyz || !mesh->tets || !mesh->dirichlet)
            fail(OCP_ERR_INVALID_ARG, "mesh needs positive counts and xyz, tets, dirichlet arrays");
        if ((int64_t)mesh->n_tets * 4 > INT32_MAX) fail(OCP_ERR_UNSUPPORTED, "more than 2^29 tetrahedra");
        if (!(rho > 0.0) || !std::isfinite(rho)) fail(OCP_ERR_INVALID_ARG, "rho must be positive and finite");
        if (!(flags & OCP_NO_LOAD)) check_target(target, mesh->n_vertices);
        sys = new ocp_system();
        sys->ctx = ctx;
        assemble(ctx, mesh, rho, target, flags, sys);
    });
    if (rc != OCP_OK) {
        delete sys;
        return rc;
    }
    *out = sys;
    return OCP_OK;
}

extern "C" void ocp_system_destroy(ocp_system *sys) { delete sys; }

extern "C" int fe_derive(ocp_ctx *ctx, const ocp_system *base, double rho, ocp_system **out) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    if (out) *out = nullptr;
    ocp_system *sys = nullptr;
    int rc = run_guarded(ctx, [&] {
        if (!base || !out) fail(OCP_ERR_INVALID_ARG, "base and out must not be NULL");
        if (!(rho > 0.0) || !std::isfinite(rho)) fail(OCP_ERR_INVALID_ARG, "rho must be positive and finite");
        if (!base->valK.get()) fail(OCP_ERR_INVALID_ARG, "base system was assembled without OCP_KEEP_KM");
        sys = new ocp_system();
        sys->ctx = ctx;
        sys->nv = base->nv;
        sys->n = base->n;
        sys->nt = base->nt;
        sys->nnz = base->nnz;
        sys->rho = rho;
        sys->max_row_len = base->max_row_len;
        sys->tets_ref = base->tets_ref;
        sys->mesh = base->mesh;
        auto dup = [&](auto &dst, const auto &src) {
            using T = std::remove_pointer_t<decltype(src.get())>;
            dst.reset(ctx, src.size());
            if (src.size())
                OCP_HIP(hipMemcpyAsync(dst.get(), src.get(), sizeof(T) * src.size(), hipMemcpyDeviceToDevice,
                                       ctx->stream));
        };
        dup(sys->inc_ptr, base->inc_ptr);
        dup(sys->inc, base->inc);
        dup(sys->dof_of_vertex, base->dof_of_vertex);
        dup(sys->vertex_of_dof, base->vertex_of_dof);
        dup(sys->row_ptr, base->row_ptr);
        dup(sys->col, base->col);
        dup(sys->f, base->f);
        sys->val.reset(ctx, (size_t)sys->nnz);
        k_set_rho<<<grid_for(sys->nnz, 256), 256, 0, ctx->stream>>>(sys->nnz, rho, base->valK.get(),
                                                                    base->valM.get(), sys->val.get());
        OCP_LAUNCH_CHECK();
        sell_build(ctx, sys->sell, sys->n, sys->row_ptr.get(), sys->col.get(), sys->val.get());
        sync(ctx);
    });
    if (rc != OCP_OK) {
        delete sys;
        return rc;
    }
    *out = sys;
    return OCP_OK;
}

extern "C" int fe_set_rho(ocp_ctx *ctx, ocp_system *sys, double rho) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    return run_guarded(ctx, [&] {
        if (!sys) fail(OCP_ERR_INVALID_ARG, "system is NULL");
        if (!(rho > 0.0) || !std::isfinite(rho)) fail(OCP_ERR_INVALID_ARG, "rho must be positive and finite");
        if (!sys->valK.get()) fail(OCP_ERR_INVALID_ARG, "system was assembled without OCP_KEEP_KM");
        k_set_rho<<<grid_for(sys->nnz, 256), 256, 0, ctx->stream>>>(sys->nnz, rho, sys->valK.get(), sys->valM.get(),
                                                                    sys->val.get());
        OCP_LAUNCH_CHECK();
        sys->rho = rho;
        // derived data of the old values: dropped and rebuilt (no solve may
        // use the system meanwhile); hierarchies built on it become stale
        {
            std::lock_guard<std::mutex> lock(sys->derived_mu);
            sys->dinv_ready.store(false, std::memory_order_release);
            sys->dinv.release();
        }
        sys->sell = Sell();
        sell_build(ctx, sys->sell, sys->n, sys->row_ptr.get(), sys->col.get(), sys->val.get());
        sys->generation.fetch_add(1, std::memory_order_acq_rel);
        sync(ctx);
    });
}

extern "C" int fe_load(ocp_ctx *ctx, const ocp_system *sys, const ocp_target *target, double *f_dev) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    return run_guarded(ctx, [&] {
        if (!sys || !f_dev) fail(OCP_ERR_INVALID_ARG, "system and f must not be NULL");
        check_target(target, sys->nv);
        compute_loads(ctx, sys, &sys->mesh, target, f_dev);
    });
}

extern "C" int fe_load_multi(ocp_ctx *ctx, const ocp_system *sys, int32_t k, const ocp_target *targets, double *F) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    return run_guarded(ctx, [&] {
        if (!sys || !targets || !F) fail(OCP_ERR_INVALID_ARG, "system, targets and F must not be NULL");
        if (k < 1) fail(OCP_ERR_INVALID_ARG, "k must be >= 1");
        for (int j = 0; j < k; ++j) check_target(&targets[j], sys->nv);
        for (int j = 0; j < k; ++j) compute_loads(ctx, sys, &sys->mesh, &targets[j], F + j, k);
    });
}

extern "C" int ocp_system_get_view(const ocp_system *sys, ocp_system_view *v) {
    if (!sys || !v) return OCP_ERR_INVALID_ARG;
    v->n_vertices = sys->nv;
    v->n_dofs = sys->n;
    v->nnz = sys->nnz;
    v->rho = sys->rho;
    v->row_ptr = sys->row_ptr.get();
    v->col = sys->col.get();
    v->val = sys->val.get();
    v->f = sys->f.get();
    v->dof_of_vertex = sys->dof_of_vertex.get();
    v->vertex_of_dof = sys->vertex_of_dof.get();
    v->sell_coded = sys->sell.code.get() ? 1 : 0;
    v->sell_entries = sys->sell.nnz_padded;
    return OCP_OK;
}
