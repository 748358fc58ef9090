// Smoothed-aggregation AMG setup on the GPU.
//
// Section 3.1 builds the coarse space from a greedy colouring of the matrix
// graph (pick an unmarked dof as coarse, mark its neighbours fine, repeat),
// interpolates by averaging, and forms Galerkin coarse operators
// A_c = P^T A P recursively.  Here the same three ingredients are realised as
// smoothed aggregation:
//
//   strength   j ~ i  if  |a_ij| >= theta * sqrt(a_ii a_jj), a_ij != 0;
//              theta = 0 (the default) makes every off-diagonal entry of
//              the pattern strong
//   coarsening roots = a maximal distance-2 independent set of the strength
//              graph, chosen greedily in the order of a fixed hash priority
//              (the parallel rounds below select exactly the set the
//              sequential greedy pass in that order selects); every node
//              joins the aggregate of an adjacent root, else of an adjacent
//              node that did
//   P_tent     one entry per row, 1/sqrt(|aggregate|) (constant near-kernel)
//   P          (I - omega/lambda D^-1 A) P_tent, lambda = Gershgorin bound of
//              D^-1 A (max_i sum_j |a_ij| / a_ii)
//   R = P^T,   A_c = R (A P)
//
// Every step is deterministic: integer atomics only count, lists filled in
// arbitrary order are sorted, and the sparse products accumulate each output
// entry in a fixed order.  The last level (n <= coarse_max) is inverted
// densely with Gauss-Jordan elimination in one workgroup.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>

#include "kernels.h"
#include "system.h"

namespace ocp {

constexpr int kDenseMax = 2048;

// ------------------------------------------------------------------ hashing
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// MIS key: class (in=3 > undecided=2 > out=1), 30-bit priority, node id
__device__ __forceinline__ uint64_t mis_key(int i, int8_t state, uint32_t salt) {
    const uint64_t cls = state == 1 ? 3u : (state == 0 ? 2u : 1u);
    const uint64_t pr = mix32((uint32_t)i ^ salt) >> 2;
    return (cls << 62) | (pr << 32) | (uint32_t)i;
}

// ------------------------------------------------------------- diagnostics
// diag[i] = a_ii, dl1[i] = 1 / sum_j |a_ij|, gersh[i] = sum_j |a_ij| / a_ii
__global__ void k_level_diag(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                             const double *__restrict__ val, double *__restrict__ diag, double *__restrict__ dl1,
                             double *__restrict__ gersh, int32_t *flag) {
    // XCD x takes a contiguous run of blocks (measured faster here)
    const int i = (int)dev::xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0, s = 0.0;
    int k = rp[i];
    const int e = rp[i + 1];
    // eight entries' loads in flight before any is used (same summation order)
    constexpr int U = 8;
    for (; k + U <= e; k += U) {
        double v[U];
        int c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            v[u] = val[k + u];
            c[u] = col[k + u];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s += fabs(v[u]);
            if (c[u] == i) d = v[u];
        }
    }
    for (; k < e; ++k) {
        const double v = val[k];
        s += fabs(v);
        if (col[k] == i) d = v;
    }
    if (!(d > 0.0) || !isfinite(s)) {
        atomicOr(flag, 8);
        d = 1.0;
        s = 1.0;
    }
    diag[i] = d;
    dl1[i] = 1.0 / s;
    gersh[i] = s / d;
}

__global__ void k_recip(int32_t n, const double *__restrict__ a, double *__restrict__ b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = 1.0 / a[i];
}

__global__ void k_strength(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const double *__restrict__ val, const double *__restrict__ diag, double theta,
                           uint8_t *__restrict__ strong) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double di = diag[i];
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const int j = col[k];
        const double a = fabs(val[k]);
        strong[k] = (j != i && a > 0.0 && a >= theta * sqrt(di * diag[j])) ? 1 : 0;
    }
}

// Strength flag of entry k (column j) of row i; with theta = 0 there is no
// flag array and every off-diagonal entry of the pattern is strong.
__device__ __forceinline__ bool is_strong(const uint8_t *__restrict__ strong, int k, int j, int i) {
    return strong ? strong[k] != 0 : j != i;
}

// The same on the system's sliced-ELL copy (level 0): one wavefront per 64-row
// slice, coalesced loads.  Entries are taken in row order and the padding
// (value 0) only adds zeros, so the results are the CSR kernel's bits; the
// diagonal is the entry in column row with a nonzero value (padding sits in
// column row with value 0).
__global__ void __launch_bounds__(kBlock) k_level_diag_sell(int32_t n, int64_t nslices, int spb,
                                                            const int32_t *__restrict__ sp,
                                                            const int32_t *__restrict__ sw, SellCols cols,
                                                            const double *__restrict__ val, double *__restrict__ diag,
                                                            double *__restrict__ dl1, double *__restrict__ gersh,
                                                            int32_t *flag) {
    OCP_SELL_BEGIN(nslices, spb)
    const int ww = __builtin_amdgcn_readfirstlane(w);
    const int rr = row < n ? row : 0;
    const int dl = cols.code ? cols.dict[slice * kSellDict + (lane & (kSellDict - 1))] : 0;
    const int64_t cb = cols.code ? cols.cp[slice] + lane : 0;
    double d = 0.0, sum = 0.0;
    for (int j0 = 0; j0 < ww; j0 += kSellChunk) {
        double v[kSellChunk];
        int c[kSellChunk];
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) {
            const int jj = j0 + j < ww ? j0 + j : ww - 1;
            v[j] = val[base + (int64_t)jj * kSellC];
            if (cols.code) {
                const uint32_t word = cols.code[cb + (int64_t)(jj >> 3) * kSellC];
                c[j] = rr + __shfl(dl, (int)((word >> (4 * (jj & 7))) & 15u), 64);
            } else {
                c[j] = cols.col[base + (int64_t)jj * kSellC];
            }
        }
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j)
            if (j0 + j < ww) {
                sum += fabs(v[j]);
                if (c[j] == row && v[j] != 0.0) d = v[j];
            }
    }
    if (row < n) {
        if (!(d > 0.0) || !isfinite(sum)) {
            atomicOr(flag, 8);
            d = 1.0;
            sum = 1.0;
        }
        diag[row] = d;
        dl1[row] = 1.0 / sum;
        gersh[row] = sum / d;
    }
    OCP_SELL_END()
}

// ------------------------------------------------------------------- MIS-2
// Round of the distance-2 independent set, G lanes per row:
//   m1[i] = max key over i and its strong neighbours
//   m2    = max m1 over i and its strong neighbours; an undecided i joins
//           if m2 is its own key and leaves if m2 belongs to a joined node.
template <int G>
__device__ __forceinline__ uint64_t group_max_u64(uint64_t v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) {
        const uint64_t w = __shfl_xor(v, o, G);
        v = w > v ? w : v;
    }
    return v;
}

// FIRST: every node undecided (the first round), no states read.
// Rounds only touch what can still change: m2 skips decided nodes, and from
// round kMisMarkFrom + 1 on m1 is recomputed only for nodes marked (need[i]
// == round) as the closed neighbourhood of an undecided node.
constexpr int kMisMarkFrom = 5;   // first round whose m2 marks
constexpr int kMisMaxRounds = 1024;
// list the undecided nodes at the first host check after round kMisListFrom
// when they are at most n / kMisListFrac (levels of kMisListMinN nodes or more)
constexpr int kMisListFrom = 4;
constexpr int kMisListFrac = 64;
constexpr int kMisListMinN = 1 << 16;
template <int G, bool FIRST>
__global__ void __launch_bounds__(256) k_mis_m1(int32_t n, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ col, const uint8_t *__restrict__ strong,
                                                const int8_t *__restrict__ state, uint32_t salt,
                                                const int32_t *__restrict__ need, int32_t round,
                                                const int32_t *__restrict__ prev_undecided,
                                                uint64_t *__restrict__ m1) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / G), lane = (int)(t % G);
    if (i >= n) return;
    if (prev_undecided && *prev_undecided == 0) return;   // every node decided in an earlier round
    if (need && need[i] != round) return;   // uniform over the group
    uint64_t m = 0;
    const int ke = rp[i + 1];
    // U of this lane's entries at a time: columns, then their states, all
    // requested before any is used
    constexpr int U = 4;
    for (int k0 = rp[i] + lane; k0 < ke; k0 += U * G) {
        int j[U];
        int8_t st[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * G < ke) j[u] = col[k0 + u * G];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * G < ke) st[u] = FIRST ? (int8_t)0 : state[j[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * G;
            if (k < ke && is_strong(strong, k, j[u], i)) {
                const uint64_t kj = mis_key(j[u], st[u], salt);
                m = kj > m ? kj : m;
            }
        }
    }
    m = group_max_u64<G>(m);
    if (lane == 0) {
        const uint64_t ki = mis_key(i, FIRST ? (int8_t)0 : state[i], salt);
        m1[i] = ki > m ? ki : m;
    }
}

// A node that stays undecided marks itself and its strong neighbours with
// need = round + 1: the nodes whose m1 the next round recomputes.
template <int G>
__global__ void __launch_bounds__(256) k_mis_m2(int32_t n, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ col, const uint8_t *__restrict__ strong,
                                                int8_t *__restrict__ state, uint32_t salt,
                                                const uint64_t *__restrict__ m1, int32_t *__restrict__ need,
                                                int32_t round, const int32_t *__restrict__ prev_undecided,
                                                int32_t *undecided) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / G), lane = (int)(t % G);
    if (i >= n) return;
    if (prev_undecided && *prev_undecided == 0) return;   // every node decided in an earlier round
    if (state[i] != 0) return;   // uniform over the group
    uint64_t m = 0;
    const int ke = rp[i + 1];
    constexpr int U = 4;   // as in k_mis_m1
    for (int k0 = rp[i] + lane; k0 < ke; k0 += U * G) {
        int j[U];
        uint64_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * G < ke) j[u] = col[k0 + u * G];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * G < ke) v[u] = m1[j[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * G;
            if (k < ke && is_strong(strong, k, j[u], i)) m = v[u] > m ? v[u] : m;
        }
    }
    m = group_max_u64<G>(m);
    const uint64_t mi = m1[i];
    m = mi > m ? mi : m;
    // every lane of the group holds the same m
    const bool joins = m == mis_key(i, 0, salt);
    const bool leaves = !joins && (m >> 62) == 3u;
    const bool still = !joins && !leaves && lane == 0;
    if (lane == 0) {
        if (joins)
            state[i] = 1;
        else if (leaves)
            state[i] = 2;
    }
    if (!joins && !leaves && need) {
        if (lane == 0) need[i] = round + 1;
        for (int k = rp[i] + lane; k < ke; k += G) {
            const int j = col[k];
            if (is_strong(strong, k, j, i)) need[j] = round + 1;
        }
    }
    // "some node is still undecided": every writer stores the same value, so
    // one plain store per wavefront suffices (no contended atomic)
    const unsigned long long any = __ballot(still);
    if (any != 0ull && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)any) - 1)) *undecided = 1;
}

// The same rounds on level 0 over the system's sliced-ELL copy, when every
// entry is strong: one lane per row, half a byte of column code per entry
// instead of four, and since the rows of a slice mostly share their offsets,
// the gathers of one entry over the slice's rows are mostly contiguous.  The
// maxima take every stored entry, the diagonal and the padding (the row
// itself) included; these add only the row's own key (m1) or m1 value (m2),
// which enter the maximum anyway, so the results are those of k_mis_m1 /
// k_mis_m2.
//
// f(c, j0) for chunks of kSellChunk columns of this lane's row: c[j] is the
// column of entry j0 + j for j0 + j < w, entries past w repeat entry w-1; rows
// past n name columns of row 0.  Every lane of the wavefront calls it (w is
// uniform over the slice).
template <typename F>
__device__ __forceinline__ void sell_cols_of(const SellCols &C, int64_t slice, int row, int n, int64_t base, int w,
                                             F f) {
    w = __builtin_amdgcn_readfirstlane(w);
    int c[kSellChunk];
    if (!C.code) {
        for (int j0 = 0; j0 < w; j0 += kSellChunk) {
#pragma unroll
            for (int j = 0; j < kSellChunk; ++j) {
                const int jj = j0 + j < w ? j0 + j : w - 1;
                c[j] = C.col[base + (int64_t)jj * kSellC];
            }
            f(c, j0);
        }
        return;
    }
    const int lane = threadIdx.x & 63;
    const int rr = row < n ? row : 0;
    const int dl = C.dict[slice * kSellDict + (lane & (kSellDict - 1))];
    const int64_t cb = C.cp[slice] + lane;
    for (int j0 = 0; j0 < w; j0 += kSellChunk) {
        uint32_t cw[kSellChunk / 8];
#pragma unroll
        for (int q = 0; q < kSellChunk / 8; ++q) {
            const int qq = j0 + 8 * q < w ? j0 / 8 + q : (w - 1) / 8;
            cw[q] = C.code[cb + (int64_t)qq * kSellC];
        }
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) {
            const int jj = j0 + j < w ? j : w - 1 - j0;
            const uint32_t word = (jj >> 3) ? cw[1] : cw[0];
            c[j] = rr + __shfl(dl, (int)((word >> (4 * (jj & 7))) & 15u), 64);
        }
        f(c, j0);
    }
}

template <bool FIRST>
__global__ void __launch_bounds__(kBlock) k_mis_m1_sell(int32_t n, int64_t nslices, int spb,
                                                        const int32_t *__restrict__ sp,
                                                        const int32_t *__restrict__ sw, SellCols C,
                                                        const int8_t *__restrict__ state, uint32_t salt,
                                                        const int32_t *__restrict__ need, int32_t round,
                                                        const int32_t *__restrict__ prev_undecided,
                                                        uint64_t *__restrict__ m1) {
    if (prev_undecided && *prev_undecided == 0) return;   // every node decided in an earlier round
    OCP_SELL_BEGIN(nslices, spb)
    const bool act = row < n && (!need || need[row] == round);
    if (__ballot(act) == 0ull) continue;   // uniform over the slice
    const int rr = row < n ? row : 0;
    uint64_t m = mis_key(rr, FIRST ? (int8_t)0 : state[rr], salt);
    sell_cols_of(C, slice, row, n, base, w, [&](const int (&c)[kSellChunk], int) {
        int8_t st[kSellChunk];
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) st[j] = FIRST ? (int8_t)0 : state[c[j]];
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) {
            const uint64_t kj = mis_key(c[j], st[j], salt);
            m = kj > m ? kj : m;
        }
    });
    if (act) m1[row] = m;
    OCP_SELL_END()
}

__global__ void __launch_bounds__(kBlock) k_mis_m2_sell(int32_t n, int64_t nslices, int spb,
                                                        const int32_t *__restrict__ sp,
                                                        const int32_t *__restrict__ sw, SellCols C,
                                                        int8_t *__restrict__ state, uint32_t salt,
                                                        const uint64_t *__restrict__ m1, int32_t *__restrict__ need,
                                                        int32_t round, const int32_t *__restrict__ prev_undecided,
                                                        int32_t *undecided) {
    if (prev_undecided && *prev_undecided == 0) return;   // every node decided in an earlier round
    OCP_SELL_BEGIN(nslices, spb)
    const bool act = row < n && state[row] == 0;
    if (__ballot(act) == 0ull) continue;   // uniform over the slice
    const int rr = row < n ? row : 0;
    uint64_t m = m1[rr];
    sell_cols_of(C, slice, row, n, base, w, [&](const int (&c)[kSellChunk], int) {
        uint64_t v[kSellChunk];
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) v[j] = m1[c[j]];
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) m = v[j] > m ? v[j] : m;
    });
    const bool joins = act && m == mis_key(row, 0, salt);
    const bool leaves = act && !joins && (m >> 62) == 3u;
    const bool still = act && !joins && !leaves;
    if (joins)
        state[row] = 1;
    else if (leaves)
        state[row] = 2;
    if (need && __ballot(still) != 0ull) {
        if (still) need[row] = round + 1;
        sell_cols_of(C, slice, row, n, base, w, [&](const int (&c)[kSellChunk], int) {
            if (still) {
#pragma unroll
                for (int j = 0; j < kSellChunk; ++j) need[c[j]] = round + 1;
            }
        });
    }
    const unsigned long long any = __ballot(still);
    if (any != 0ull && lane == __ffsll((long long)any) - 1) *undecided = 1;
    OCP_SELL_END()
}

// Rounds over a list of the nodes still undecided when few are left (the
// list is built once; nodes decided later stay in it and are skipped).
// k_mis_m1_list recomputes m1 for every node of the closed neighbourhood of
// a listed undecided node (lane t of the group: node t of N[u], u itself for
// t = 0), which is the set the full-size rounds mark; a node shared by
// several listed nodes is written by each with the same value (its
// neighbours' states do not change during the kernel).  k_mis_m2_list then
// decides the listed undecided nodes as k_mis_m2 does.
__global__ void k_undecided_flags(int32_t n, const int8_t *__restrict__ state, int32_t *__restrict__ fl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) fl[i] = state[i] == 0 ? 1 : 0;
}
__global__ void k_list_fill(int32_t n, const int32_t *__restrict__ fl, const int32_t *__restrict__ pos,
                            int32_t *__restrict__ list) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && fl[i]) list[pos[i]] = i;
}
constexpr int kMisListG = 16;   // lanes per listed node
__device__ __forceinline__ uint64_t mis_m1_of(int v, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                              const uint8_t *__restrict__ strong, const int8_t *__restrict__ state,
                                              uint32_t salt) {
    uint64_t m = mis_key(v, state[v], salt);
    const int ke = rp[v + 1];
    for (int k = rp[v]; k < ke; ++k) {
        const int j = col[k];
        if (is_strong(strong, k, j, v)) {
            const uint64_t kj = mis_key(j, state[j], salt);
            m = kj > m ? kj : m;
        }
    }
    return m;
}
__global__ void __launch_bounds__(256) k_mis_m1_list(const int32_t *__restrict__ list, int32_t nl,
                                                     const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                     const uint8_t *__restrict__ strong,
                                                     const int8_t *__restrict__ state, uint32_t salt,
                                                     const int32_t *__restrict__ prev_undecided,
                                                     uint64_t *__restrict__ m1) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = (int)(t / kMisListG), lane = (int)(t % kMisListG);
    if (r >= nl) return;
    if (prev_undecided && *prev_undecided == 0) return;
    const int u = list[r];
    if (state[u] != 0) return;   // uniform over the group
    if (lane == 0) m1[u] = mis_m1_of(u, rp, col, strong, state, salt);
    const int ke = rp[u + 1];
    for (int k = rp[u] + lane - 1; k < ke; k += kMisListG) {
        if (k < rp[u]) continue;   // lane 0 took u
        const int j = col[k];
        if (is_strong(strong, k, j, u)) m1[j] = mis_m1_of(j, rp, col, strong, state, salt);
    }
}
__global__ void __launch_bounds__(256) k_mis_m2_list(const int32_t *__restrict__ list, int32_t nl,
                                                     const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                                     const uint8_t *__restrict__ strong, int8_t *__restrict__ state,
                                                     uint32_t salt, const uint64_t *__restrict__ m1,
                                                     const int32_t *__restrict__ prev_undecided,
                                                     int32_t *undecided) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int r = (int)(t / kMisListG), lane = (int)(t % kMisListG);
    bool still = false;
    if (r < nl && !(prev_undecided && *prev_undecided == 0)) {
        const int u = list[r];
        if (state[u] == 0) {   // uniform over the group
            uint64_t m = 0;
            const int ke = rp[u + 1];
            for (int k = rp[u] + lane; k < ke; k += kMisListG) {
                const int j = col[k];
                if (is_strong(strong, k, j, u)) {
                    const uint64_t v = m1[j];
                    m = v > m ? v : m;
                }
            }
            m = group_max_u64<kMisListG>(m);
            const uint64_t mu = m1[u];
            m = mu > m ? mu : m;
            const bool joins = m == mis_key(u, 0, salt);
            const bool leaves = !joins && (m >> 62) == 3u;
            if (lane == 0) {
                if (joins)
                    state[u] = 1;
                else if (leaves)
                    state[u] = 2;
            }
            still = !joins && !leaves && lane == 0;
        }
    }
    const unsigned long long any = __ballot(still);
    if (any != 0ull && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)any) - 1)) *undecided = 1;
}

__global__ void k_root_flags(int32_t n, const int8_t *__restrict__ state, int32_t *__restrict__ fl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) fl[i] = state[i] == 1 ? 1 : 0;
}

// roots and their strong neighbours
__global__ void k_agg1(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                       const uint8_t *__restrict__ strong, const int8_t *__restrict__ state,
                       const int32_t *__restrict__ root_pos, uint32_t salt, int32_t *__restrict__ agg,
                       int8_t *__restrict__ assigned) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (state[i] == 1) {
        agg[i] = root_pos[i];
        assigned[i] = 1;
        return;
    }
    uint64_t best = 0;
    int bj = -1;
    const int ke = rp[i + 1];
    constexpr int U = 8;   // columns, then their states, requested together
    for (int k0 = rp[i]; k0 < ke; k0 += U) {
        int j[U];
        int8_t st[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < ke) j[u] = col[k0 + u];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < ke) st[u] = state[j[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u;
            if (k < ke && is_strong(strong, k, j[u], i) && st[u] == 1) {
                const uint64_t kj = mis_key(j[u], 1, salt);
                if (kj > best) {
                    best = kj;
                    bj = j[u];
                }
            }
        }
    }
    agg[i] = bj >= 0 ? root_pos[bj] : -1;
    assigned[i] = bj >= 0 ? 2 : 0;
}

// nodes two steps from a root join a neighbour's aggregate
__global__ void k_agg2(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                       const uint8_t *__restrict__ strong, int8_t *__restrict__ assigned, uint32_t salt,
                       int32_t *__restrict__ agg, int32_t *flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (assigned[i] != 0) return;
    uint64_t best = 0;
    int bj = -1;
    const int ke = rp[i + 1];
    constexpr int U = 8;   // columns, then their states, requested together
    for (int k0 = rp[i]; k0 < ke; k0 += U) {
        int j[U];
        int8_t st[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < ke) j[u] = col[k0 + u];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < ke) st[u] = assigned[j[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u;
            if (k < ke && is_strong(strong, k, j[u], i) && st[u] == 2) {
                const uint64_t kj = mis_key(j[u], 2, salt);
                if (kj > best) {
                    best = kj;
                    bj = j[u];
                }
            }
        }
    }
    if (bj < 0) {
        atomicOr(flag, 16);
        return;
    }
    agg[i] = agg[bj];
    assigned[i] = 3;
}

// The same two passes on level 0 over the system's sliced-ELL copy when every
// entry is strong (as the independent-set rounds there).  The diagonal and the
// padding name the row itself, which is neither a root (k_agg1 looks for roots
// only for non-roots) nor assigned in the first pass (k_agg2 runs for nodes
// that are not), so the choices are those of k_agg1 / k_agg2.
__global__ void __launch_bounds__(kBlock) k_agg1_sell(int32_t n, int64_t nslices, int spb,
                                                      const int32_t *__restrict__ sp, const int32_t *__restrict__ sw,
                                                      SellCols C, const int8_t *__restrict__ state,
                                                      const int32_t *__restrict__ root_pos, uint32_t salt,
                                                      int32_t *__restrict__ agg, int8_t *__restrict__ assigned) {
    OCP_SELL_BEGIN(nslices, spb)
    const int8_t si = row < n ? state[row] : (int8_t)1;
    if (__ballot(si != 1) == 0ull) {   // every row of the slice a root (or past n)
        if (row < n) {
            agg[row] = root_pos[row];
            assigned[row] = 1;
        }
        continue;
    }
    uint64_t best = 0;
    int bj = -1;
    sell_cols_of(C, slice, row, n, base, w, [&](const int (&c)[kSellChunk], int) {
        int8_t st[kSellChunk];
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) st[j] = state[c[j]];
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j)
            if (st[j] == 1) {
                const uint64_t kj = mis_key(c[j], 1, salt);
                if (kj > best) {
                    best = kj;
                    bj = c[j];
                }
            }
    });
    if (row < n) {
        if (si == 1) {
            agg[row] = root_pos[row];
            assigned[row] = 1;
        } else {
            agg[row] = bj >= 0 ? root_pos[bj] : -1;
            assigned[row] = bj >= 0 ? 2 : 0;
        }
    }
    OCP_SELL_END()
}

__global__ void __launch_bounds__(kBlock) k_agg2_sell(int32_t n, int64_t nslices, int spb,
                                                      const int32_t *__restrict__ sp, const int32_t *__restrict__ sw,
                                                      SellCols C, int8_t *__restrict__ assigned, uint32_t salt,
                                                      int32_t *__restrict__ agg, int32_t *flag) {
    OCP_SELL_BEGIN(nslices, spb)
    const bool act = row < n && assigned[row] == 0;
    if (__ballot(act) == 0ull) continue;   // uniform over the slice
    uint64_t best = 0;
    int bj = -1;
    sell_cols_of(C, slice, row, n, base, w, [&](const int (&c)[kSellChunk], int) {
        int8_t st[kSellChunk];
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) st[j] = assigned[c[j]];
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j)
            if (st[j] == 2) {
                const uint64_t kj = mis_key(c[j], 2, salt);
                if (kj > best) {
                    best = kj;
                    bj = c[j];
                }
            }
    });
    if (act) {
        if (bj < 0) {
            atomicOr(flag, 16);
        } else {
            agg[row] = agg[bj];
            assigned[row] = 3;
        }
    }
    OCP_SELL_END()
}

// Aggregate sizes.  Neighbouring nodes often share an aggregate: within a
// wavefront each run of equal aggregates adds its length with one atomic
// (lanes past n hold -1, so a run never extends past the last node).
__global__ void k_agg_sizes(int32_t n, const int32_t *__restrict__ agg, int32_t *__restrict__ size) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = (int)(threadIdx.x & 63);
    const int a = i < n ? agg[i] : -1;
    const int prev = __shfl_up(a, 1, 64);
    const bool head = lane == 0 || prev != a;
    const unsigned long long heads = __ballot(head);
    if (!head || i >= n) return;
    const unsigned long long above = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
    const int next = above ? __ffsll((long long)above) - 1 : 64;
    atomicAdd(&size[a], next - lane);
}

__global__ void k_ptent(int32_t n, const int32_t *__restrict__ agg, const int32_t *__restrict__ size,
                        int32_t *__restrict__ rp, int32_t *__restrict__ col, double *__restrict__ val) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > n) return;
    rp[i] = i;
    if (i == n) return;
    col[i] = agg[i];
    val[i] = 1.0 / sqrt((double)size[agg[i]]);
}

// P = P_tent - w D^-1 (A P_tent), in place over the entries of A P_tent
__global__ void k_smooth_p(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                           double *__restrict__ val, const double *__restrict__ diag, const int32_t *__restrict__ agg,
                           const double *__restrict__ ptent, double w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double s = w / diag[i];
    const int a = agg[i];
    for (int k = rp[i]; k < rp[i + 1]; ++k) val[k] = (col[k] == a ? ptent[i] : 0.0) - s * val[k];
}

// ------------------------------------------------------------------ SpGEMM
// C = A B, row by row.  A group of G lanes owns one output row and an LDS
// hash table of H slots (G and H chosen per row from the bound
// ub_i = sum_k nnz(B row k) over the entries of A row i).  The group walks
// the entries of its A row in ascending order; at each step its lanes take
// distinct columns of one B row, so no two lanes touch one slot and every
// output entry is accumulated in the fixed order of the A row.  Finally the
// occupied slots are ranked by column and written in ascending order.  The
// lanes of a group live in one wavefront; their LDS accesses are ordered with
// wavefront-scope fences instead of workgroup barriers.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// B rows are CSR (blen == nullptr: row c spans brp[c] .. brp[c+1]) or given
// by start and length (row c spans brp[c] .. brp[c] + blen[c]).
__global__ void k_spgemm_ub(int32_t m, const int32_t *__restrict__ arp, const int32_t *__restrict__ acol,
                            const int32_t *__restrict__ brp, const int32_t *__restrict__ blen,
                            int32_t *__restrict__ ub) {
    // XCD x takes a contiguous run of blocks (measured faster here)
    const int i = (int)dev::xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int64_t s = 0;
    const int ke = arp[i + 1];
    constexpr int U = 8;   // columns, then their row extents, requested together
    for (int k0 = arp[i]; k0 < ke; k0 += U) {
        int c[U], b0[U], b1[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < ke) c[u] = acol[k0 + u];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < ke) {
                b0[u] = brp[c[u]];
                b1[u] = blen ? b0[u] + blen[c[u]] : brp[c[u] + 1];
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < ke) s += b1[u] - b0[u];
    }
    ub[i] = (int32_t)(s > INT32_MAX ? INT32_MAX : s);
}

// the same bound with G lanes per row, for long A rows
template <int G>
__global__ void __launch_bounds__(256) k_spgemm_ub_grp(int32_t m, const int32_t *__restrict__ arp,
                                                       const int32_t *__restrict__ acol,
                                                       const int32_t *__restrict__ brp,
                                                       const int32_t *__restrict__ blen, int32_t *__restrict__ ub) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int i = (int)(t / G), lane = (int)(t % G);
    if (i >= m) return;   // uniform over the group
    int64_t s = 0;
    const int ke = arp[i + 1];
    constexpr int U = 2;   // columns, then their row extents, requested together
    for (int k0 = arp[i] + lane; k0 < ke; k0 += U * G) {
        int c[U], b0[U], b1[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * G < ke) c[u] = acol[k0 + u * G];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * G < ke) {
                b0[u] = brp[c[u]];
                b1[u] = blen ? b0[u] + blen[c[u]] : brp[c[u] + 1];
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * G < ke) s += b1[u] - b0[u];
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
    if (lane == 0) ub[i] = (int32_t)(s > INT32_MAX ? INT32_MAX : s);
}

constexpr int kSpgemmClasses = 5;
struct ClassBounds {
    int lim[kSpgemmClasses - 1];   // class q holds keys <= lim[q]; the last class the rest
};

// Row lists per size class.  Positions are reserved with LDS atomics inside
// the block and one global atomic per class per block.
constexpr int kBinChunks = 16;   // 256-row chunks per block of the binning pass

__device__ __forceinline__ int bin_class(int u, const ClassBounds &cb) {
    int c = kSpgemmClasses - 1;
    for (int q = 0; q < kSpgemmClasses - 1; ++q)
        if (u <= cb.lim[q]) {
            c = q;
            break;
        }
    return c;
}

// Each block bins kBinChunks chunks of 256 rows: positions inside a
// wavefront come from ballots, the block's per-class offsets from a prefix
// over its (chunk, wavefront) counts, and one global atomic per class and
// block reserves the block's range (one atomic per 256 rows serialized on
// the few class counters).
__global__ void __launch_bounds__(256) k_bin_rows(int32_t m, const int32_t *__restrict__ key, ClassBounds cb,
                                                  int32_t *__restrict__ counts, int32_t *__restrict__ lists) {
    __shared__ int wcnt[kBinChunks][4][kSpgemmClasses], lbase[kSpgemmClasses];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * kBinChunks * 256;
    for (int ch = 0; ch < kBinChunks; ++ch) {
        const int64_t i = r0 + ch * 256 + threadIdx.x;
        const bool valid = i < m;
        const int c = valid ? bin_class(key[i], cb) : -1;
#pragma unroll
        for (int q = 0; q < kSpgemmClasses; ++q) {
            const unsigned long long mask = __ballot(c == q);
            if (lane == 0) wcnt[ch][wv][q] = __popcll(mask);
        }
    }
    __syncthreads();
    if (threadIdx.x < kSpgemmClasses) {
        const int q = threadIdx.x;
        int tot = 0;
        for (int ch = 0; ch < kBinChunks; ++ch)
            for (int w = 0; w < 4; ++w) {
                const int t = wcnt[ch][w][q];
                wcnt[ch][w][q] = tot;
                tot += t;
            }
        if (tot > 0) lbase[q] = atomicAdd(&counts[q], tot);
    }
    __syncthreads();
    for (int ch = 0; ch < kBinChunks; ++ch) {
        const int64_t i = r0 + ch * 256 + threadIdx.x;
        const bool valid = i < m;
        const int c = valid ? bin_class(key[i], cb) : -1;
        int lpos = 0;
#pragma unroll
        for (int q = 0; q < kSpgemmClasses; ++q) {
            const unsigned long long mask = __ballot(c == q);
            if (c == q) lpos = __popcll(mask & ((1ull << lane) - 1ull));
        }
        if (valid) lists[(int64_t)c * m + lbase[c] + wcnt[ch][wv][c] + lpos] = (int32_t)i;
    }
}

template <int H>
__device__ __forceinline__ int hash_insert(int *keys, int key, int *count) {
    int s = (int)(((uint32_t)key * 2654435761u) >> (32 - __builtin_ctz(H)));
    for (;;) {
        const int prev = atomicCAS(&keys[s], -1, key);
        if (prev == -1) {
            if (count) atomicAdd(count, 1);
            return s;
        }
        if (prev == key) return s;
        s = (s + 1) & (H - 1);
    }
}

// hash_insert that gives up (returns -1) after probing every slot once
template <int H>
__device__ __forceinline__ int hash_insert_bounded(int *keys, int key) {
    int s = (int)(((uint32_t)key * 2654435761u) >> (32 - __builtin_ctz(H)));
    for (int p = 0; p < H; ++p) {
        const int prev = atomicCAS(&keys[s], -1, key);
        if (prev == -1 || prev == key) return s;
        s = (s + 1) & (H - 1);
    }
    return -1;
}

// B rows as in k_spgemm_ub (CSR, or start and length).
// NUMERIC = false: cnt[i] = number of distinct columns of C row i.
// NUMERIC = true, W = 0: write C row i (columns ascending) at crp[i].
// NUMERIC = true, W > 0: write the row at ccol/cval + r W, r its position in
//   rows, and its length at cnt[i]; a row with more than W columns, or one
//   that fills the table (it then stops after the current B row), is listed
//   in retry[] (counted in *nretry) and written nowhere.
template <int G, int H, bool NUMERIC, int W = 0>
__global__ void __launch_bounds__(64) k_spgemm_grp(const int32_t *__restrict__ rows, int32_t nrows,
                                                   const int32_t *__restrict__ arp, const int32_t *__restrict__ acol,
                                                   const double *__restrict__ aval, const int32_t *__restrict__ brp,
                                                   const int32_t *__restrict__ blen,
                                                   const int32_t *__restrict__ bcol, const double *__restrict__ bval,
                                                   const int32_t *__restrict__ crp, int32_t *__restrict__ cnt,
                                                   int32_t *__restrict__ ccol, double *__restrict__ cval,
                                                   int32_t *flag, int32_t *retry, int32_t *nretry) {
    constexpr int RPW = 64 / G;
    constexpr int MB = G <= 16 ? 16 / G : 0;   // B entries per lane and A entry fetched ahead
    static_assert(W <= H, "a padded row fits its table");
    constexpr int LIM = (3 * H) / 4;   // symbolic: count past which the row is retried
    __shared__ __align__(16) int keys[RPW][H];
    __shared__ double vals[NUMERIC ? RPW : 1][NUMERIC ? H : 1];
    __shared__ int list[NUMERIC ? RPW : 1][NUMERIC ? H : 1];
    __shared__ int count[RPW];
    __shared__ int full[RPW];
    const int g = threadIdx.x / G, lane = threadIdx.x % G;
    const int r = blockIdx.x * RPW + g;
    const int i = r < nrows ? (rows ? rows[r] : r) : 0;   // rows == nullptr: every row, in order
    // a CSR numeric pass over every row leaves rows past half its table to another launch
    const bool active = r < nrows && !(NUMERIC && W == 0 && !rows && crp[i + 1] - crp[i] > H / 2);
    for (int q = lane; q < H; q += G) {
        keys[g][q] = -1;
        if (NUMERIC) vals[g][q] = 0.0;
    }
    if (lane == 0) {
        count[g] = 0;
        full[g] = 0;
    }
    wave_sync();
    // one product into the table: symbolic passes count new columns, padded
    // passes flag a full table, the others rely on a table sized for the row
    auto put = [&](int key, double v) {
        if (!NUMERIC) {
            // the count is checked before every insert, so the table never fills
            if (*(volatile int *)&count[g] <= LIM) hash_insert<H>(keys[g], key, &count[g]);
        } else if (W > 0) {
            const int q = hash_insert_bounded<H>(keys[g], key);
            if (q < 0)
                full[g] = 1;
            else
                vals[g][q] += v;
        } else {
            vals[g][hash_insert<H>(keys[g], key, nullptr)] += v;
        }
    };
    // after each B row: the group stops once its row is known to be retried
    auto stop = [&]() {
        return (!NUMERIC && *(volatile int *)&count[g] > LIM) || (W > 0 && *(volatile int *)&full[g] != 0);
    };
    if (active) {
        const int ke = arp[i + 1];
        bool done = false;
        for (int kb = arp[i]; kb < ke && !done; kb += G) {
            // lanes fetch the metadata of G consecutive A entries at once
            double am = 0.0;
            int tb = 0, tn = 0;
            if (kb + lane < ke) {
                const int c = acol[kb + lane];
                if (NUMERIC) am = aval[kb + lane];
                tb = brp[c];
                tn = blen ? tb + blen[c] : brp[c + 1];
            }
            const int cnt = ke - kb < G ? ke - kb : G;
            if constexpr (MB > 0) {
                // the first MB of this lane's entries of each of the G B rows
                // are requested before any is inserted; longer rows continue
                // in the loop below.  Insertion order is unchanged.
                int bc[G][MB];
                double bv[NUMERIC ? G : 1][MB];
#pragma unroll
                for (int jj = 0; jj < G; ++jj) {
                    const int t0 = __shfl(tb, jj, G), t1 = __shfl(tn, jj, G);
#pragma unroll
                    for (int m = 0; m < MB; ++m) {
                        const int t = t0 + lane + m * G;
                        if (jj < cnt && t < t1) {
                            bc[jj][m] = bcol[t];
                            if (NUMERIC) bv[jj][m] = bval[t];
                        }
                    }
                }
#pragma unroll
                for (int jj = 0; jj < G; ++jj) {
                    if (jj >= cnt || done) break;
                    const int t0 = __shfl(tb, jj, G), t1 = __shfl(tn, jj, G);
                    const double a = NUMERIC ? __shfl(am, jj, G) : 0.0;
#pragma unroll
                    for (int m = 0; m < MB; ++m) {
                        if (t0 + lane + m * G >= t1) break;
                        put(bc[jj][m], NUMERIC ? a * bv[NUMERIC ? jj : 0][m] : 0.0);
                    }
                    for (int t = t0 + lane + MB * G; t < t1; t += G) put(bcol[t], NUMERIC ? a * bval[t] : 0.0);
                    wave_sync();
                    done = stop();
                }
            } else {
                for (int jj = 0; jj < cnt && !done; ++jj) {
                    const int t0 = __shfl(tb, jj, G), t1 = __shfl(tn, jj, G);
                    const double a = NUMERIC ? __shfl(am, jj, G) : 0.0;
                    for (int t = t0 + lane; t < t1; t += G) put(bcol[t], NUMERIC ? a * bval[t] : 0.0);
                    wave_sync();
                    done = stop();
                }
            }
        }
    }
    if (!NUMERIC) {
        if (active && lane == 0) {
            cnt[i] = count[g];
            if (count[g] > (3 * H) / 4) {
                if (retry)
                    retry[atomicAdd(nretry, 1)] = i;   // recount with a larger table
                else
                    atomicOr(flag, 32);
            }
        }
        return;
    }
    // compact the occupied slots (spreading them over the lanes), rank each
    // by column, write the row
    for (int q = lane; q < H; q += G)
        if (keys[g][q] >= 0) list[g][atomicAdd(&count[g], 1)] = q;
    wave_sync();
    if (!active) return;
    const int nc = count[g];
    if (W > 0 && (full[g] != 0 || nc > W)) {
        if (lane == 0) retry[atomicAdd(nretry, 1)] = i;
        return;
    }
    const int64_t base = W > 0 ? (int64_t)r * W : crp[i];
    if (W > 0 && lane == 0) cnt[i] = nc;
    for (int e = lane; e < nc; e += G) {
        const int se = list[g][e];
        const int kk = keys[g][se];
        int rank = 0;
        if constexpr (H <= 512) {
            // against the whole table, four slots per read; an empty slot
            // (-1) is the largest unsigned value and never counts
            const uint4 *kt = reinterpret_cast<const uint4 *>(&keys[g][0]);
            const uint32_t ku = (uint32_t)kk;
#pragma unroll 8
            for (int f = 0; f < H / 4; ++f) {
                const uint4 v = kt[f];
                rank += (int)(v.x < ku) + (int)(v.y < ku) + (int)(v.z < ku) + (int)(v.w < ku);
            }
        } else {
            for (int f = 0; f < nc; ++f) rank += keys[g][list[g][f]] < kk;
        }
        ccol[base + rank] = kk;
        cval[base + rank] = vals[g][se];
    }
}

struct Csr {
    int32_t rows = 0, cols = 0;
    int64_t nnz = 0;
    DevBuf<int32_t> rp, col;
    DevBuf<double> val;
};

template <int G, int H, bool NUMERIC, int W = 0>
static void launch_grp(ocp_ctx *ctx, const int32_t *rows, int32_t nrows, const int32_t *arp, const int32_t *acol,
                       const double *aval, const int32_t *brp, const int32_t *bcol, const double *bval,
                       const int32_t *crp, int32_t *cnt, int32_t *ccol, double *cval, int32_t *retry = nullptr,
                       int32_t *nretry = nullptr, const int32_t *blen = nullptr) {
    if (nrows <= 0) return;
    constexpr int RPW = 64 / G;
    const unsigned blocks = (unsigned)((nrows + RPW - 1) / RPW);
    k_spgemm_grp<G, H, NUMERIC, W><<<blocks, 64, 0, ctx->stream>>>(rows, nrows, arp, acol, aval, brp, blen, bcol, bval,
                                                                    crp, cnt, ccol, cval, ctx->dev_flag, retry,
                                                                    nretry);
    OCP_LAUNCH_CHECK();
}

__global__ void k_row_len(int32_t m, const int32_t *__restrict__ rp, double *__restrict__ len) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) len[i] = (double)(rp[i + 1] - rp[i]);
}

static int csr_max_row(ocp_ctx *ctx, int32_t m, const int32_t *rp) {
    DevBuf<double> len(ctx, (size_t)std::max(m, 1));
    k_row_len<<<grid_for(m, 256), 256, 0, ctx->stream>>>(m, rp, len.get());
    OCP_LAUNCH_CHECK();
    return (int)reduce_max_abs(ctx, len.get(), m);
}

// C = A P_tent (one entry per row of P_tent: column agg[j], value pt[j]),
// one thread per row with up to 16 distinct columns held in registers;
// entries accumulate in the order of the A row and are sorted by a network.
template <bool NUMERIC>
__global__ void __launch_bounds__(256) k_ap_tent(int32_t m, const int32_t *__restrict__ arp,
                                                 const int32_t *__restrict__ acol, const double *__restrict__ aval,
                                                 const int32_t *__restrict__ agg, const double *__restrict__ pt,
                                                 const int32_t *__restrict__ crp, int32_t *__restrict__ cnt,
                                                 int32_t *__restrict__ ccol, double *__restrict__ cval,
                                                 int32_t *flag, const double *__restrict__ diag, double w) {
    constexpr int S = 16;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int keys[S];
    double acc[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        keys[q] = INT_MAX;
        acc[q] = 0.0;
    }
    int nk = 0;
    const int ke = arp[i + 1];
    // U entries at a time: their columns, then the aggregates and tentative
    // values of those columns, are requested before any is used (entries are
    // still taken in row order)
    constexpr int U = 8;
    for (int k0 = arp[i]; k0 < ke; k0 += U) {
        int j[U], J[U];
        double av[U], pv[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < ke) {
                j[u] = acol[k0 + u];
                if (NUMERIC) av[u] = aval[k0 + u];
            }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u < ke) {
                J[u] = agg[j[u]];
                if (NUMERIC) pv[u] = pt[j[u]];
            }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (k0 + u >= ke) break;
            const double v = NUMERIC ? av[u] * pv[u] : 0.0;
            bool found = false;
#pragma unroll
            for (int q = 0; q < S; ++q)
                if (keys[q] == J[u]) {
                    acc[q] += v;
                    found = true;
                }
            if (!found) {
                if (nk == S) {
                    atomicOr(flag, 32);
                    return;
                }
#pragma unroll
                for (int q = 0; q < S; ++q)
                    if (q == nk) {
                        keys[q] = J[u];
                        acc[q] = v;
                    }
                ++nk;
            }
        }
    }
    if (!NUMERIC) {
        cnt[i] = nk;
        return;
    }
    dev::sort_slots(keys, acc);
    const int b = crp[i];
    // with diag given, the row of the smoothed prolongator
    // P = P_tent - w D^-1 (A P_tent), as k_smooth_p forms it
    const double sw = diag ? w / diag[i] : 0.0;
    const int ai = agg[i];
    const double pti = pt[i];
#pragma unroll
    for (int q = 0; q < S; ++q)
        if (q < nk) {
            ccol[b + q] = keys[q];
            cval[b + q] = diag ? (keys[q] == ai ? pti : 0.0) - sw * acc[q] : acc[q];
        }
}

// Rows formed in padded slots (row r of a class list at pcol/pval + r W)
// copied to their CSR positions, L lanes per row; rows longer than W were
// formed in the CSR directly.
template <int L>
__global__ void __launch_bounds__(256) k_pad_copy(const int32_t *__restrict__ rows, int32_t nrows, int W,
                                                  const int32_t *__restrict__ pcol, const double *__restrict__ pval,
                                                  const int32_t *__restrict__ crp, int32_t *__restrict__ ccol,
                                                  double *__restrict__ cval) {
    const int r = blockIdx.x * (256 / L) + (int)(threadIdx.x / L);
    const int lane = (int)(threadIdx.x % L);
    if (r >= nrows) return;
    const int i = rows ? rows[r] : r;   // rows == nullptr: every row, in order
    const int b = crp[i], len = crp[i + 1] - b;
    if (len > W) return;
    const int64_t p = (int64_t)r * W;
    for (int e = lane; e < len; e += L) {
        ccol[b + e] = pcol[p + e];
        cval[b + e] = pval[p + e];
    }
}

// C = A B by hash tables in LDS.  Rows are binned by their product bound
// (the sum of the B row lengths over the A row) and formed in one numeric
// pass that writes each row, columns ascending, into a padded slot of its
// class and records its length: bound <= 16 in 32 slots by 4 lanes, <= 64 in
// 64 slots by 4 lanes (rows past 48 columns retried), larger bounds in 128
// slots by 8 lanes (past 96 columns retried), or, when fewer than
// kWideRows rows have such bounds, in 512 slots by a whole wavefront (past
// 384 columns retried).  Retried rows are counted in 512 slots (4096 past
// 384 columns) and formed in the CSR directly, after the scan of the lengths.
constexpr int kWideRows = 16384;
static void spgemm(ocp_ctx *ctx, int32_t m, int32_t ncols, int64_t annz, const int32_t *arp, const int32_t *acol,
                   const double *aval, const int32_t *brp, const int32_t *bcol, const double *bval, Csr &C,
                   const int32_t *blen = nullptr) {
    hipStream_t s = ctx->stream;
    DevBuf<int32_t> ub(ctx, (size_t)m + 1);
    if (annz >= 32 * (int64_t)m)   // long A rows: 16 lanes per row
        k_spgemm_ub_grp<16><<<grid_for((int64_t)m * 16, 256), 256, 0, s>>>(m, arp, acol, brp, blen, ub.get());
    else
        k_spgemm_ub<<<grid_for(m, 256), 256, 0, s>>>(m, arp, acol, brp, blen, ub.get());
    OCP_LAUNCH_CHECK();
    DevBuf<int32_t> counts(ctx, 8);
    fill_zero_bytes(ctx, counts.get(), 32);
    DevBuf<int32_t> lists(ctx, (size_t)kSpgemmClasses * m);
    const ClassBounds cls{{16, 64, INT_MAX - 1, INT_MAX - 1}};
    k_bin_rows<<<grid_for(m, 256 * kBinChunks), 256, 0, s>>>(m, ub.get(), cls, counts.get(), lists.get());
    OCP_LAUNCH_CHECK();
    int32_t hc[8];
    read_back(ctx, hc, counts.get(), 32);
    const int64_t M = m;
    const bool wide = hc[2] < kWideRows;
    const int32_t W[3] = {16, 48, wide ? 384 : 96};   // padded widths of the three classes
    int64_t off[4] = {0, 0, 0, 0};
    for (int c = 0; c < 3; ++c) off[c + 1] = off[c] + (int64_t)hc[c] * W[c];
    DevBuf<int32_t> pcol(ctx, (size_t)std::max<int64_t>(off[3], 1));
    DevBuf<double> pval(ctx, (size_t)std::max<int64_t>(off[3], 1));
    DevBuf<int32_t> cnt(ctx, (size_t)m + 1);
    DevBuf<int32_t> retry(ctx, (size_t)m + 1);   // retry[m]: number of listed rows
    fill_zero_bytes(ctx, retry.get() + m, 4);
    int32_t *nr = retry.get() + m;
    launch_grp<4, 32, true, 16>(ctx, lists.get(), hc[0], arp, acol, aval, brp, bcol, bval, nullptr, cnt.get(),
                                pcol.get(), pval.get(), retry.get(), nr, blen);
    launch_grp<4, 64, true, 48>(ctx, lists.get() + M, hc[1], arp, acol, aval, brp, bcol, bval, nullptr, cnt.get(),
                                pcol.get() + off[1], pval.get() + off[1], retry.get(), nr, blen);
    if (wide)
        launch_grp<64, 512, true, 384>(ctx, lists.get() + 2 * M, hc[2], arp, acol, aval, brp, bcol, bval, nullptr,
                                       cnt.get(), pcol.get() + off[2], pval.get() + off[2], retry.get(), nr, blen);
    else
        launch_grp<8, 128, true, 96>(ctx, lists.get() + 2 * M, hc[2], arp, acol, aval, brp, bcol, bval, nullptr,
                                     cnt.get(), pcol.get() + off[2], pval.get() + off[2], retry.get(), nr, blen);
    int32_t nretry = 0;
    read_back(ctx, &nretry, nr, 4);
    int32_t nlong = 0;
    DevBuf<int32_t> retry2(ctx, (size_t)std::max(nretry, 1) + 1);
    if (nretry > 0) {
        fill_zero_bytes(ctx, retry2.get() + std::max(nretry, 1), 4);
        fill_zero_bytes(ctx, ctx->dev_flag, 4);
        launch_grp<16, 512, false>(ctx, retry.get(), nretry, arp, acol, aval, brp, bcol, bval, nullptr, cnt.get(),
                                   nullptr, nullptr, retry2.get(), retry2.get() + std::max(nretry, 1), blen);
        read_back(ctx, &nlong, retry2.get() + std::max(nretry, 1), 4);
        if (nlong > 0)
            launch_grp<64, 4096, false>(ctx, retry2.get(), nlong, arp, acol, aval, brp, bcol, bval, nullptr,
                                        cnt.get(), nullptr, nullptr, nullptr, nullptr, blen);
        int32_t fl = 0;
        read_back(ctx, &fl, ctx->dev_flag, 4);
        if (fl & 32) fail(OCP_ERR_UNSUPPORTED, "sparse product row with more than 3072 entries");
    }
    C.rows = m;
    C.cols = ncols;
    C.rp.reset(ctx, (size_t)m + 1);
    C.nnz = scan_exclusive(ctx, cnt.get(), C.rp.get(), m);
    C.col.reset(ctx, (size_t)std::max<int64_t>(C.nnz, 1));
    C.val.reset(ctx, (size_t)std::max<int64_t>(C.nnz, 1));
    for (int c = 0; c < 3; ++c) {
        if (hc[c] <= 0) continue;
        if (W[c] <= 16)
            k_pad_copy<16><<<(unsigned)((hc[c] + 15) / 16), 256, 0, s>>>(lists.get() + c * M, hc[c], W[c],
                                                                         pcol.get() + off[c], pval.get() + off[c],
                                                                         C.rp.get(), C.col.get(), C.val.get());
        else
            k_pad_copy<64><<<(unsigned)((hc[c] + 3) / 4), 256, 0, s>>>(lists.get() + c * M, hc[c], W[c],
                                                                       pcol.get() + off[c], pval.get() + off[c],
                                                                       C.rp.get(), C.col.get(), C.val.get());
        OCP_LAUNCH_CHECK();
    }
    if (nretry == 0) return;
    // every listed row holds at most 384 columns unless some were recounted,
    // then all of them go through the 4096-slot table
    if (nlong == 0)
        launch_grp<16, 512, true>(ctx, retry.get(), nretry, arp, acol, aval, brp, bcol, bval, C.rp.get(), nullptr,
                                  C.col.get(), C.val.get(), nullptr, nullptr, blen);
    else
        launch_grp<64, 4096, true>(ctx, retry.get(), nretry, arp, acol, aval, brp, bcol, bval, C.rp.get(), nullptr,
                                   C.col.get(), C.val.get(), nullptr, nullptr, blen);
}

// A product kept in padded form for use as the B operand of a following
// product: row i spans col/val[start[i] .. start[i] + len[i]).
struct PadCsr {
    DevBuf<int32_t> start, len, col;
    DevBuf<double> val;
};

__global__ void k_pad_starts(int32_t m, int W, int32_t *__restrict__ start) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) start[i] = i * W;
}

__global__ void k_gather_len(int32_t nr, const int32_t *__restrict__ rows, const int32_t *__restrict__ len,
                             int32_t *__restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nr) out[r] = len[rows[r]];
}

__global__ void k_set_starts(int32_t nr, const int32_t *__restrict__ rows, const int32_t *__restrict__ off,
                             int32_t base, int32_t *__restrict__ start) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nr) start[rows[r]] = base + off[r];
}

// C = A B when nearly every row of C has at most 16 columns, left in padded
// form: every row is formed in a 32-slot table by 4 lanes into its 16-wide
// slot; the few longer rows are counted and formed in larger tables into a
// region after the slots (m entries are reserved for them; a larger need
// moves the slots to a bigger buffer first).
static void spgemm_small_rows(ocp_ctx *ctx, int32_t m, const int32_t *arp, const int32_t *acol, const double *aval,
                              const int32_t *brp, const int32_t *bcol, const double *bval, PadCsr &C) {
    constexpr int W = 16;
    hipStream_t s = ctx->stream;
    const int64_t slots = (int64_t)m * W;
    if (slots + m > INT32_MAX) fail(OCP_ERR_UNSUPPORTED, "padded product too large");
    int64_t cap = slots + std::max<int64_t>(m, 1);
    C.col.reset(ctx, (size_t)cap);
    C.val.reset(ctx, (size_t)cap);
    C.len.reset(ctx, (size_t)m + 1);
    C.start.reset(ctx, (size_t)m + 1);
    k_pad_starts<<<grid_for(m, 256), 256, 0, s>>>(m, W, C.start.get());
    OCP_LAUNCH_CHECK();
    DevBuf<int32_t> retry(ctx, (size_t)m + 1);   // retry[m]: number of listed rows
    fill_zero_bytes(ctx, retry.get() + m, 4);
    launch_grp<4, 32, true, W>(ctx, nullptr, m, arp, acol, aval, brp, bcol, bval, nullptr, C.len.get(), C.col.get(),
                               C.val.get(), retry.get(), retry.get() + m);
    int32_t nretry = 0;
    read_back(ctx, &nretry, retry.get() + m, 4);
    if (nretry == 0) return;
    // rows past 16 columns: counted in 512 slots, recounted in 4096 slots
    // when more than 384 columns show up
    int32_t nlong = 0;
    DevBuf<int32_t> retry2(ctx, (size_t)nretry + 1);
    fill_zero_bytes(ctx, retry2.get() + nretry, 4);
    fill_zero_bytes(ctx, ctx->dev_flag, 4);
    launch_grp<16, 512, false>(ctx, retry.get(), nretry, arp, acol, aval, brp, bcol, bval, nullptr, C.len.get(),
                               nullptr, nullptr, retry2.get(), retry2.get() + nretry);
    read_back(ctx, &nlong, retry2.get() + nretry, 4);
    if (nlong > 0)
        launch_grp<64, 4096, false>(ctx, retry2.get(), nlong, arp, acol, aval, brp, bcol, bval, nullptr, C.len.get(),
                                    nullptr, nullptr);
    int32_t fl = 0;
    read_back(ctx, &fl, ctx->dev_flag, 4);
    if (fl & 32) fail(OCP_ERR_UNSUPPORTED, "sparse product row with more than 3072 entries");
    // the listed rows go after the slots, in list order
    DevBuf<int32_t> lens(ctx, (size_t)nretry + 1), off(ctx, (size_t)nretry + 1);
    k_gather_len<<<grid_for(nretry, 256), 256, 0, s>>>(nretry, retry.get(), C.len.get(), lens.get());
    OCP_LAUNCH_CHECK();
    const int64_t extra = scan_exclusive(ctx, lens.get(), off.get(), nretry);
    if (slots + extra > INT32_MAX) fail(OCP_ERR_UNSUPPORTED, "padded product too large");
    if (slots + extra > cap) {
        DevBuf<int32_t> col2(ctx, (size_t)(slots + extra));
        DevBuf<double> val2(ctx, (size_t)(slots + extra));
        OCP_HIP(hipMemcpyAsync(col2.get(), C.col.get(), sizeof(int32_t) * (size_t)slots, hipMemcpyDeviceToDevice, s));
        OCP_HIP(hipMemcpyAsync(val2.get(), C.val.get(), sizeof(double) * (size_t)slots, hipMemcpyDeviceToDevice, s));
        C.col = std::move(col2);
        C.val = std::move(val2);
    }
    k_set_starts<<<grid_for(nretry, 256), 256, 0, s>>>(nretry, retry.get(), off.get(), (int32_t)slots,
                                                        C.start.get());
    OCP_LAUNCH_CHECK();
    // every listed row holds at most 384 columns unless some were recounted,
    // then all of them go through the 4096-slot table
    if (nlong == 0)
        launch_grp<16, 512, true>(ctx, retry.get(), nretry, arp, acol, aval, brp, bcol, bval, C.start.get(), nullptr,
                                  C.col.get(), C.val.get());
    else
        launch_grp<64, 4096, true>(ctx, retry.get(), nretry, arp, acol, aval, brp, bcol, bval, C.start.get(),
                                   nullptr, C.col.get(), C.val.get());
}

// The numeric pass of the same product on level 0 over the system's
// sliced-ELL copy (one lane per row, half a byte of column code and the value
// per entry, both read by whole slices).  The entries come in row order, so
// the sums are formed in the same order; the padding (column the row, value 0)
// adds zero to the row's own aggregate, which its diagonal entry has already
// entered, so the row has the columns the count pass found.
__global__ void __launch_bounds__(kBlock) k_ap_tent_sell(int32_t m, int64_t nslices, int spb,
                                                         const int32_t *__restrict__ sp,
                                                         const int32_t *__restrict__ sw, SellCols C,
                                                         const double *__restrict__ sval,
                                                         const int32_t *__restrict__ agg,
                                                         const double *__restrict__ pt,
                                                         const int32_t *__restrict__ crp, int32_t *__restrict__ ccol, double *__restrict__ cval,
                                                         int32_t *flag, const double *__restrict__ diag, double wgt) {
    constexpr int S = 16;
    OCP_SELL_BEGIN(nslices, spb)
    int keys[S];
    double acc[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
        keys[q] = INT_MAX;
        acc[q] = 0.0;
    }
    int nk = 0;
    bool over = false;
    sell_cols_of(C, slice, row, m, base, w, [&](const int (&c)[kSellChunk], int j0) {
        int J[kSellChunk];
        double av[kSellChunk], pv[kSellChunk];
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) {
            const int jj = j0 + j < w ? j0 + j : w - 1;
            av[j] = sval[base + (int64_t)jj * kSellC];
            J[j] = agg[c[j]];
            pv[j] = pt[c[j]];
        }
#pragma unroll
        for (int j = 0; j < kSellChunk; ++j) {
            if (j0 + j >= w) break;
            const double v = av[j] * pv[j];
            bool found = false;
#pragma unroll
            for (int q = 0; q < S; ++q)
                if (keys[q] == J[j]) {
                    acc[q] += v;
                    found = true;
                }
            if (!found) {
                if (nk == S) {
                    over = true;
                } else {
#pragma unroll
                    for (int q = 0; q < S; ++q)
                        if (q == nk) {
                            keys[q] = J[j];
                            acc[q] = v;
                        }
                    ++nk;
                }
            }
        }
    });
    if (row < m) {
        if (over) atomicOr(flag, 32);
        dev::sort_slots(keys, acc);
        const int b = crp[row];
        const double swi = diag ? wgt / diag[row] : 0.0;   // (w is the slice width here)
        const int ai = agg[row];
        const double pti = pt[row];
#pragma unroll
        for (int q = 0; q < S; ++q)
            if (q < nk) {
                ccol[b + q] = keys[q];
                cval[b + q] = diag ? (keys[q] == ai ? pti : 0.0) - swi * acc[q] : acc[q];
            }
    }
    OCP_SELL_END()
}

// C = A P_tent: the register kernel when every A row has at most 16 entries,
// otherwise the general product with P_tent as a CSR matrix
// With diag given, the register kernel writes the smoothed prolongator
// P = P_tent - w D^-1 (A P_tent) directly; returns whether it did (else C
// holds A P_tent).
static bool spgemm_ptent(ocp_ctx *ctx, int32_t m, int32_t ncols, int64_t annz, const int32_t *arp,
                         const int32_t *acol, const double *aval, const int32_t *agg, const int32_t *trp,
                         const double *pt, Csr &C, const double *diag, double w, const Sell *sell) {
    if (csr_max_row(ctx, m, arp) > 16) {
        spgemm(ctx, m, ncols, annz, arp, acol, aval, trp, agg, pt, C);
        return false;
    }
    DevBuf<int32_t> cnt(ctx, (size_t)m + 1);
    fill_zero_bytes(ctx, ctx->dev_flag, 4);
    // counts from the CSR rows (measured faster than from the sliced-ELL copy;
    // the same counts, every row holding its diagonal)
    k_ap_tent<false><<<grid_for(m, 256), 256, 0, ctx->stream>>>(m, arp, acol, aval, agg, pt, nullptr, cnt.get(),
                                                                nullptr, nullptr, ctx->dev_flag, nullptr, 0.0);
    OCP_LAUNCH_CHECK();
    const SellLaunch LS = sell_launch(sell ? sell->nslices : 1);
    C.rows = m;
    C.cols = ncols;
    C.rp.reset(ctx, (size_t)m + 1);
    C.nnz = scan_exclusive(ctx, cnt.get(), C.rp.get(), m);
    C.col.reset(ctx, (size_t)std::max<int64_t>(C.nnz, 1));
    C.val.reset(ctx, (size_t)std::max<int64_t>(C.nnz, 1));
    if (sell)
        k_ap_tent_sell<<<LS.blocks, kBlock, 0, ctx->stream>>>(m, sell->nslices, LS.slices_per_block, sell->sp.get(),
                                                              sell->sw.get(), sell_cols(*sell), sell->val.get(), agg,
                                                              pt, C.rp.get(), C.col.get(), C.val.get(), ctx->dev_flag,
                                                              diag, w);
    else
        k_ap_tent<true><<<grid_for(m, 256), 256, 0, ctx->stream>>>(m, arp, acol, aval, agg, pt, C.rp.get(), nullptr,
                                                                   C.col.get(), C.val.get(), ctx->dev_flag, diag, w);
    OCP_LAUNCH_CHECK();
    return diag != nullptr;
}

// --------------------------------------------------------------- transpose
// Column counts and the scatter of the transpose, 256 rows per block.  When
// the block's rows hold at most kTHash/2 entries and none more than kTRow,
// the block first combines its entries per column in an LDS hash table, so
// one global atomic per distinct column and block reserves the space (rows of
// an aggregation operator share few columns); otherwise every entry takes
// its own global atomic.  The order inside a transposed row is fixed by the
// sort that follows.
constexpr int kTHash = 4096;
constexpr int kTRow = 16;

__device__ __forceinline__ int t_slot(int *keys, int v) {
    int s = (int)(((uint32_t)v * 2654435761u) >> (32 - 12));
    for (;;) {
        const int prev = atomicCAS(&keys[s], -1, v);
        if (prev == -1 || prev == v) return s;
        s = (s + 1) & (kTHash - 1);
    }
}

__device__ __forceinline__ bool t_combine(int32_t m, const int32_t *__restrict__ rp, int r0) {
    const int r1 = r0 + 256 < m ? r0 + 256 : m;
    const int i = r0 + (int)threadIdx.x;
    const bool longrow = i < m && rp[i + 1] - rp[i] > kTRow;
    return !__syncthreads_or(longrow) && rp[r1] - rp[r0] <= kTHash / 2;
}

__global__ void __launch_bounds__(256) k_count_cols(int32_t m, const int32_t *__restrict__ rp,
                                                    const int32_t *__restrict__ col, int32_t *__restrict__ cnt) {
    __shared__ int keys[kTHash];
    __shared__ int c[kTHash];
    const int r0 = blockIdx.x * 256;
    const bool combine = t_combine(m, rp, r0);   // uniform over the block
    const int i = r0 + (int)threadIdx.x;
    if (combine) {
        for (int q = threadIdx.x; q < kTHash; q += 256) {
            keys[q] = -1;
            c[q] = 0;
        }
        __syncthreads();
        if (i < m)
            for (int k = rp[i]; k < rp[i + 1]; ++k) atomicAdd(&c[t_slot(keys, col[k])], 1);
        __syncthreads();
        for (int q = threadIdx.x; q < kTHash; q += 256)
            if (keys[q] >= 0) atomicAdd(&cnt[keys[q]], c[q]);
    } else if (i < m) {
        for (int k = rp[i]; k < rp[i + 1]; ++k) atomicAdd(&cnt[col[k]], 1);
    }
}

__global__ void __launch_bounds__(256) k_fill_t(int32_t m, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ col, const double *__restrict__ val,
                                                const int32_t *__restrict__ trp, int32_t *__restrict__ fill,
                                                int32_t *__restrict__ tcol, double *__restrict__ tval) {
    __shared__ int keys[kTHash];
    __shared__ int c[kTHash];
    __shared__ int base[kTHash];
    const int r0 = blockIdx.x * 256;
    const bool combine = t_combine(m, rp, r0);   // uniform over the block
    const int i = r0 + (int)threadIdx.x;
    if (!combine) {
        if (i < m)
            for (int k = rp[i]; k < rp[i + 1]; ++k) {
                const int j = col[k];
                const int pos = trp[j] + atomicAdd(&fill[j], 1);
                tcol[pos] = i;
                tval[pos] = val[k];
            }
        return;
    }
    for (int q = threadIdx.x; q < kTHash; q += 256) {
        keys[q] = -1;
        c[q] = 0;
    }
    __syncthreads();
    int slot[kTRow], pos[kTRow];
    const int kb = i < m ? rp[i] : 0, len = i < m ? rp[i + 1] - kb : 0;
#pragma unroll
    for (int u = 0; u < kTRow; ++u)
        if (u < len) {
            slot[u] = t_slot(keys, col[kb + u]);
            pos[u] = atomicAdd(&c[slot[u]], 1);
        }
    __syncthreads();
    for (int q = threadIdx.x; q < kTHash; q += 256)
        if (keys[q] >= 0) base[q] = trp[keys[q]] + atomicAdd(&fill[keys[q]], c[q]);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kTRow; ++u)
        if (u < len) {
            const int p = base[slot[u]] + pos[u];
            tcol[p] = i;
            tval[p] = val[kb + u];
        }
}

constexpr int kSortCap = 2048;
constexpr int kSortWave = 256;   // rows up to this length are sorted by one wavefront

// Sort each row of at most kSortWave entries by column, one wavefront per
// row (4 per block), rank sort in the wavefront's LDS slice.  Longer rows are
// left to k_sort_rows (flag bit 1 of *longrows).
__global__ void __launch_bounds__(256) k_sort_rows_wave(int32_t m, const int32_t *__restrict__ rp,
                                                        int32_t *__restrict__ col, double *__restrict__ val,
                                                        int32_t *longrows) {
    __shared__ int keys[4][kSortWave];
    __shared__ double vals[4][kSortWave];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + wv;
    if (i >= m) return;   // uniform over the wavefront
    const int b = rp[i], len = rp[i + 1] - b;
    if (len > kSortWave) {
        if (lane == 0) atomicOr(longrows, 1);
        return;
    }
    for (int e = lane; e < len; e += 64) {
        keys[wv][e] = col[b + e];
        vals[wv][e] = val[b + e];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int e = lane; e < len; e += 64) {
        const int ke = keys[wv][e];
        int rank = 0;
        for (int f = 0; f < len; ++f) rank += keys[wv][f] < ke;
        col[b + rank] = ke;
        val[b + rank] = vals[wv][e];
    }
}

// Sort each row by column (keys unique within a row): rank sort in LDS.
__global__ void __launch_bounds__(256) k_sort_rows(int32_t m, const int32_t *__restrict__ rp, int32_t *__restrict__ col,
                                                   double *__restrict__ val, int32_t *flag) {
    __shared__ int keys[kSortCap];
    __shared__ double vals[kSortCap];
    for (int i = blockIdx.x; i < m; i += gridDim.x) {
        const int b = rp[i], len = rp[i + 1] - b;
        if (len <= kSortWave) continue;   // sorted by k_sort_rows_wave
        if (len > kSortCap) {
            if (threadIdx.x == 0) atomicOr(flag, 64);
            continue;
        }
        for (int e = threadIdx.x; e < len; e += blockDim.x) {
            keys[e] = col[b + e];
            vals[e] = val[b + e];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < len; e += blockDim.x) {
            const int ke = keys[e];
            int rank = 0;
            for (int f = 0; f < len; ++f) rank += keys[f] < ke;
            col[b + rank] = ke;
            val[b + rank] = vals[e];
        }
        __syncthreads();
    }
}

static void transpose(ocp_ctx *ctx, int32_t m, int32_t ncols, int64_t nnz, const int32_t *rp, const int32_t *col,
                      const double *val, Csr &T) {
    hipStream_t s = ctx->stream;
    DevBuf<int32_t> cnt(ctx, (size_t)ncols + 1);
    fill_zero_bytes(ctx, cnt.get(), sizeof(int32_t) * ((size_t)ncols + 1));
    k_count_cols<<<grid_for(m, 256), 256, 0, s>>>(m, rp, col, cnt.get());
    OCP_LAUNCH_CHECK();
    T.rows = ncols;
    T.cols = m;
    T.rp.reset(ctx, (size_t)ncols + 1);
    T.nnz = scan_exclusive(ctx, cnt.get(), T.rp.get(), ncols);
    T.col.reset(ctx, (size_t)std::max<int64_t>(T.nnz, 1));
    T.val.reset(ctx, (size_t)std::max<int64_t>(T.nnz, 1));
    fill_zero_bytes(ctx, cnt.get(), sizeof(int32_t) * ((size_t)ncols + 1));
    k_fill_t<<<grid_for(m, 256), 256, 0, s>>>(m, rp, col, val, T.rp.get(), cnt.get(), T.col.get(), T.val.get());
    OCP_LAUNCH_CHECK();
    fill_zero_bytes(ctx, ctx->dev_flag, 4);
    k_sort_rows_wave<<<(unsigned)((std::max<int32_t>(ncols, 1) + 3) / 4), 256, 0, s>>>(ncols, T.rp.get(), T.col.get(),
                                                                                  T.val.get(), ctx->dev_flag);
    OCP_LAUNCH_CHECK();
    int32_t fl = 0;
    read_back(ctx, &fl, ctx->dev_flag, 4);
    if (fl & 1) {   // some rows are longer than a wavefront's slice: sort those by blocks
        fill_zero_bytes(ctx, ctx->dev_flag, 4);
        k_sort_rows<<<(unsigned)std::min<int64_t>(std::max<int32_t>(ncols, 1), 65536), 256, 0, s>>>(
            ncols, T.rp.get(), T.col.get(), T.val.get(), ctx->dev_flag);
        OCP_LAUNCH_CHECK();
        read_back(ctx, &fl, ctx->dev_flag, 4);
        if (fl & 64) fail(OCP_ERR_UNSUPPORTED, "transpose row with more than 2048 entries");
    }
}

// ------------------------------------------------------------ dense inverse
__global__ void k_csr_to_dense(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                               const double *__restrict__ val, double *__restrict__ D) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = rp[i]; k < rp[i + 1]; ++k) D[(int64_t)i * n + col[k]] = val[k];
}

// Gauss-Jordan inversion of an SPD matrix (no pivoting needed), one launch
// per elimination step k over the whole n x n matrix, reading the previous
// step's matrix A and writing B (two buffers, so no block overwrites the
// pivot row or column that another block still reads):
//   B[k][k] = 1/a_kk,  B[k][j] = a_kj / a_kk,  B[i][k] = -a_ik / a_kk,
//   B[i][j] = a_ij - a_ik (a_kj / a_kk).
__global__ void __launch_bounds__(256) k_gj_step(int32_t n, int32_t k, const double *__restrict__ A,
                                                 double *__restrict__ B) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
    const double p = 1.0 / A[(int64_t)k * n + k];
    const double rkj = A[(int64_t)k * n + j] * p;
    double v;
    if (i == k)
        v = (j == k) ? p : rkj;
    else
        v = (j == k) ? -A[(int64_t)i * n + k] * p : A[e] - A[(int64_t)i * n + k] * rkj;
    B[e] = v;
}

static void dense_inverse(ocp_ctx *ctx, int32_t n, double *D) {
    DevBuf<double> tmp(ctx, (size_t)n * n);
    double *a = D, *b = tmp.get();
    const unsigned g = grid_for((int64_t)n * n, 256);
    for (int k = 0; k < n; ++k) {
        k_gj_step<<<g, 256, 0, ctx->stream>>>(n, k, a, b);
        std::swap(a, b);
    }
    OCP_LAUNCH_CHECK();
    if (a != D) OCP_HIP(hipMemcpyAsync(D, a, sizeof(double) * n * n, hipMemcpyDeviceToDevice, ctx->stream));
    sync(ctx);   // tmp is released on return
}

__global__ void k_to_float(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

static void to_float(ocp_ctx *ctx, const double *a, DevBuf<float> &b, int64_t n) {
    b.reset(ctx, (size_t)std::max<int64_t>(n, 1));
    if (n > 0) {
        k_to_float<<<grid_for(n, 256), 256, 0, ctx->stream>>>(n, a, b.get());
        OCP_LAUNCH_CHECK();
    }
}

// ------------------------------------------------------------------- setup
// ------------------------------------------------------ red-black method
// Section 3.1: red-black colouring coarsening.  Sequentially: pick an
// unmarked dof, mark it black (coarse) and its unmarked neighbours red
// (fine), until every dof is marked.  With the dofs picked in decreasing
// order of a fixed key (the hash priority of the aggregation, ties by index)
// the result is the independent set that parallel rounds produce: in a round
// an undecided dof whose key exceeds every undecided neighbour's turns
// coarse (k_rb_pick), and then every undecided neighbour of a new coarse dof
// turns fine (k_rb_mark).  The pick is written to its own array so that no
// dof reads a state another dof of the same round changes.
__device__ __forceinline__ uint64_t rb_key(int i, uint32_t salt) {
    return ((uint64_t)(mix32((uint32_t)i ^ salt) >> 2) << 32) | (uint32_t)i;
}

template <int G>
__global__ void __launch_bounds__(256) k_rb_pick(int32_t n, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col, const uint8_t *__restrict__ strong,
                                                 const int8_t *__restrict__ state, uint32_t salt, int32_t round,
                                                 const int32_t *__restrict__ prev_undecided, int32_t *__restrict__ pick) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / G), lane = (int)(t % G);
    if (i >= n) return;
    if (prev_undecided && *prev_undecided == 0) return;
    if (state[i] != 0) return;   // uniform over the group
    const uint64_t ki = rb_key(i, salt);
    int beaten = 0;
    for (int k = rp[i] + lane; k < rp[i + 1]; k += G) {
        const int j = col[k];
        if (is_strong(strong, k, j, i) && state[j] == 0 && rb_key(j, salt) > ki) beaten = 1;
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) beaten |= __shfl_xor(beaten, o, G);
    if (lane == 0 && !beaten) pick[i] = round;
}

template <int G>
__global__ void __launch_bounds__(256) k_rb_mark(int32_t n, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col, const uint8_t *__restrict__ strong,
                                                 int8_t *__restrict__ state, const int32_t *__restrict__ pick,
                                                 int32_t round, const int32_t *__restrict__ prev_undecided,
                                                 int32_t *undecided) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / G), lane = (int)(t % G);
    if (i >= n) return;
    if (prev_undecided && *prev_undecided == 0) return;
    if (state[i] != 0) return;   // uniform over the group
    const bool black = pick[i] == round;
    int red = 0;
    if (!black)
        for (int k = rp[i] + lane; k < rp[i + 1]; k += G) {
            const int j = col[k];
            if (is_strong(strong, k, j, i) && pick[j] == round) red = 1;
        }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) red |= __shfl_xor(red, o, G);
    if (lane == 0) {
        if (black)
            state[i] = 1;
        else if (red)
            state[i] = 2;
    }
    const bool still = lane == 0 && !black && !red;
    const unsigned long long any = __ballot(still);
    if (any != 0ull && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)any) - 1)) *undecided = 1;
}

// Interpolation by averaging (Section 3.1): a coarse dof keeps its value
// (P[i, c(i)] = 1); a fine dof takes the mean of its coarse strong
// neighbours (P[i, c(j)] = 1 / #coarse neighbours).  cidx[j] = coarse number
// of a coarse dof (ascending in j, so each row's columns are sorted).
__global__ void k_rb_p_len(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const uint8_t *__restrict__ strong, const int8_t *__restrict__ state,
                           int32_t *__restrict__ len, int32_t *flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    if (state[i] == 1) {
        c = 1;
    } else {
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int j = col[k];
            if (is_strong(strong, k, j, i) && state[j] == 1) ++c;
        }
        if (c == 0) atomicOr(flag, 32);   // a fine dof without a coarse neighbour (not maximal)
    }
    len[i] = c;
}

__global__ void k_rb_p_fill(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                            const uint8_t *__restrict__ strong, const int8_t *__restrict__ state,
                            const int32_t *__restrict__ cidx, const int32_t *__restrict__ prp,
                            int32_t *__restrict__ pcol, double *__restrict__ pval, int32_t *__restrict__ agg) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int o = prp[i];
    if (state[i] == 1) {
        pcol[o] = cidx[i];
        pval[o] = 1.0;
        agg[i] = cidx[i];
        return;
    }
    agg[i] = -1;
    const double w = 1.0 / (double)(prp[i + 1] - o);
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
        const int j = col[k];
        if (is_strong(strong, k, j, i) && state[j] == 1) {
            pcol[o] = cidx[j];
            pval[o] = w;
            ++o;
        }
    }
}

// Colouring of a level's graph (every off-diagonal entry couples) for the
// Gauss-Seidel sweeps: colour c is the independent set that round c picks
// among the uncoloured rows, each joining when its key exceeds every
// uncoloured neighbour's.
template <int G>
__global__ void __launch_bounds__(256) k_col_pick(int32_t n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ col, const int32_t *__restrict__ color,
                                                  uint32_t salt, int32_t round,
                                                  const int32_t *__restrict__ prev_uncoloured,
                                                  int32_t *__restrict__ pick) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t / G), lane = (int)(t % G);
    if (i >= n) return;
    if (prev_uncoloured && *prev_uncoloured == 0) return;
    if (color[i] >= 0) return;
    const uint64_t ki = rb_key(i, salt);
    int beaten = 0;
    for (int k = rp[i] + lane; k < rp[i + 1]; k += G) {
        const int j = col[k];
        if (j != i && color[j] < 0 && rb_key(j, salt) > ki) beaten = 1;
    }
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) beaten |= __shfl_xor(beaten, o, G);
    if (lane == 0 && !beaten) pick[i] = round;
}

__global__ void k_col_mark(int32_t n, int32_t *__restrict__ color, const int32_t *__restrict__ pick, int32_t round,
                           const int32_t *__restrict__ prev_uncoloured, int32_t *uncoloured) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (prev_uncoloured && *prev_uncoloured == 0) return;
    if (color[i] >= 0) return;
    bool still = true;
    if (pick[i] == round) {
        color[i] = round;
        still = false;
    }
    const unsigned long long any = __ballot(still);
    if (any != 0ull && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)any) - 1)) *uncoloured = 1;
}

__global__ void k_fill_i32(int64_t n, int32_t v, int32_t *__restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// rows grouped by colour, ascending within a colour: per tile of kColTile
// rows its count of each colour (cnt[c * ntiles + tile]); after a scan of
// cnt the tiles place their rows in order
constexpr int kColTile = 64;
__global__ void k_col_count(int32_t n, int32_t ncolors, const int32_t *__restrict__ color, int32_t ntiles,
                            int32_t *__restrict__ cnt) {
    const int tile = blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= ntiles) return;
    const int r0 = tile * kColTile, r1 = r0 + kColTile < n ? r0 + kColTile : n;
    for (int c = 0; c < ncolors; ++c) cnt[(int64_t)c * ntiles + tile] = 0;
    for (int i = r0; i < r1; ++i) ++cnt[(int64_t)color[i] * ntiles + tile];
}

__global__ void k_col_scatter(int32_t n, const int32_t *__restrict__ color, int32_t ntiles,
                              int32_t *__restrict__ off, int32_t *__restrict__ rows) {
    const int tile = blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= ntiles) return;
    const int r0 = tile * kColTile, r1 = r0 + kColTile < n ? r0 + kColTile : n;
    for (int i = r0; i < r1; ++i) rows[off[(int64_t)color[i] * ntiles + tile]++] = i;
}

__global__ void k_col_starts(int32_t ncolors, int32_t ntiles, const int32_t *__restrict__ off,
                             int32_t *__restrict__ starts) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncolors) starts[c] = off[(int64_t)c * ntiles];
}

constexpr int kMaxColors = 1000;   // colour offsets come back through the 4 KiB staging buffer

// Colour level L's graph and group its rows by colour.
static void colour_level(ocp_ctx *ctx, Level &L, uint32_t salt) {
    hipStream_t s = ctx->stream;
    const int32_t n = L.n;
    DevBuf<int32_t> color(ctx, (size_t)n), pick(ctx, (size_t)n), unc(ctx, (size_t)kMaxColors + 1);
    k_fill_i32<<<grid_for(n, 256), 256, 0, s>>>(n, -1, color.get());
    k_fill_i32<<<grid_for(n, 256), 256, 0, s>>>(n, -1, pick.get());
    fill_zero_bytes(ctx, unc.get(), sizeof(int32_t) * ((size_t)kMaxColors + 1));
    constexpr int G = 4;
    const unsigned gb = grid_for((int64_t)n * G, 256);
    // unc[c + 1] = 1 when rows are still uncoloured after round c
    int ncol = -1, batch = 4;
    for (int c = 0; ncol < 0;) {
        const int last = std::min(c + batch, kMaxColors);
        for (; c < last; ++c) {
            const int32_t *prev = c == 0 ? nullptr : unc.get() + c;
            k_col_pick<G><<<gb, 256, 0, s>>>(n, L.A_rp, L.A_col, color.get(), salt, c, prev, pick.get());
            k_col_mark<<<grid_for(n, 256), 256, 0, s>>>(n, color.get(), pick.get(), c, prev, unc.get() + c + 1);
        }
        OCP_LAUNCH_CHECK();
        int32_t flag = 0;
        read_back(ctx, &flag, unc.get() + last, sizeof(int32_t));
        if (flag == 0) {
            std::vector<int32_t> h((size_t)last + 1);
            read_back(ctx, h.data(), unc.get(), sizeof(int32_t) * h.size());
            ncol = last;
            for (int k = 1; k <= last; ++k)
                if (h[k] == 0) {
                    ncol = k;   // rounds 0 .. k-1 coloured every row
                    break;
                }
        } else if (last >= kMaxColors) {
            fail(OCP_ERR_UNSUPPORTED, "the Gauss-Seidel colouring needs more than 1000 colours");
        }
        batch = std::min(batch * 2, 16);
    }
    const int32_t ntiles = (n + kColTile - 1) / kColTile;
    DevBuf<int32_t> cnt(ctx, (size_t)ncol * ntiles + 1), off(ctx, (size_t)ncol * ntiles + 1);
    k_col_count<<<grid_for(ntiles, 256), 256, 0, s>>>(n, ncol, color.get(), ntiles, cnt.get());
    OCP_LAUNCH_CHECK();
    scan_exclusive(ctx, cnt.get(), off.get(), (int64_t)ncol * ntiles);
    DevBuf<int32_t> starts(ctx, (size_t)ncol);
    k_col_starts<<<grid_for(ncol, 256), 256, 0, s>>>(ncol, ntiles, off.get(), starts.get());
    L.color_rows.reset(ctx, (size_t)n);
    k_col_scatter<<<grid_for(ntiles, 256), 256, 0, s>>>(n, color.get(), ntiles, off.get(), L.color_rows.get());
    OCP_LAUNCH_CHECK();
    L.ncolors = ncol;
    L.color_ptr.assign((size_t)ncol + 1, n);
    read_back(ctx, L.color_ptr.data(), starts.get(), sizeof(int32_t) * (size_t)ncol);
}

// Levels of the red-black method, appended to h (level 0 already there).
static void redblack_levels(ocp_ctx *ctx, const ocp_system *sys, ocp_hierarchy *h) {
    (void)sys;
    hipStream_t s = ctx->stream;
    const ocp_amg_params &pr = h->params;
    for (int lev = 0;; ++lev) {
        Level &L = *h->levels.back();
        const int32_t n = L.n;
        L.gA = level_lanes(L.nnzA, n);
        DevBuf<double> diag(ctx, n), gersh(ctx, n), dl1(ctx, n);
        fill_zero_bytes(ctx, ctx->dev_flag, 4);
        k_level_diag<<<grid_for(n, 256), 256, 0, s>>>(n, L.A_rp, L.A_col, L.A_val, diag.get(), dl1.get(), gersh.get(),
                                                      ctx->dev_flag);
        OCP_LAUNCH_CHECK();
        int32_t fl = 0;
        read_back(ctx, &fl, ctx->dev_flag, 4);
        if (fl & 8) fail(OCP_ERR_INVALID_ARG, "matrix has a non-positive diagonal entry");
        L.lambda_max = reduce_max_abs(ctx, gersh.get(), n);
        L.dinv.reset(ctx, n);   // 1 / a_ii for the Gauss-Seidel updates
        k_recip<<<grid_for(n, 256), 256, 0, s>>>(n, diag.get(), L.dinv.get());
        OCP_LAUNCH_CHECK();
        L.deg = 1;
        const uint32_t salt = 0x9E3779B9u * (uint32_t)(lev + 1);
        const bool last = (n <= pr.coarse_max) || (lev + 1 >= pr.max_levels);
        if (!last) colour_level(ctx, L, salt ^ 0x5bd1e995u);
        int32_t nc = 0;
        DevBuf<uint8_t> strong;
        DevBuf<int8_t> state;
        if (!last) {
            if (pr.theta > 0.0) {
                strong.reset(ctx, (size_t)L.nnzA);
                k_strength<<<grid_for(n, 256), 256, 0, s>>>(n, L.A_rp, L.A_col, L.A_val, diag.get(), pr.theta,
                                                            strong.get());
                OCP_LAUNCH_CHECK();
            }
            state.reset(ctx, (size_t)n);
            fill_zero_bytes(ctx, state.get(), (size_t)n);
            DevBuf<int32_t> pick(ctx, (size_t)n), undec(ctx, (size_t)kMisMaxRounds + 1);
            fill_zero_bytes(ctx, pick.get(), sizeof(int32_t) * (size_t)n);
            fill_zero_bytes(ctx, undec.get(), sizeof(int32_t) * ((size_t)kMisMaxRounds + 1));
            constexpr int G = 4;
            const unsigned gb = grid_for((int64_t)n * G, 256);
            int batch = 4;
            for (int round = 1;;) {
                const int lastr = std::min(round + batch - 1, kMisMaxRounds);
                for (; round <= lastr; ++round) {
                    const int32_t *prev = round == 1 ? nullptr : undec.get() + round - 1;
                    k_rb_pick<G><<<gb, 256, 0, s>>>(n, L.A_rp, L.A_col, strong.get(), state.get(), salt, round, prev,
                                                    pick.get());
                    k_rb_mark<G><<<gb, 256, 0, s>>>(n, L.A_rp, L.A_col, strong.get(), state.get(), pick.get(), round,
                                                    prev, undec.get() + round);
                }
                OCP_LAUNCH_CHECK();
                int32_t und = 0;
                read_back(ctx, &und, undec.get() + lastr, sizeof(int32_t));
                if (und == 0) break;
                if (lastr >= kMisMaxRounds) fail(OCP_ERR_HIP, "red-black colouring rounds did not terminate");
                batch = std::min(batch * 2, 16);
            }
            DevBuf<int32_t> rflag(ctx, (size_t)n + 1);
            L.agg.reset(ctx, n);   // coarse number of a coarse dof, -1 for a fine one
            k_root_flags<<<grid_for(n, 256), 256, 0, s>>>(n, state.get(), rflag.get());
            OCP_LAUNCH_CHECK();
            DevBuf<int32_t> cidx(ctx, (size_t)n + 1);
            nc = (int32_t)scan_exclusive(ctx, rflag.get(), cidx.get(), n);
            if (!(last || nc <= 0 || 2 * (int64_t)nc > n)) {
                Csr P;
                P.rows = n;
                P.cols = nc;
                DevBuf<int32_t> len(ctx, (size_t)n + 1);
                fill_zero_bytes(ctx, ctx->dev_flag, 4);
                k_rb_p_len<<<grid_for(n, 256), 256, 0, s>>>(n, L.A_rp, L.A_col, strong.get(), state.get(), len.get(),
                                                            ctx->dev_flag);
                OCP_LAUNCH_CHECK();
                read_back(ctx, &fl, ctx->dev_flag, 4);
                if (fl & 32) fail(OCP_ERR_HIP, "a fine dof has no coarse neighbour");
                P.rp.reset(ctx, (size_t)n + 1);
                P.nnz = scan_exclusive(ctx, len.get(), P.rp.get(), n);
                P.col.reset(ctx, (size_t)P.nnz);
                P.val.reset(ctx, (size_t)P.nnz);
                k_rb_p_fill<<<grid_for(n, 256), 256, 0, s>>>(n, L.A_rp, L.A_col, strong.get(), state.get(), cidx.get(),
                                                             P.rp.get(), P.col.get(), P.val.get(), L.agg.get());
                OCP_LAUNCH_CHECK();
                Csr R;
                transpose(ctx, n, nc, P.nnz, P.rp.get(), P.col.get(), P.val.get(), R);
                Csr AP, Ac;
                spgemm(ctx, n, nc, L.nnzA, L.A_rp, L.A_col, L.A_val, P.rp.get(), P.col.get(), P.val.get(), AP);
                spgemm(ctx, nc, nc, P.nnz, R.rp.get(), R.col.get(), R.val.get(), AP.rp.get(), AP.col.get(),
                       AP.val.get(), Ac);
                sync(ctx);
                L.nc = nc;
                L.nnzP = P.nnz;
                L.P_rp = std::move(P.rp);
                L.P_col = std::move(P.col);
                L.P_val = std::move(P.val);
                L.R_rp = std::move(R.rp);
                L.R_col = std::move(R.col);
                L.R_val = std::move(R.val);
                L.gP = level_lanes(L.nnzP, n);
                L.gR = level_lanes(L.nnzP, nc);
                L.maxP = csr_max_row(ctx, n, L.P_rp.get());
                auto nxt = std::make_unique<Level>();
                nxt->n = nc;
                nxt->nnzA = Ac.nnz;
                nxt->own_rp = std::move(Ac.rp);
                nxt->own_col = std::move(Ac.col);
                nxt->own_val = std::move(Ac.val);
                nxt->A_rp = nxt->own_rp.get();
                nxt->A_col = nxt->own_col.get();
                nxt->A_val = nxt->own_val.get();
                h->levels.push_back(std::move(nxt));
                continue;
            }
        }
        // last level: dense inverse (or Gauss-Seidel sweeps alone when too large)
        L.agg.release();
        if (n <= kDenseMax) {
            L.dense_inv.reset(ctx, (size_t)n * n);
            fill_zero_bytes(ctx, L.dense_inv.get(), sizeof(double) * (size_t)n * n);
            k_csr_to_dense<<<grid_for(n, 256), 256, 0, s>>>(n, L.A_rp, L.A_col, L.A_val, L.dense_inv.get());
            OCP_LAUNCH_CHECK();
            dense_inverse(ctx, n, L.dense_inv.get());
        } else if (L.ncolors == 0) {
            colour_level(ctx, L, salt ^ 0x5bd1e995u);
        }
        break;
    }
}

static void setup(ocp_ctx *ctx, const ocp_system *sys, ocp_hierarchy *h) {
    hipStream_t s = ctx->stream;
    const ocp_amg_params &pr = h->params;
    auto l0 = std::make_unique<Level>();
    l0->n = sys->n;
    l0->nnzA = sys->nnz;
    l0->A_rp = sys->row_ptr.get();
    l0->A_col = sys->col.get();
    l0->A_val = sys->val.get();
    h->levels.push_back(std::move(l0));

    if (pr.method == OCP_AMG_REDBLACK) redblack_levels(ctx, sys, h);
    else for (int lev = 0;; ++lev) {
        Level &L = *h->levels.back();
        const int32_t n = L.n;
        L.gA = level_lanes(L.nnzA, n);
        DevBuf<double> diag(ctx, n), gersh(ctx, n), dl1(ctx, n);
        fill_zero_bytes(ctx, ctx->dev_flag, 4);
        if (lev == 0 && sys->sell.col.get() && sys->sell.n == n) {
            const Sell &S = sys->sell;
            const SellLaunch LS = sell_launch(S.nslices);
            k_level_diag_sell<<<LS.blocks, kBlock, 0, s>>>(n, S.nslices, LS.slices_per_block, S.sp.get(),
                                                            S.sw.get(), sell_cols(S), S.val.get(), diag.get(),
                                                            dl1.get(), gersh.get(), ctx->dev_flag);
        } else {
            k_level_diag<<<grid_for(n, 256), 256, 0, s>>>(n, L.A_rp, L.A_col, L.A_val, diag.get(), dl1.get(),
                                                          gersh.get(), ctx->dev_flag);
        }
        OCP_LAUNCH_CHECK();
        int32_t fl = 0;
        read_back(ctx, &fl, ctx->dev_flag, 4);
        if (fl & 8) fail(OCP_ERR_INVALID_ARG, "matrix has a non-positive diagonal entry");
        L.lambda_max = reduce_max_abs(ctx, gersh.get(), n);
        // smoother diagonal and polynomial coefficients
        if (pr.smoother == OCP_SMOOTH_CHEBYSHEV) {
            L.dinv.reset(ctx, n);
            k_recip<<<grid_for(n, 256), 256, 0, s>>>(n, diag.get(), L.dinv.get());
            OCP_LAUNCH_CHECK();
            const double lmax = L.lambda_max, lmin = lmax / pr.cheb_ratio;
            const double th = 0.5 * (lmax + lmin), de = 0.5 * (lmax - lmin);
            const double sg = th / de, r1 = 1.0 / sg, r2 = 1.0 / (2.0 * sg - r1);
            L.deg = pr.degree;
            L.cheb_a = 1.0 / th;
            L.cheb_c1 = (1.0 + r2 * r1) / th;
            L.cheb_c2 = 2.0 * r2 / de;
        } else {
            L.dinv = std::move(dl1);
            L.deg = 1;
            L.cheb_a = 1.0;
        }

        const bool last = (n <= pr.coarse_max) || (lev + 1 >= pr.max_levels);
        int32_t nc = 0;
        DevBuf<uint8_t> strong;
        if (!last) {
            // strength and distance-2 maximal independent set
            if (pr.theta > 0.0) {
                strong.reset(ctx, (size_t)L.nnzA);
                k_strength<<<grid_for(n, 256), 256, 0, s>>>(n, L.A_rp, L.A_col, L.A_val, diag.get(), pr.theta,
                                                            strong.get());
                OCP_LAUNCH_CHECK();
            }
            DevBuf<int8_t> state(ctx, n);
            fill_zero_bytes(ctx, state.get(), (size_t)n);
            DevBuf<uint64_t> m1(ctx, n);
            DevBuf<int32_t> need(ctx, n);
            fill_zero_bytes(ctx, need.get(), sizeof(int32_t) * (size_t)n);
            const uint32_t salt = 0x9E3779B9u * (uint32_t)(lev + 1);
            constexpr int GM = 4;
            const unsigned gb = grid_for((int64_t)n * GM, 256);
            // level 0 with every entry strong: the full rounds walk the
            // system's sliced-ELL copy
            const bool sell0 = lev == 0 && !strong.get() && sys->sell.col.get() && sys->sell.n == n;
            const SellLaunch LS0 = sell_launch(sell0 ? sys->sell.nslices : 1);
            // undec[r] = 1 when some node is still undecided after round r
            // (r = 1..kMisMaxRounds).  Rounds are enqueued in batches between
            // host reads of the flag of a batch's last round; the kernels of a
            // round after the one that decided every node return at once.
            DevBuf<int32_t> undec(ctx, (size_t)kMisMaxRounds + 1);
            fill_zero_bytes(ctx, undec.get(), sizeof(int32_t) * ((size_t)kMisMaxRounds + 1));
            int batch = 4;
            // once few nodes are undecided, the rounds run over a list of them
            DevBuf<int32_t> ulist;
            int32_t nlist = -1;
            for (int round = 1;;) {
                const int last = std::min(round + batch - 1, kMisMaxRounds);
                if (nlist >= 0) {
                    const unsigned gl = grid_for((int64_t)std::max(nlist, 1) * kMisListG, 256);
                    for (; round <= last; ++round) {
                        const int32_t *prev = undec.get() + round - 1;
                        k_mis_m1_list<<<gl, 256, 0, s>>>(ulist.get(), nlist, L.A_rp, L.A_col, strong.get(),
                                                         state.get(), salt, prev, m1.get());
                        k_mis_m2_list<<<gl, 256, 0, s>>>(ulist.get(), nlist, L.A_rp, L.A_col, strong.get(),
                                                         state.get(), salt, m1.get(), prev, undec.get() + round);
                    }
                }
                for (; round <= last; ++round) {
                    const int32_t *prev = round == 1 ? nullptr : undec.get() + round - 1;
                    int32_t *nd1 = round > kMisMarkFrom ? need.get() : nullptr;
                    int32_t *nd2 = round >= kMisMarkFrom ? need.get() : nullptr;
                    if (sell0) {
                        const Sell &S = sys->sell;
                        if (round == 1)
                            k_mis_m1_sell<true><<<LS0.blocks, kBlock, 0, s>>>(
                                n, S.nslices, LS0.slices_per_block, S.sp.get(), S.sw.get(), sell_cols(S),
                                state.get(), salt, nullptr, round, nullptr, m1.get());
                        else
                            k_mis_m1_sell<false><<<LS0.blocks, kBlock, 0, s>>>(
                                n, S.nslices, LS0.slices_per_block, S.sp.get(), S.sw.get(), sell_cols(S),
                                state.get(), salt, nd1, round, prev, m1.get());
                        k_mis_m2_sell<<<LS0.blocks, kBlock, 0, s>>>(n, S.nslices, LS0.slices_per_block, S.sp.get(),
                                                                    S.sw.get(), sell_cols(S), state.get(), salt,
                                                                    m1.get(), nd2, round, prev, undec.get() + round);
                        continue;
                    }
                    // the first rounds leave most nodes undecided: marking their
                    // neighbourhoods would cost more than the m1 work it skips,
                    // so m1 takes every node until the marks start
                    // round 1: every node undecided, no states to gather
                    if (round == 1)
                        k_mis_m1<GM, true><<<gb, 256, 0, s>>>(n, L.A_rp, L.A_col, strong.get(), state.get(), salt,
                                                              nullptr, round, nullptr, m1.get());
                    else
                        k_mis_m1<GM, false><<<gb, 256, 0, s>>>(n, L.A_rp, L.A_col, strong.get(), state.get(), salt,
                                                               nd1, round, prev, m1.get());
                    k_mis_m2<GM><<<gb, 256, 0, s>>>(n, L.A_rp, L.A_col, strong.get(), state.get(), salt, m1.get(), nd2,
                                                    round, prev, undec.get() + round);
                }
                OCP_LAUNCH_CHECK();
                int32_t und = 0;
                read_back(ctx, &und, undec.get() + last, sizeof(int32_t));
                if (und == 0) break;
                if (last >= kMisMaxRounds) fail(OCP_ERR_HIP, "independent-set rounds did not terminate");
                if (nlist < 0 && last >= kMisListFrom && n >= kMisListMinN) {
                    // few undecided nodes left: list them once
                    DevBuf<int32_t> fl(ctx, (size_t)n + 1), pos(ctx, (size_t)n + 1);
                    k_undecided_flags<<<grid_for(n, 256), 256, 0, s>>>(n, state.get(), fl.get());
                    OCP_LAUNCH_CHECK();
                    const int64_t cnt = scan_exclusive(ctx, fl.get(), pos.get(), n);
                    if (cnt * kMisListFrac <= n) {
                        nlist = (int32_t)cnt;
                        ulist.reset(ctx, (size_t)std::max<int64_t>(cnt, 1));
                        k_list_fill<<<grid_for(n, 256), 256, 0, s>>>(n, fl.get(), pos.get(), ulist.get());
                        OCP_LAUNCH_CHECK();
                    }
                }
                batch = std::min(batch * 2, 16);
            }
            // aggregates
            DevBuf<int32_t> rflag(ctx, (size_t)n + 1), rpos(ctx, (size_t)n + 1);
            k_root_flags<<<grid_for(n, 256), 256, 0, s>>>(n, state.get(), rflag.get());
            OCP_LAUNCH_CHECK();
            nc = (int32_t)scan_exclusive(ctx, rflag.get(), rpos.get(), n);
            L.agg.reset(ctx, n);
            DevBuf<int8_t> assigned(ctx, n);
            if (sell0) {
                const Sell &S = sys->sell;
                k_agg1_sell<<<LS0.blocks, kBlock, 0, s>>>(n, S.nslices, LS0.slices_per_block, S.sp.get(), S.sw.get(),
                                                          sell_cols(S), state.get(), rpos.get(), salt, L.agg.get(),
                                                          assigned.get());
                fill_zero_bytes(ctx, ctx->dev_flag, 4);
                k_agg2_sell<<<LS0.blocks, kBlock, 0, s>>>(n, S.nslices, LS0.slices_per_block, S.sp.get(), S.sw.get(),
                                                          sell_cols(S), assigned.get(), salt, L.agg.get(),
                                                          ctx->dev_flag);
            } else {
                k_agg1<<<grid_for(n, 256), 256, 0, s>>>(n, L.A_rp, L.A_col, strong.get(), state.get(), rpos.get(),
                                                        salt, L.agg.get(), assigned.get());
                fill_zero_bytes(ctx, ctx->dev_flag, 4);
                k_agg2<<<grid_for(n, 256), 256, 0, s>>>(n, L.A_rp, L.A_col, strong.get(), assigned.get(), salt,
                                                        L.agg.get(), ctx->dev_flag);
            }
            OCP_LAUNCH_CHECK();
            read_back(ctx, &fl, ctx->dev_flag, 4);
            if (fl & 16) fail(OCP_ERR_HIP, "aggregation left a node unassigned");
        }
        // stop where aggregation no longer halves the level
        if (last || nc <= 0 || 2 * (int64_t)nc > n) {
            // last level: dense inverse (or Jacobi when too large)
            L.agg.release();
            if (n <= kDenseMax) {
                L.dense_inv.reset(ctx, (size_t)n * n);
                fill_zero_bytes(ctx, L.dense_inv.get(), sizeof(double) * (size_t)n * n);
                k_csr_to_dense<<<grid_for(n, 256), 256, 0, s>>>(n, L.A_rp, L.A_col, L.A_val, L.dense_inv.get());
                OCP_LAUNCH_CHECK();
                dense_inverse(ctx, n, L.dense_inv.get());
            }
            break;
        }

        // tentative prolongator
        DevBuf<int32_t> size(ctx, nc);
        fill_zero_bytes(ctx, size.get(), sizeof(int32_t) * (size_t)nc);
        k_agg_sizes<<<grid_for(n, 256), 256, 0, s>>>(n, L.agg.get(), size.get());
        DevBuf<int32_t> trp(ctx, (size_t)n + 1), tcol(ctx, n);
        DevBuf<double> tval(ctx, n);
        k_ptent<<<grid_for(n + 1, 256), 256, 0, s>>>(n, L.agg.get(), size.get(), trp.get(), tcol.get(), tval.get());
        OCP_LAUNCH_CHECK();
        // smoothed prolongator P = (I - w D^-1 A) P_tent
        Csr P;
        const double w = pr.omega / L.lambda_max;
        const Sell *sell = lev == 0 && sys->sell.col.get() && sys->sell.n == n ? &sys->sell : nullptr;
        if (!spgemm_ptent(ctx, n, nc, L.nnzA, L.A_rp, L.A_col, L.A_val, tcol.get(), trp.get(), tval.get(), P,
                          diag.get(), w, sell))
            k_smooth_p<<<grid_for(n, 256), 256, 0, s>>>(n, P.rp.get(), P.col.get(), P.val.get(), diag.get(),
                                                        L.agg.get(), tval.get(), w);
        OCP_LAUNCH_CHECK();
        // restriction and Galerkin product
        Csr R;
        transpose(ctx, n, nc, P.nnz, P.rp.get(), P.col.get(), P.val.get(), R);
        Csr Ac;
        // A P in padded 16-wide rows when A's rows are short on average
        // (their products rarely pass 16 columns), else in CSR
        if (L.nnzA <= 16 * (int64_t)n) {
            PadCsr AP;
            spgemm_small_rows(ctx, n, L.A_rp, L.A_col, L.A_val, P.rp.get(), P.col.get(), P.val.get(), AP);
            spgemm(ctx, nc, nc, P.nnz, R.rp.get(), R.col.get(), R.val.get(), AP.start.get(), AP.col.get(),
                   AP.val.get(), Ac, AP.len.get());
        } else {
            Csr AP;
            spgemm(ctx, n, nc, L.nnzA, L.A_rp, L.A_col, L.A_val, P.rp.get(), P.col.get(), P.val.get(), AP);
            spgemm(ctx, nc, nc, P.nnz, R.rp.get(), R.col.get(), R.val.get(), AP.rp.get(), AP.col.get(),
                   AP.val.get(), Ac);
        }
        sync(ctx);

        L.nc = nc;
        L.nnzP = P.nnz;
        L.P_rp = std::move(P.rp);
        L.P_col = std::move(P.col);
        L.P_val = std::move(P.val);
        L.R_rp = std::move(R.rp);
        L.R_col = std::move(R.col);
        L.R_val = std::move(R.val);
        L.gP = level_lanes(L.nnzP, n);
        L.gR = level_lanes(L.nnzP, nc);
        L.maxP = csr_max_row(ctx, n, L.P_rp.get());

        auto nxt = std::make_unique<Level>();
        nxt->n = nc;
        nxt->nnzA = Ac.nnz;
        nxt->own_rp = std::move(Ac.rp);
        nxt->own_col = std::move(Ac.col);
        nxt->own_val = std::move(Ac.val);
        nxt->A_rp = nxt->own_rp.get();
        nxt->A_col = nxt->own_col.get();
        nxt->A_val = nxt->own_val.get();
        h->levels.push_back(std::move(nxt));
    }

    // sliced-ELL copies of the larger coarse operators (their smoothing
    // passes then stream 64-row slices instead of one wide row group per row)
    for (size_t l = 1; l < h->levels.size() && pr.method == OCP_AMG_AGGREGATION; ++l) {
        Level &L = *h->levels[l];
        if (L.n >= kSellMinRows && !L.dense_inv.get()) sell_build(ctx, L.sell, L.n, L.A_rp, L.A_col, L.A_val);
    }
    // precision copies and work vectors
    const bool mixed = pr.precision == OCP_PREC_MIXED;
    for (size_t l = 0; l < h->levels.size(); ++l) {
        Level &L = *h->levels[l];
        if (mixed) {
            to_float(ctx, L.A_val, L.A_val32, L.nnzA);
            if (l == 0 && pr.method == OCP_AMG_AGGREGATION)
                sell_values32(ctx, system_sell(ctx, sys), L.A_rp, L.A_val32.get(), L.sell_val32);
            if (l > 0 && L.sell.col.get()) sell_values32(ctx, L.sell, L.A_rp, L.A_val32.get(), L.sell_val32);
            to_float(ctx, L.dinv.get(), L.dinv32, L.n);
            if (L.P_val.get()) to_float(ctx, L.P_val.get(), L.P_val32, L.nnzP);
            if (L.R_val.get()) to_float(ctx, L.R_val.get(), L.R_val32, L.nnzP);
            if (L.dense_inv.get()) to_float(ctx, L.dense_inv.get(), L.dense_inv32, (int64_t)L.n * L.n);
        }
    }
    sync(ctx);
}

}  // namespace ocp

using namespace ocp;

extern "C" void amg_default_params(ocp_amg_params *p) {
    if (!p) return;
    p->precision = OCP_PREC_FP64;
    p->smoother = OCP_SMOOTH_CHEBYSHEV;
    p->degree = 2;
    p->coarse_max = 512;
    p->max_levels = 10;
    p->theta = 0.0;
    p->omega = 1.9;
    p->cheb_ratio = 10.0;
    p->method = OCP_AMG_AGGREGATION;
}

extern "C" int amg_setup(ocp_ctx *ctx, const ocp_system *sys, const ocp_amg_params *params, ocp_hierarchy **out) {
    if (!ctx) return OCP_ERR_INVALID_ARG;
    if (out) *out = nullptr;
    ocp_hierarchy *h = nullptr;
    int rc = run_guarded(ctx, [&] {
        if (!sys || !out) fail(OCP_ERR_INVALID_ARG, "system and out must not be NULL");
        const auto t0 = std::chrono::steady_clock::now();
        h = new ocp_hierarchy();
        h->ctx = ctx;
        h->sys = sys;
        h->sys_generation = sys->generation.load(std::memory_order_acquire);
        if (params)
            h->params = *params;
        else
            amg_default_params(&h->params);
        const ocp_amg_params &p = h->params;
        if (p.method != OCP_AMG_AGGREGATION && p.method != OCP_AMG_REDBLACK) fail(OCP_ERR_INVALID_ARG, "unknown AMG method");
        if (p.precision != OCP_PREC_FP64 && p.precision != OCP_PREC_MIXED) fail(OCP_ERR_INVALID_ARG, "bad precision");
        if (p.smoother != OCP_SMOOTH_L1JACOBI && p.smoother != OCP_SMOOTH_CHEBYSHEV)
            fail(OCP_ERR_INVALID_ARG, "unknown smoother");
        if (p.smoother == OCP_SMOOTH_CHEBYSHEV && (p.degree < 1 || p.degree > 2))
            fail(OCP_ERR_UNSUPPORTED, "Chebyshev degree must be 1 or 2");
        if (p.smoother == OCP_SMOOTH_CHEBYSHEV && !(p.cheb_ratio > 1.0))
            fail(OCP_ERR_INVALID_ARG, "cheb_ratio must exceed 1");
        if (p.coarse_max < 1 || p.coarse_max > kDenseMax) fail(OCP_ERR_INVALID_ARG, "coarse_max must be in 1..2048");
        if (p.max_levels < 1 || p.max_levels > 16) fail(OCP_ERR_INVALID_ARG, "max_levels must be in 1..16");
        if (!(p.theta >= 0.0) || !(p.omega > 0.0)) fail(OCP_ERR_INVALID_ARG, "theta >= 0 and omega > 0 required");
        setup(ctx, sys, h);   // ends with a stream synchronization
        h->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    });
    if (rc != OCP_OK) {
        delete h;
        return rc;
    }
    *out = h;
    return OCP_OK;
}

extern "C" void ocp_hierarchy_destroy(ocp_hierarchy *h) { delete h; }

extern "C" int ocp_hierarchy_get_level(const ocp_hierarchy *h, int32_t level, ocp_level_view *v) {
    if (!h || !v || level < 0 || level >= (int32_t)h->levels.size()) return OCP_ERR_INVALID_ARG;
    const Level &L = *h->levels[level];
    v->n_levels = (int32_t)h->levels.size();
    v->level = level;
    v->n = L.n;
    v->n_coarse = L.nc;
    v->nnz_A = L.nnzA;
    v->nnz_P = L.nnzP;
    v->A_row_ptr = L.A_rp;
    v->A_col = L.A_col;
    v->A_val = L.A_val;
    v->P_row_ptr = L.P_rp.get();
    v->P_col = L.P_col.get();
    v->P_val = L.P_val.get();
    v->R_row_ptr = L.R_rp.get();
    v->R_col = L.R_col.get();
    v->R_val = L.R_val.get();
    v->agg = L.agg.get();
    v->dense_inv = L.dense_inv.get();
    v->lambda_max = L.lambda_max;
    return OCP_OK;
}
