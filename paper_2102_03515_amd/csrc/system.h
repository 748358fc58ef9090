// Library-side objects behind the opaque handles of the C interface: the
// assembled system and the AMG hierarchy.
#pragma once

#include <atomic>
#include <mutex>

#include "common.h"

namespace ocp {
// Sliced-ELL copy of the fine-level matrix (64-row slices, see kernels.h).
struct Sell {
    int32_t n = 0;
    int64_t nslices = 0;
    int64_t nnz_padded = 0;
    DevBuf<int32_t> sp;    // [nslices+1] element offset of each slice
    DevBuf<int32_t> sw;    // [nslices]   slice width
    DevBuf<int32_t> col;   // [nnz_padded]
    DevBuf<double> val;    // [nnz_padded]
    // Column codes, kept when every slice's column offsets (col - row) take
    // at most kSellDict distinct values: entry j of lane l of slice s has
    // column row + dict[s][c], c the 4-bit code j % 8 of dword
    // code[cp[s] + (j / 8) * 64 + l]; dict[s] is ascending.  Empty otherwise.
    DevBuf<uint32_t> code;   // [cp[nslices]]
    DevBuf<int32_t> cp;      // [nslices+1] dword offset of each slice
    DevBuf<int32_t> dict;    // [nslices][kSellDict]
};
void sell_build(ocp_ctx *ctx, Sell &S, int32_t n, const int32_t *rp, const int32_t *col, const double *val);
void sell_layout(ocp_ctx *ctx, Sell &S, int32_t n, const int32_t *rp);
void sell_codes(ocp_ctx *ctx, Sell &S);
void sell_code_layout(ocp_ctx *ctx, Sell &S);
void sell_code_finish(ocp_ctx *ctx, Sell &S);
inline SellCols sell_cols(const Sell &S) { return SellCols{S.col.get(), S.code.get(), S.cp.get(), S.dict.get()}; }
void sell_values32(ocp_ctx *ctx, const Sell &S, const int32_t *rp, const float *val32, DevBuf<float> &out);
}  // namespace ocp

struct ocp_system {
    ocp_ctx *ctx = nullptr;
    int32_t nv = 0;           // mesh vertices
    int32_t n = 0;            // interior unknowns
    int64_t nt = 0;           // tetrahedra
    int64_t nnz = 0;
    double rho = 0.0;
    int max_row_len = -1;     // longest assembled row (computed during assembly)
    const int32_t *tets_ref = nullptr;  // mesh tets the system was assembled from (borrowed)
    ocp_mesh mesh{};          // that mesh (device pointers, borrowed): later load vectors read it
    // incremented by fe_set_rho: hierarchies built before a change of the
    // values are refused by the solves (their diagonal, bounds and coarse
    // operators belong to the old matrix)
    std::atomic<uint64_t> generation{0};
    ocp::DevBuf<int32_t> inc_ptr, inc;  // vertex -> incident tets, ascending
    ocp::DevBuf<int32_t> dof_of_vertex, vertex_of_dof;
    ocp::DevBuf<int32_t> row_ptr, col;
    ocp::DevBuf<double> val, valK, valM, f;
    // Derived data.  The sliced-ELL copy is built with the values (fe_assemble,
    // fe_derive, fe_set_rho).  1/a_ii is built by the first Jacobi solve under
    // `derived_mu` and published only after its kernel has finished, so
    // concurrent solves on other contexts never read it half-filled; the block
    // SpMM panel widths are set once by compare-and-swap.  Solves otherwise
    // only read the system.
    std::mutex derived_mu;
    std::atomic<bool> dinv_ready{false};
    ocp::DevBuf<double> dinv;   // 1 / a_ii
    ocp::Sell sell;             // sliced-ELL copy of A for the solve phase
    std::atomic<int> blk_kb_spmm[65] = {};   // block SpMM panel width chosen per column count k (0: not yet)
};

namespace ocp {

// One level of the smoothed-aggregation hierarchy.  Level 0 borrows the
// system's CSR; coarser levels own theirs.
struct Level {
    int32_t n = 0, nc = 0;
    int64_t nnzA = 0, nnzP = 0;
    const int32_t *A_rp = nullptr, *A_col = nullptr;
    const double *A_val = nullptr;
    DevBuf<int32_t> own_rp, own_col;
    DevBuf<double> own_val;
    DevBuf<int32_t> P_rp, P_col, R_rp, R_col, agg;
    DevBuf<double> P_val, R_val;
    DevBuf<double> dinv;       // smoother diagonal: 1/a_ii (Chebyshev) or 1/sum_j |a_ij| (L1-Jacobi)
    DevBuf<double> dense_inv;  // last level only: A^{-1}, dense row-major
    // single-precision copies (mixed precision)
    DevBuf<float> A_val32, P_val32, R_val32, dinv32, dense_inv32;
    // level 0: values of the system's sliced-ELL copy in the hierarchy's precision
    // (FP32 hierarchies); levels >= 1 with at least kSellMinRows rows: a
    // sliced-ELL copy of their own A (FP64 values, and the FP32 copy)
    DevBuf<float> sell_val32;
    Sell sell;
    double lambda_max = 0.0;   // Gershgorin bound of D^-1 A
    // polynomial smoother: first step x = a D^-1 r; degree 2 adds
    // x = D^-1 (c1 r0 + c2 r1) with r1 the residual after the first step
    int deg = 1;
    double cheb_a = 1.0, cheb_c1 = 0.0, cheb_c2 = 0.0;
    int gA = 16, gP = 4, gR = 64;  // lanes per row of the A, P and R kernels
    int maxP = 0;                  // longest row of P
    // red-black hierarchies: a colouring of A's graph (no two coupled rows
    // share a colour) for the Gauss-Seidel sweeps, rows grouped by colour
    int ncolors = 0;
    std::vector<int32_t> color_ptr;   // host [ncolors + 1]
    DevBuf<int32_t> color_rows;       // [n] rows of colour c at color_ptr[c] .. color_ptr[c+1], ascending
};

}  // namespace ocp

struct ocp_hierarchy {
    ocp_ctx *ctx = nullptr;
    const ocp_system *sys = nullptr;
    uint64_t sys_generation = 0;   // sys->generation when the hierarchy was built
    double setup_ms = 0.0;         // wall time of amg_setup
    ocp_amg_params params{};
    std::vector<std::unique_ptr<ocp::Level>> levels;
    // block V-cycle panel width chosen per column count k (0: not yet), set
    // once by compare-and-swap so that every later solve uses the same kernels
    std::atomic<int> blk_kb_vc[65] = {};
};

namespace ocp {
// V-cycle work vectors of one solve, per level, in the hierarchy's precision
// (k columns for the block solve).  They belong to the solve, not to the
// hierarchy, so one hierarchy serves concurrent solves on several streams.
struct VcWork {
    struct Lvl {
        DevBuf<char> vb, vr, vx, vxp, vx1, vx2;
    };
    std::vector<Lvl> lv;
    double *part = nullptr;   // partials of the fine-level r.z (null: the context's)
    // Level 0's first pre-smoothing step a D^-1 r, written beside r by the
    // kernel that produced r (hierarchy precision); null: rebuilt from r.
    const void *y0 = nullptr;
};
void vc_work_alloc(ocp_ctx *ctx, const ocp_hierarchy *h, VcWork &w, int k = 1);

// Enqueue z = B r (one V-cycle).  If cg != nullptr the level-0 post-smoother
// also forms r.z and updates the CG scalars (through a one-block finalize
// kernel), and every kernel returns at once when cg->flag is set.
void vcycle_enqueue(ocp_ctx *ctx, const ocp_hierarchy *h, const double *r, double *z, CgScalars *cg, VcWork &w);
// Lanes per row for a matrix with the given average row length.
int level_lanes(int64_t nnz, int64_t rows);
// 1/a_ii of the system, built (and waited for) by the first caller.
const double *system_dinv(ocp_ctx *ctx, const ocp_system *sys);
// A hierarchy may precondition its own system or any system on the same
// mesh with the same sparsity pattern (another rho): the V-cycle then
// applies the operator built for the hierarchy's system.
bool hierarchy_fits(const ocp_hierarchy *h, const ocp_system *sys);
// Fail with INVALID_ARG if h cannot precondition sys: another pattern, or
// its own system's values changed (fe_set_rho) after it was built.
void check_hierarchy(const ocp_hierarchy *h, const ocp_system *sys);
// The sliced-ELL copy of the system's matrix (built with the values).
const Sell &system_sell(ocp_ctx *ctx, const ocp_system *sys);
}  // namespace ocp
