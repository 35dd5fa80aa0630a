// The H(div) variant of the interface-perturbed problem (Sec. 3, remark on H(div)-elliptic
// problems, eq. (graddiv)): host plan, device views and kernel launchers.
//
//   K int (u.v + div u div v) + gamma int_{dOmega} (u.nu)(v.nu),  Omega = (0, 1)^2,
//
// lowest-order BDM elements on the diagonal-split mesh, Gamma = the whole boundary, trace space
// Q_h = discontinuous P1 on the 4n boundary segments.  Dof order: two dofs per edge (the normal
// component at the edge's first and second endpoint), interior edges first (horizontal, vertical,
// diagonal), then the boundary segments along the counter-clockwise loop from (0, 0).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "fdd_internal.h"

namespace fdd {

constexpr int kHdPatch = 12;       // dofs of a vertex patch (six incident edges)
constexpr int kHdMaxTypes = 16;    // distinct patch matrices per level
constexpr int kHdMaxLevels = 12;
constexpr int kHdCoarseN = 8;      // the coarsest level: min(n, 8) cells per side, dense inverse
constexpr int kHdMaxN = 1024;      // the loop solves hold 4n segments in one workgroup's LDS

// Device state of one H(div) problem: scalars of the interior PCG (A^00 u = f) and of the outer
// Schur-complement PCG on the trace.
struct HdState {
  double rz, rz_old, alpha, beta, rr, ff, tol2;   // interior PCG
  double o_rz, o_rz0, o_alpha;                   // outer PCG
  double t_res[2];                               // ||b - A x||^2, ||b||^2
  int done, its, breakdown, pad;   // interior; breakdown bit 0 inner, 1 outer, 2 non-finite
  int o_done, o_its, pad2[2];
};

// The trace operator's blocks on the loop (row-major 2 x 2): segment k's own block, its
// coupling to segment k - 1 (the coupling to k + 1 is the transpose) and the mass block.
struct HdLoopBlocks {
  double own[4], prev[4], mass[4];
};

// A rational table (d0, d_k, q_k) of f(lam) / lam for the trace preconditioner (by value).
struct HdTable {
  int m;
  double d0, dsum;
  double d[kMaxPoles], q[kMaxPoles];
};

// A sparse matrix in ELL form with typed rows: every row holds `width` column slots, slot k of
// row i at k * rows + i (consecutive rows are consecutive in memory, so a wave's loads coalesce;
// unused slots point at column min(i, cols - 1) with value 0), and its values come from a small
// table: row i's slot k has value tval[rtype[i] * width + k].  On the uniform mesh rows repeat
// (translation invariance), so a product reads 4 bytes per slot and per row instead of 12.
// Where the column pattern repeats too (a row's neighbours at fixed index offsets, as on the
// structured P2 grid), the type also fixes the columns: slot k of row i is column
// i + toff[rtype[i] * width + k], and the per-row column array is not stored on the device (a
// product then reads 4 bytes per row for the type plus the gathered x).  The relative form is
// chosen when its type table stays small (to_ell); toff is empty otherwise.
// Host copies (val: the expanded values, col: absolute columns) built at setup, device copies in
// the workspace.
struct HdMat {
  int rows = 0, cols = 0, width = 0, ntypes = 0;
  std::vector<int> col, rtype, toff;
  std::vector<double> val, tval;
  int *dcol = nullptr, *drtype = nullptr, *dtoff = nullptr;
  double* dtval = nullptr;
};

struct HdLevel {
  int n = 0;        // cells per side
  int n0 = 0;       // interior dofs
  int nvert = 0;    // (n + 1)^2 vertices
  int ntypes = 0;   // distinct patch matrices
  HdMat A;          // A^00 of this level (K(mass + div-div) on V_0)
  HdMat P, R;       // prolongation from the next coarser level (rows: this level) and R = P^T
  int pw = kHdPatch;        // patch stride: 12 (H(div)), 8 (P2 velocity) or 1 (one-dof patches)
  std::vector<int> patch;   // nvert x pw interior dofs of the patch (-1: none)
  std::vector<int> ptype;   // nvert: index of the patch matrix (-1: no interior edge)
  std::vector<int> slot;    // n0 x 2: vertex * pw + position, for both patches holding the dof (-1: none)
  std::vector<double> pinv; // ntypes x pw x pw inverses (zero-padded)
  // device views
  int *dpatch = nullptr, *dptype = nullptr, *dslot = nullptr;
  double* dpinv = nullptr;
  double *x = nullptr, *b = nullptr, *r = nullptr, *Y = nullptr;
};

struct ProblemHdiv {
  int n = 0, nlev = 0;
  double K = 1, gamma = 0, theta = 0.5;
  int N = 0, N0 = 0, NG = 0;
  HdLevel lev[kHdMaxLevels];
  std::vector<double> cinv;  // dense inverse of the coarsest A^00 (n0 x n0, row-major)
  HdMat A0G, AG0, AGG, Afull;
  HdLoopBlocks blk;          // the trace operator L and mass M_Q on the loop
  int its_hint = 0;          // iterations of the last interior solve (enqueued ahead)
  // device
  HdState* st = nullptr;
  HdState* hst = nullptr;    // pinned copy
  double* dcinv = nullptr;
  double *u = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *f = nullptr;
  double *t0 = nullptr;      // interior scratch
  double *xG = nullptr, *rG = nullptr, *zG = nullptr, *pG = nullptr, *yG = nullptr, *tG = nullptr;
  double* partials = nullptr;  // kHdPartials per reduction
  double* scratch = nullptr;   // (m + 2) x 8n loop solutions
  size_t ws_need = 0;
};

constexpr int kHdPartials = 8192;

// ---- host setup (hdiv_setup.cpp) ------------------------------------------------------------
// Builds every level's matrices, transfers and patch tables.  Returns 0 or a message.
const char* hdiv_build(ProblemHdiv* Q, int n, double K, double gamma);
// Workspace bytes; with base != nullptr also assigns the device views.
size_t hdiv_plan(ProblemHdiv* Q, char* base);
// The generalized spectrum of (L, M_Q) on the loop (closed form per Fourier mode), ascending.
std::vector<double> hdiv_loop_eigs(const ProblemHdiv* Q);

// ---- kernels (kernels_hdiv.hip) --------------------------------------------------------------
struct HdView {
  const int* col;     // absolute columns (null when toff is set)
  const int* rtype;
  const double* tval;
  const int* toff;    // per-type column offsets, or null
  int rows, width, ntypes;
};
inline HdView view(const HdMat& m) {
  return HdView{m.dcol, m.drtype, m.dtval, m.dtoff, m.rows, m.width, m.ntypes};
}

// Every launcher takes `stop`: kernels return at once when stop->done is set (null: never).
// y = beta y + alpha A x  (beta = 0: y is only written)
void launch_hd_spmv(hipStream_t s, HdView A, const double* x, double* y, double alpha,
                    double beta, const HdState* stop);
// r = b - A x
void launch_hd_residual(hipStream_t s, HdView A, const double* b, const double* x, double* r,
                        const HdState* stop);
// Y[v] = (patch matrix of v)^{-1} r restricted to v's patch, for every vertex with a patch
void launch_hd_patch_solve(hipStream_t s, const HdLevel& L, const double* r, const HdState* stop);
// x = (add ? x : 0) + theta (sum of the patch solutions holding each dof)
void launch_hd_patch_sum(hipStream_t s, const HdLevel& L, double theta, double* x, int add,
                         const HdState* stop);
// One Jacobi-Chebyshev step for L.A x = b on a level with one-dof patches (the diagonal
// inverse): first: d = c_res D^{-1} b, x_out = d; else d = c_prev d + c_res D^{-1} (b - A x_in),
// x_out = x_in + d
void launch_hd_cheb_step(hipStream_t s, const HdLevel& L, const double* b, const double* x_in,
                         double* x_out, double* d, double c_prev, double c_res, int first);
// x = C b on the coarsest level (dense, row-major C, one wave per row)
void launch_hd_coarse(hipStream_t s, const double* C, int n0, const double* b, double* x,
                      const HdState* stop);
// interior PCG on A^00 (scalars on the device, fixed-order reductions)
//   start: u = 0, r = f, ff = f.f, the stop tolerance tol2 (relative, squared)
void launch_hd_pcg_start(hipStream_t s, int n0, const double* f, double* u, double* r,
                         double* partials, HdState* st, double tol2);
//   rz = r.z; beta = rz / rz_old (first: 0)
void launch_hd_pcg_rz(hipStream_t s, int n0, const double* r, const double* z, double* partials,
                      HdState* st, int first);
//   p_new = z + beta p_old (first: z), q = A p_new, pq -> alpha = rz / pq
void launch_hd_pcg_pq(hipStream_t s, HdView A, const double* z, const double* p_old,
                      double* p_new, double* q, double* partials, HdState* st, int first);
//   u += alpha p, r -= alpha q, rr = r.r, stop when rr <= tol2 ff
void launch_hd_pcg_update(hipStream_t s, int n0, const double* p, const double* q, double* u,
                          double* r, double* partials, HdState* st);
// The trace preconditioner from a table (d0, d_k, q_k) of f(lam) / lam:
//   z = d0 M^-1 L M^-1 r + (sum d) M^-1 r - sum d_k q_k (L + q_k M)^{-1} r,
// one workgroup per shifted system (block-circulant cyclic reduction in LDS) plus one for the
// M^-1 terms, then the weighted sum in fixed order.  scratch: (m + 1) x 8n.
void launch_hd_loop_precond(hipStream_t s, int n, const HdLoopBlocks& blk, const HdTable& T,
                            const double* r, double* z, double* scratch);
// outer PCG on the trace (one workgroup each): alpha = rz / p.y; x += alpha p, r -= alpha y;
// rz = r.z, beta, p = z + beta p, stop test (rz <= rtol2 rz0)
void launch_hd_outer_alpha(hipStream_t s, int m, const double* p, const double* y, HdState* st);
void launch_hd_outer_update(hipStream_t s, int m, const double* p, const double* y, double* x,
                            double* r, HdState* st);
void launch_hd_outer_direction(hipStream_t s, int m, const double* r, const double* z, double* p,
                               HdState* st, int first, double rtol2);
// ||b - A x||^2 and ||b||^2 into st->t_res
void launch_hd_true_residual(hipStream_t s, HdView A, const double* b, const double* x,
                             double* partials, HdState* st);
// b = scale a
void launch_hd_scale(hipStream_t s, const double* a, double* b, int n, double scale);

}  // namespace fdd
