// The coupled Darcy-Stokes problem (Sec. 4, eq. (darcy_stokes)) and its block-diagonal
// preconditioner (eq. (darcy_stokes_precond)): host plan, device views and kernel launchers.
//
// Geometry: Darcy on (0, 1)^2, Stokes on (0, 1) x (1, 2), interface Gamma = (0, 1) x {1}; no slip
// on the Stokes sides, zero traction on the Stokes top, zero Darcy pressure on the rest of the
// Darcy boundary.  Taylor-Hood P2-P1 for Stokes and P1 for the Darcy pressure on the
// diagonal-split meshes of n cells per side.  Unknowns, in this order:
//   u_x, u_y  P2 nodes (A h/2, 1 + B h/2), A = 1..2n-1, B = 0..2n:
//             index c NV + B (2n - 1) + (A - 1), NV = (2n - 1)(2n + 1)
//   p_S       vertices (i h, 1 + j h): Nu + j (n + 1) + i
//   p_D       the facet problem's free dofs (interior points row by row, then Gamma)
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "hdiv_internal.h"

struct fdd_problem_s;

namespace fdd {

constexpr int kDsCoarseN = 4;      // the velocity hierarchy's coarsest level (dense inverse)
constexpr int kDsMaxN = 1024;
constexpr int kDsMaxKrylov = 400;  // FGMRES basis vectors the workspace may hold

// Device state of the FGMRES iteration.
struct DsState {
  double beta;      // ||b||_2
  double res;       // |g_{k+1}|: the least-squares residual ||b - A x_k||_2
  double hnext;     // h_{k+1,k} of the last Arnoldi step
  double t_res[2];  // ||b - A x||^2, ||b||^2 of the returned x
  int its, done, breakdown, pad;  // breakdown: bit 2 non-finite
};

struct ProblemDS {
  int n = 0, nlev = 0, krylov = 0;
  double K = 1, mu = 1, alpha = 0;
  int Nu = 0, Np = 0, ND = 0, N = 0;
  // the velocity block a(., .) on every level (finest first) and the pressure mass (one level,
  // one-dof patches: the Jacobi diagonal of its Chebyshev iteration)
  HdLevel lev[kHdMaxLevels];
  HdLevel mass;
  std::vector<double> cinv;   // dense inverse of the coarsest velocity matrix (row-major)
  // the coupled operator by row blocks, global columns: [A_u B^T C], [B], [C^T -K A_D]
  HdMat Au, Bp, Dd;
  fdd_problem_s* darcy = nullptr;  // the facet problem of the Darcy block (own workspace)
  int its_u = 0;                   // iterations of the last velocity solve
  // device
  double* dcinv = nullptr;
  double *ur = nullptr, *uz = nullptr, *up = nullptr, *uq = nullptr;   // velocity PCG
  double *pz = nullptr, *pq = nullptr, *pp = nullptr;   // pressure Chebyshev: x (two), d
  double *V = nullptr, *Z = nullptr;       // (krylov + 1) x N and krylov x N
  double *Hm = nullptr;                    // (krylov + 1) x krylov, column-major
  double *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr, *hp = nullptr;
  double* partials = nullptr;              // (krylov + 1) x kDsChunks
  HdState *st_u = nullptr, *hst_u = nullptr;
  DsState* st = nullptr;
  DsState* hst = nullptr;
  size_t ws_need = 0;
};

constexpr int kDsChunks = 512;   // blocks of one vector's reduction

// ---- host set-up (ds_setup.cpp) --------------------------------------------------------------
// Builds every velocity level, the pressure mass and the operator rows.  Returns 0 or a message.
const char* ds_build(ProblemDS* D, int n, double K, double mu, double alpha, int krylov);
// Workspace bytes of the Darcy-Stokes part; with base != nullptr also assigns the device views.
size_t ds_plan(ProblemDS* D, char* base);

// ---- kernels (kernels_ds.hip) ------------------------------------------------------------------
// beta = ||b||, V_0 = b / beta, g = (beta, 0, ...), state reset (rtol2 kept by the Givens step)
void launch_ds_start(hipStream_t s, int n, const double* b, double* V0, double* g, double* partials,
                     DsState* st);
// Two classical Gram-Schmidt passes against V_0..V_k: h_i = V_i . w, w -= sum_i h_i V_i; Hcol
// (column k of H) receives the sum of both passes' coefficients, hpass (k + 1) is scratch
void launch_ds_orthogonalize(hipStream_t s, int n, int k, const double* V, double* w, double* Hcol,
                             double* hpass, double* partials, const DsState* st);
// h_{k+1,k} = ||w||, w /= h_{k+1,k}; then the Givens rotations of column k, the new residual
// estimate and the stop test |g_{k+1}| <= rtol ||b||
void launch_ds_normalize_givens(hipStream_t s, int n, int k, int ldh, double* w, double* Hm,
                                double* cs, double* sn, double* g, double* partials, DsState* st,
                                double rtol);
// y = R^{-1} g (k x k upper triangle of H), x = sum_i y_i Z_i
void launch_ds_solution(hipStream_t s, int n, int k, int ldh, const double* Hm, const double* g,
                        double* y, const double* Z, double* x);
// y = a x
void launch_ds_scale(hipStream_t s, int n, double a, const double* x, double* y);
// ||b - A x||^2 and ||b||^2 into st->t_res (the three row blocks of A)
void launch_ds_true_residual(hipStream_t s, HdView Au, HdView Bp, HdView Dd, const double* b,
                             const double* x, double* partials, DsState* st);

}  // namespace fdd
