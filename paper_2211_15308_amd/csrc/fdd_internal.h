// Internal declarations shared by the host orchestration and the HIP kernels.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace fdd {

constexpr int kMaxLevels = 16;
constexpr int kMaxPoles = 64;
constexpr int kTile = 32;            // fine-grid tile edge of the fused multigrid kernels
constexpr int kMidTile = 16;         // tile edge of an intermediate level (latency-bound: small
                                     // tiles spread it over more compute units)
constexpr int kPresumTiles = 2048;  // above this many level-0 tiles the inner-PCG dot products
                                     // are summed by a pass of their own
constexpr int kResidentTiles = 1024; // level-0 tiles that are all in flight at once (4 per CU)
constexpr int kBlock = 256;          // threads per block of the tiled kernels
constexpr int kCoarseThreads = 1024; // threads of the single-workgroup coarse V-cycle
constexpr int kMaxCoarsestNf = 16;   // dense inverse on the coarsest grid up to 16 x 16 points
constexpr int kDstN = 64;            // FP32 coarse solve by sine transforms: up to 63 x 63 points

// One multigrid level of the interior Dirichlet grid.
struct Level {
  int nf;      // interior points per side
  int pitch;   // row pitch in elements
};

struct LaunchLevels {
  int first;   // first level handled inside one workgroup
  int nlev;
  int nf[kMaxLevels];
};

// Device-resident scalars and flags of one problem.  Kernels write them; the host clears the
// block at bind time and reads it back after synchronizations.
struct DevState {
  // inner PCG (in the precision of the multigrid-PCG)
  double rho;        // r^T z of the current iterate
  double rho_old;
  double pq;         // p^T q
  double rr;         // ||r||^2 after the last update
  double rr0;        // ||r||^2 at the start of this PCG run
  double tau2;       // the PCG run stops when rr <= tau2 * rr0
  // interior solve (FP64 refinement)
  double ff;         // ||f||^2 of the interior right-hand side
  double res2;       // ||f - A u||^2 (FP64)
  double tol2;       // the interior solve stops when res2 <= tol2 * ff
  // outer PCG
  double o_rho[2];   // r^T z, indexed by iterate parity
  double o_rho0;
  double o_pq, o_alpha, o_beta;
  double t_res[2];   // true residual: ||b - A x||^2, ||b||^2
  double cg_alpha[2];  // step length of the inner PCG, by iteration parity
  double cg_gam[2];    // r . z of the inner PCG, by iteration parity
  double warm_alpha;   // Galerkin factor of the learned initial guess (0: not used)
  double dots[2];      // r . z and z . A z for the next inner PCG update, when a separate
                       // pass sums their partials (large grids, batches)
  // counters / flags
  int inner_done;    // the running multigrid-PCG has converged (or broke down)
  int solve_done;    // the interior solve has met its tolerance
  int inner_its;     // multigrid-PCG iterations of the current interior solve
  int pcg_k;         // iterations executed in the current PCG run
  int refine_steps;  // refinement steps of the current interior solve (also buffer parity)
  int breakdown;     // bit 0: inner breakdown, bit 1: outer breakdown, bit 2: non-finite
  int pcg_is_final;  // FP64 mode: the PCG residual is the interior solve's residual
  int run_its_max;   // largest iteration count of a PCG run in this interior solve
  int run_len[8];    // PCG iterations of each refinement step's run (first 8 steps)
  int warm_used;     // the running interior solve started from a learned guess (alpha > 0)
  int pad3;
  int outer_done;    // batched solve: this instance's outer PCG has converged
  int o_ver;         // batched solve: version (parity) holding the final interface iterate
  int o_its;         // batched solve: outer iterations of this instance
  int pad2;
  unsigned counters[16];   // ticket of the true-residual reduction
};

// Right-hand side of an interior solve, formed on the fly:
//   f(i, j) = sb * b[(j-1) nf + (i-1)]  +  (j == nf ? sg * g[i-1] : 0)
struct RhsDesc {
  const double* b;   // may be null
  double sb;
  const double* g;   // may be null: values placed on the last interior row (next to Gamma)
  double sg;
};

template <typename T>
struct MGBuffers {
  T* f[kMaxLevels];   // right-hand side per level (level 0: unused, the PCG residual is used)
  T* u[kMaxLevels];   // pre-smoothed iterate per level
  T* e[kMaxLevels];   // result of the V-cycle per level (level 0: z)
};

// Per-block partial sums of the level-0 reductions (each has one slot per level-0 tile).
struct Reductions {
  double* pq;      // unused slot (kept for layout)
  double* rr;      // ||r||^2 after the update
  double* rz[2];   // r . z, by iteration parity
  double* zw[2];   // z . A z, by iteration parity
  double* ir;      // ||f - A u||^2 of the refinement residual
  double* ff;      // ||f||^2
  int nb0;         // number of level-0 tiles
  int nbd;         // r . z and z . A z partials per iteration (nb0; fewer when one up kernel
                   // covers several level-0 tiles per block)
};

// Optional HIP-event timing of one kernel kind (pairs of events around each launch of it).
enum TimedKernel { kTimeNone = 0, kTimeDown0 = 1, kTimeUp0 = 2, kTimeCoarse = 3 };
struct EventHook {
  int kind = kTimeNone;
  hipEvent_t* ev = nullptr;  // 2 * cap events
  int cap = 0;
  int used = 0;              // pairs recorded since the last harvest
  long long skipped = 0;     // launches not timed because the pool was full
};
// Launch `kernel`, attaching the next event pair of the hook to its dispatch packet when the hook
// times this kernel kind (hipExtLaunchKernelGGL stamps the events at kernel begin and end).
template <typename F, typename... Args>
inline void launch_timed(EventHook* h, int kind, F kernel, dim3 grid, dim3 block, hipStream_t s,
                         Args... args) {
  if (h && h->kind == kind) {
    if (h->used < h->cap) {
      hipExtLaunchKernelGGL(kernel, grid, block, 0, s, h->ev[2 * h->used], h->ev[2 * h->used + 1],
                            0, args...);
      ++h->used;
      return;
    }
    ++h->skipped;
  }
  hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

struct LaunchCtx {
  EventHook* hook = nullptr;
  hipStream_t stream;
  int nlev;
  int first_coarse;        // first level handled by the single-workgroup kernel
  Level lev[kMaxLevels];
  int nu;                  // red-black sweep pairs
  const double* coarse_inv64;  // FP64: dense inverse on the coarsest level (nfc^2 x nfc^2)
  const float* dst_S;      // FP32 coarse solve: sine-transform matrix (kDstN x kDstN, zero-padded)
  const float* dst_lam;    // ... and the 1D symbols 2 - 2 cos(k pi / (m + 1)) (kDstN entries)
  DevState* st;
  Reductions red;
};

// ---- multigrid-PCG (kernels_mg.hip) --------------------------------------------------------
template <typename T>
void launch_pcg_init(const LaunchCtx& c, const MGBuffers<T>& mg, const T* r, T* z_out);
// Iteration k of the inner PCG in its single-reduction (Chronopoulos-Gear) form: z = V r and the
// dots r.z, z.A z come from the previous V-cycle; p = z + beta p', x += alpha p, r -= alpha A p
// (A p as a stencil of p), then the V-cycle of the new r yields the next z and dots.
// update_only (the last scheduled iteration of a run that a refinement residual follows): the
// update only; the next z would not be used, and the residual takes the convergence test.
template <typename T>
void launch_pcg_iteration(const LaunchCtx& c, const MGBuffers<T>& mg, int k, T* x, T* r_old,
                          T* r_new, T* z, T* p_old, T* p_new, bool update_only = false);

// One V-cycle z = V f on its own (the preconditioner of the full-system PCG, not inside an
// interior solve): the same kernels as the start of a PCG run, without its bookkeeping.  The
// problem's flags must not mark a stopped solve (the kernels return at once then).
template <typename T>
void launch_vcycle(const LaunchCtx& c, const MGBuffers<T>& mg, const T* f, T* z);

// FP64 refinement residual: uout = uin + e (uout = 0 on the first call; a plain copy once the
// solve has converged), r = f - A uout.  The step's bookkeeping (convergence test, state of the
// next PCG run) is done by the first kernel of the next PCG run; finalize = true adds a one-block
// kernel for it, for a residual that no PCG run follows in the same launch sequence.  run_check:
// the run before it ended with an update-only iteration, whose convergence test it takes.
void launch_ir_residual(const LaunchCtx& c, const RhsDesc& f, const double* uin, const float* e32,
                        const double* e64, double* uout, float* r32, double* r64, int first,
                        double tol2, double tau2, int pcg_is_final, const float* warm,
                        const double* wscale, bool finalize, bool run_check = false);
// Galerkin factor of a learned guess g (FP32 image, pitch nf) for the right-hand side f, into
// st->warm_alpha (0 when the guess does not lower the energy error).
void launch_warm_alpha(const LaunchCtx& c, const RhsDesc& f, const float* g);

// ---- interface kernels (kernels_iface.hip) -------------------------------------------------
struct ShiftTable {
  int m;                       // number of shifted systems in the batch
  double alpha[kMaxPoles + 1]; // system k: (alpha_k A_G + beta_k M_G) y_k = rhs
  double beta[kMaxPoles + 1];
  double coef[kMaxPoles + 1];  // sum_k coef_k y_k
  double d0;                   // operator mode: H p = dL L p + d0 M p + M sum
  double dL;                   // (nonzero only for L^t with t >= 0 of the model problem)
};

enum IfaceMode { kIfacePrecond = 0, kIfaceOperator = 1, kIfacePrecondOuter = 2 };

// Static scratch of the no-allocation preconditioner apply: kStaticPrecondSystems systems of up
// to kStaticPrecondN unknowns.  static_precond_scratch looks its address up on `device`, which
// must be current, once per device (0 on success).
constexpr int kStaticPrecondSystems = kMaxPoles + 1;
constexpr int kStaticPrecondN = 2048;
constexpr int kMaxStaticDevices = 64;
int static_precond_scratch(int device, double** out);
// Copies *st into pinned host memory `host` and then stores `seq` into the pinned word
// `seq_word` (one small kernel; the host waits for the word instead of a stream synchronization).
void launch_publish_state(hipStream_t s, const DevState* st, DevState* host, unsigned* seq_word,
                          unsigned seq);

void launch_iface_batch(hipStream_t s, int ng, double h, const ShiftTable& tab, int mode,
                        const double* in, double* out, double* scratch, DevState* st,
                        const double* p_prev, double* p_next, int ver, int first);
void launch_schur_gather(hipStream_t s, int ng, int nf, int pitch, double K, double gamma,
                         const double* p, const double* u0, const double* u1, const int* sel,
                         const double* Hp, double* y, const double* x, double* xn,
                         const double* r, double* rn, DevState* st, int mode, int ver);
void launch_rhs_reduce(hipStream_t s, int n, int pitch, const double* bG, const double* u0,
                       const double* u1, const int* sel, double* g, double* x);
void launch_scatter(hipStream_t s, int nf, int pitch, const double* u0, const double* u1,
                    const int* sel, const double* xG, double* x);
void launch_copy_rows(hipStream_t s, const double* src, int sp, double* dst, int dp, int width,
                      int rows);
// out = a + c u on the nf x nf interior grid (row pitch `pitch`, FP64); a may be null (zero);
// c = *coef when coef is non-null (a device scalar, read by the kernel), else c = scale.
void launch_interior_axpy(hipStream_t s, int nf, int pitch, const double* a, const double* u,
                          const double* coef, double scale, double* out);
void launch_full_operator(hipStream_t s, int n, double K, double gamma, const double* x,
                          const double* Hx, double* y, const double* b, double* partials,
                          double* res);

// ---- batched solve (kernels_batch.hip) ------------------------------------------------------
// One independent 2D instance of a batch, as seen by the batched kernels (device memory).  All
// pointers refer to the instance's own bound workspace; the FP32 multigrid-PCG set is used.
struct BInst {
  int nlev, fc;                       // levels; first level solved inside one workgroup
  int nf[kMaxLevels], pitch[kMaxLevels];
  int tiles_x[kMaxLevels];            // tiles per row of each tiled level (0 if not tiled)
  float* f[kMaxLevels];
  float* u[kMaxLevels];
  float* e[kMaxLevels];
  float *x, *r[2], *p[2], *z;
  double* u64[2];
  double* xI[2];                      // interior part of the solution, by outer version
  const float* dstS;                  // sine-transform matrix of the first coarse level
  const float* dstL;                  // its 1D symbols
  DevState* st;
  Reductions red;
  // interface / outer PCG
  int ng, mP, mH;                     // interface size; systems in the P and H batches
  double h, K, gamma;
  const double* b;                    // caller right-hand side (free-dof order)
  double* xout;                       // caller solution
  double *xG[2], *rG[2], *pG[2], *zG, *yG, *Hp, *scrP, *scrH;
  const ShiftTable* tabP;
  const ShiftTable* tabH;
  // learned warm start of the lifted-p interior solves (null: zero initial guess)
  const float* warm;                  // the network's image for this instance (pitch nf[0])
  double* trace;                      // this instance's row of the network's input traces
};

// Work lists of a batch (device memory): prefix sums over instances.
struct BLists {
  const int* tiles[kMaxLevels];       // tiles of each instance at level l (ninst + 1 entries)
  const int* sysP;                    // RA systems of the preconditioner batch
  const int* sysH;                    // RA systems of the operator batch
  int ninst;
};

// right-hand side kinds of a batched interior solve
enum BRhs { kRhsB = 0, kRhsLiftP = 1, kRhsBack = 2 };

struct BatchCtx {
  EventHook* hook;                    // optional kernel timer
  hipStream_t stream;
  const BInst* inst;
  BLists lists;
  int nu;
  int max_tiled;                      // largest number of tiled levels over the instances
  int tiles_total[kMaxLevels];        // grid sizes of the tiled levels
  int tile_edge[kMaxLevels];          // tile edge of each tiled level (kTile or kMidTile)
  int sysP_total, sysH_total;
  int skip_done;                      // kernels skip instances whose outer PCG has converged
};

void launch_b_inner_start(const BatchCtx& c, int rhs, int ver, double tol2, double tau2);
// learned warm start: every instance's p_G (version ver) into its trace row; the Galerkin factor
// alpha = f.g / g.A g of every instance's image g for its lifted right-hand side
void launch_b_gather_traces(const BatchCtx& c, int ver);
void launch_b_warm_alpha(const BatchCtx& c, int ver);
void launch_b_inner_step(const BatchCtx& c, int rhs, int ver, int its, int S, int& cur_r,
                         int& cur_p);
void launch_b_rhs_reduce(const BatchCtx& c, int S);
void launch_b_precond_init(const BatchCtx& c, double rtol);
// accumulate: x_I(v+1) = x_I(v) + alpha E p after the Schur product (no back-substitution solve)
void launch_b_outer_tail(const BatchCtx& c, int S, int v, double rtol, bool accumulate);
// x_I(0) = A_II^{-1} b_I / K from the interior solve of the right-hand side
void launch_b_xI_init(const BatchCtx& c, int S);
void launch_b_operator(const BatchCtx& c, int v);
// from_xI: the interior part comes from the accumulated x_I, else from the last interior solve
void launch_b_scatter(const BatchCtx& c, int S, int ver, bool from_xI);
void launch_b_gather_states(const BatchCtx& c, DevState* out);

// ---- host rational approximation (ra_build.cpp) --------------------------------------------
struct RaResult {
  int status;                  // 0 ok, otherwise an FDD_E_* code
  double c0;
  int m;
  double c[kMaxPoles];
  double p[kMaxPoles];         // shifts p_k >= 0 (poles of f_RA at -p_k)
  double max_rel_err;
  int aaa_support;             // support points used by AAA
  int dropped;                 // poles discarded by the filter
};

// f(lam) = 1 / (K lam^{1/2} + gamma lam^t) (which = 0) or lam^t (which = 1); t = -1/2 for the
// Riesz map of the facet problems.
RaResult build_rational(int which, double K, double gamma, double lam_lo, double lam_hi,
                        const double* check_pts, int ncheck, double tol, int max_poles,
                        double t = -0.5);
double ra_eval_rel_err(int which, double K, double gamma, const RaResult& r, const double* pts,
                       int npts, double t = -0.5);

// dense linear algebra used by the builder (exposed for host tests)
int eig_real_general(int n, const double* A, double* wr, double* wi);   // A row-major
int svd_min_right(int rows, int cols, const double* A, double* v, double* smin, double* smax);

// ---- full-system PCG with the lazy block preconditioner (kernels_full.hip) ----------------
// Buffers of one problem as the full-system PCG uses them: interior parts on the padded level-0
// grid (FP64), Gamma parts as n - 1 vectors.
struct FullCtx {
  hipStream_t stream;
  int nf, pitch;
  double K, gamma, h;
  double *xI, *rI, *pI[2], *qI;
  double *xG, *rG, *pG[2], *qG, *zG, *tG, *Hp;
  double *scratchP, *scratchH, *partials;
  DevState* st;
};
// r = b, x = 0; vr = vf = r_I in the V-cycle's precision
template <typename VT>
void launch_full_init(const FullCtx& c, const double* b, VT* vr, VT* vf);
// t_G = r_G + W|top row, z_G = S_Gamma^{-1} t_G (table P), vf|top row = r_I + K z_G
template <typename VT>
void launch_full_precond_tail(const FullCtx& c, const ShiftTable& tabP, const VT* W, VT* vf);
// rz = r . z (z_I = Z / K) into st->o_rho[cur], beta, and the stop test (first: rz_0); a
// passed test records `it` (the iterations done) and stops every later kernel of the solve
template <typename VT>
void launch_full_rz(const FullCtx& c, const VT* Z, int cur, int first, double rtol2, int it);
// p = z + beta p' (version a -> a ^ 1), q = A p with H_RA by table H, alpha = rz / p.q,
// x += alpha p, r -= alpha q, vr = vf = r_I
template <typename VT>
void launch_full_step(const FullCtx& c, const ShiftTable& tabH, const VT* Z, int a, int cur,
                      int first, VT* vr, VT* vf, int it);
// clears the stop mark the stop test leaves on the multigrid kernels
void launch_full_clear_stop(const FullCtx& c);
// out (caller layout) = (aI * sI, aG)
template <typename VT>
void launch_full_scatter(const FullCtx& c, const VT* aI, double sI, const double* aG, double* out);

// ---- the paper's model problem in 2D (kernels_model.hip) -------------------------------------
// Interior nodes on the padded level-0 grid, the 4n boundary nodes as a loop vector.
// yI = scale (A_Omega + M_Omega)(xI, xG) on the interior rows (+ add_scale addc, addc compact
// with pitch n - 1, may be null); xI or xG null means zero there.
void launch_model_interior_rows(hipStream_t s, int n, int pitch, double scale, const double* xI,
                                const double* xG, double* yI, const double* addc = nullptr,
                                double add_scale = 0.0);
// yG = add + scale (A_Omega + M_Omega)(xI, xG) + gamma Hp on the loop rows (add, Hp may be null)
void launch_model_loop_rows(hipStream_t s, int n, int pitch, double scale, double gamma,
                            const double* xI, const double* xG, const double* Hp,
                            const double* add, double* yG);
// y = K (A_Omega + M_Omega) x + gamma T^T Hx on all dofs (caller layout); with b: res[0] =
// ||b - y||^2, res[1] = ||b||^2
void launch_model_full_apply(hipStream_t s, int n, double K, double gamma, const double* x,
                             const double* Hx, double* y, const double* b, double* partials,
                             double* res);
// all shifted loop systems of a table (cyclic, eq. (RA)) and their combination
void launch_model_loop_batch(hipStream_t s, int n, const ShiftTable& tab, int mode,
                             const double* in, double* out, double* scratch);
// interior PCG on A_II = A_Omega + M_Omega (interior block) with V-cycles of the 5-point
// Laplacian as the preconditioner (scalars and flags in st: rho, pq, cg_alpha[0], cg_gam, rr, ff,
// tol2, inner_done, inner_its).  ii_rz leaves the partials of r.z; ii_step sums them (beta),
// forms p and q = A_II p, sums p.q (alpha), updates x and r and tests ||r||.  partials holds
// 8192 doubles.
template <typename VT>
void launch_model_ii_start(hipStream_t s, int nf, int pitch, const double* f, double* x,
                           double* r, VT* vr, DevState* st, double* partials, double tol2);
template <typename VT>
void launch_model_ii_rz(hipStream_t s, int nf, int pitch, const double* r, const VT* Z, double zs,
                        DevState* st, double* partials);
template <typename VT>
void launch_model_ii_step(hipStream_t s, int n, int pitch, const VT* Z, double zs, double* p_old,
                          double* p_new, double* q, double* x, double* r, VT* vr, DevState* st,
                          double* partials, int first);
// outer PCG on the loop vectors (one block each): alpha = rho / p.y, x += alpha p, r -= alpha y;
// and rho' = r.z, beta, p' = z + beta p with the stop test (first: rho_0, p = z)
void launch_model_outer_update(hipStream_t s, int m, const double* p, const double* y, double* x,
                               double* r, DevState* st);
void launch_model_outer_direction(hipStream_t s, int m, const double* r, const double* z,
                                  const double* p_old, double* p_new, DevState* st, int first,
                                  double rtol2);

}  // namespace fdd
