/*
 * fdd.h -- C ABI of the fractional-interface domain-decomposition solver (MI355X, gfx950).
 *
 * Problem (paper, Sec. 1, eq. (riesz)):   -K Delta_Omega x + mu^{-1} (-Delta_Gamma)^{-1/2} x = b
 * on Omega = (0,1)^dim with Gamma = {x_dim = 1}, homogeneous Dirichlet conditions on the rest of
 * the boundary (and at the boundary of Gamma), discretized with P1 elements (Sec. 3).  In the
 * notation of eq. (generic): A = K A_Omega + gamma T^T H T, gamma = 1/mu, H = L_h^{-1/2} with
 * L_h the interface stiffness A_Gamma and M_h the interface mass M_Gamma (eq. (gevp)).
 *
 * Method (Sec. 2): PCG on the interface Schur complement
 *     S = K (A_GG - A_GI A_II^{-1} A_IG) + gamma H          (eq. (block_op) eliminated)
 * preconditioned by the inverse of S_Gamma = K L^{1/2} + gamma L^{-1/2} (eq. (schur_precond)),
 * applied through the rational approximation c0 M^{-1} + sum_k c_k (L + p_k M)^{-1} (eq. (RA)).
 * The interior Dirichlet block A_II is inverted by geometric-multigrid-preconditioned CG, in FP32
 * wrapped by FP64 iterative refinement (or all FP64).  H itself is applied by a second rational
 * approximation of lambda^{-1/2} (remark on evaluating the operator, Sec. 3).
 *
 * Conventions
 *   - Vectors passed to the library are DEVICE pointers to contiguous float64 arrays in the
 *     free-dof order: 2D index (j-1)(n-1)+(i-1) over j = 1..n, i = 1..n-1; 3D index
 *     ((k-1)(n-1)+(j-1))(n-1)+(i-1) over i, j = 1..n-1, k = 1..n.  The N_G interface dofs are
 *     the last N_G entries.  Interface-only vectors (x_G, y_G, r_G, z_G) have length N_G.
 *   - The caller owns b, x and the workspace.  All device vectors and scratch of the solver live
 *     in the bound workspace.  Besides it the library creates, on first use: one non-blocking
 *     stream and two events per problem or batch (graph replay), instantiated hipGraphs of outer
 *     iterations, small pinned host blocks for the state read back after synchronizations, HIP
 *     events for the kernel timer, and (fdd_precond_apply_static) a static 1 MiB device array.
 *   - All device work is enqueued on the caller's HIP stream (hipStream_t passed as void*;
 *     NULL means the default stream).  fdd_schur_apply, fdd_precond_apply, fdd_apply_operator
 *     and fdd_interior_solve synchronize only where documented.  fdd_solve returns after
 *     convergence (it reads scalars back once per outer iteration).
 *   - A handle must not be used by two calls at the same time.  Distinct problems may run
 *     concurrently on distinct streams if they have distinct workspaces.
 *   - Every function returns an int status; 0 is success.  fdd_last_error() returns a
 *     thread-local message for the last non-zero status.
 */
#ifndef FDD_H
#define FDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------------- */
enum {
  FDD_OK = 0,
  FDD_NOT_CONVERGED = 1,   /* iteration limit hit; outputs hold the last iterate             */
  FDD_E_ARG = -1,          /* invalid argument (n, K, mu, pointer, size)                      */
  FDD_E_NOMEM = -2,        /* host allocation failed                                          */
  FDD_E_HIP = -3,          /* a HIP runtime call failed (no device, launch failure, ...)     */
  FDD_E_RA = -4,           /* no admissible rational approximation (real p_k >= 0 outside
                              the spectrum, error within tolerance)                          */
  FDD_E_BREAKDOWN = -5,    /* PCG breakdown: p^T S p <= 0 or r^T z <= 0                       */
  FDD_E_NONFINITE = -6,    /* NaN/Inf in an input or an iterate                               */
  FDD_E_WORKSPACE = -7,    /* no workspace bound, or the bound workspace is too small         */
  FDD_E_STATE = -8         /* call out of order (e.g. table built for another problem)       */
};

enum { FDD_FP64 = 0, FDD_MIXED = 1 };                 /* precision of the interior solves     */
enum { FDD_RA_PRECOND = 0, FDD_RA_OPERATOR = 1 };     /* which function a table approximates  */

typedef struct fdd_problem_s* fdd_problem;   /* opaque: host state + views into the workspace */
typedef struct fdd_ratpc_s* fdd_ratpc;       /* opaque: one rational table (host copy)          */
typedef struct fdd_batch_s* fdd_batch;       /* opaque: a batch of problems solved together     */
typedef struct fdd_cnn_s* fdd_cnn;           /* opaque: the warm-start network                  */

/* Problem description.  dim = 2 or 3 (Omega = (0,1)^dim, Gamma = the facet x_dim = 1);
 * n = cells per side, even, 4 <= n <= 2048 (dim 3: the limits of fdd_setup_mesh) and such that
 * halving the (n - 1)-point grid while its point count is odd ends at <= 16 points (every
 * n = 2^k and n = 2^k (2j + 1) with small j); K > 0; mu > 0.                                  */
typedef struct {
  int dim;
  int n;
  double K;
  double mu;
} fdd_desc;

/* Solver options.  Fill with fdd_opts_default() and override fields. */
typedef struct {
  double outer_rtol;   /* stop when (r^T z)^{1/2} <= outer_rtol (r0^T z0)^{1/2}  (Sec. 3)       */
  int outer_maxit;     /* outer PCG iteration limit                                            */
  double inner_rtol;   /* each interior solve stops when ||f - A_II u||_2 <= inner_rtol ||f||_2  */
  int inner_maxit;     /* limit on multigrid-PCG iterations per interior solve                 */
  int precision;       /* FDD_MIXED (FP32 multigrid-PCG inside FP64 refinement) or FDD_FP64     */
  int mg_nu;           /* red-black Gauss-Seidel sweep pairs before and after coarse correction */
  double step_rtol;    /* mixed precision: each FP32 multigrid-PCG run (one refinement step)
                          reduces its residual by this factor (default 1e-5; 1e-7 .. 1e-2)    */
  int check_true_residual; /* nonzero: fdd_solve computes ||b - A x|| / ||b|| at the end       */
  void* warmstart;     /* NULL, or a network handle of type fdd_cnn with its parameters set,
                          its workspace bound and n_max >= n:
                          fdd_solve (mixed precision) starts the interior solve of every outer
                          iteration from the network's guess g for the lifted search direction,
                          entered as a g with a = f.g / g.A g (the energy-optimal multiple) and
                          dropped when a <= 0                                                  */
  int use_graph;       /* 1 (default): fdd_solve replays each outer iteration from a captured
                          hipGraph on a library-owned stream ordered after `stream`; 0: eager */
  int back_solve;      /* 0 (default): the interior part of the solution is accumulated during
                          the outer PCG, x_I = A_II^{-1} b_I / K + sum_k alpha_k E p_k (E p_k is
                          the interior solve of outer iteration k; equal to the back-substitution
                          of eq. (block_op) by linearity), so no interior solve follows the
                          outer PCG; 1: x_I = A_II^{-1} (b_I / K - A_IG x_G) by one more
                          interior solve after the outer PCG                                   */
} fdd_opts;

/* Per-solve statistics. */
typedef struct {
  int status;
  int outer_its;        /* outer PCG iterations                                               */
  int inner_solves;     /* interior Dirichlet solves performed                                 */
  int inner_its_total;  /* multigrid-PCG iterations summed over all interior solves           */
  int inner_its_max;    /* largest count in one interior solve                                 */
  int refine_steps;     /* FP64 refinement steps summed over all interior solves              */
  double rel_precond_res;  /* final (r^T z / r0^T z0)^{1/2}                                     */
  double true_rel_res;     /* ||b - A x||_2 / ||b||_2 if requested, else -1                     */
  double t_solve_ms;       /* host wall time of fdd_solve                                      */
  int warm_starts;         /* interior solves started from the network's guess                 */
  int warm_accepted;       /* ... of which the guess was kept                                  */
} fdd_stats;

void fdd_opts_default(fdd_opts* opts);

/* ---- problem setup (Sec. 3: P1 spaces, discrete trace by nodal injection) ------------------
 * fdd_setup_mesh: validates the description and builds the host-side plan: level hierarchy of
 * the interior multigrid, the coarsest-grid inverse, the spectral interval of (A_G, M_G).
 * Host only; hip_device is recorded and made current by later device calls.
 * Errors: FDD_E_ARG for dim other than 2 or 3; in 2D n odd, n < 4 or n > 2048 (one interface
 * vector must fit in a workgroup's LDS) or n whose multigrid coarsest grid exceeds 16 x 16
 * interior points; in 3D n odd, n < 4 or n > 256, or a coarsest grid beyond 4^3 points; K <= 0,
 * mu <= 0, or non-finite values.                                                             */
int fdd_setup_mesh(const fdd_desc* desc, int hip_device, fdd_problem* out);

/* The paper's own model problem (Sec. 3, eq. (model_problem)) in 2D:
 *     K (-Delta + I) x + gamma (-Delta_Gamma + I)^t x = b,   x in V = H^1(Omega), Omega = (0,1)^2,
 * with Gamma the whole boundary, P1 on the diagonal-split mesh of n cells per side (every node is
 * a dof).  In the form of eq. (generic): A = K (A_Omega + M_Omega) + gamma T^T L^t T, L = A_G + M_G
 * the P1 matrix of -Delta_Gamma + I on the closed boundary curve (4n nodes) and L^t as in
 * eq. (gevp).  Dof order: the (n-1)^2 interior nodes (index (j-1)(n-1) + (i-1), i fastest), then
 * the N_G = 4n boundary nodes counter-clockwise from the corner (0, 0): (i, 0) -> i, (n, j) ->
 * n + j, (i, n) -> 2n + (n - i), (0, j) -> 3n + (n - j).  The returned problem takes the same
 * calls as fdd_setup_mesh's (workspace, tables, interior solve, Schur and operator products,
 * preconditioner, fdd_solve); rational tables: FDD_RA_PRECOND approximates
 * (K lam^{1/2} + gamma lam^t)^{-1} (S_Gamma = K L^{1/2} + gamma L^t, Sec. 3) and
 * FDD_RA_OPERATOR lam^t for t < 0 or lam^(t-1) for t >= 0 (then L^t = L (table)(L)), on the
 * spectrum [1, 1 + 12 n^2] of (L, M_G).  The interior block A_II = A_Omega + M_Omega is solved
 * by PCG with the interior multigrid's V-cycles.  Not offered for it: warm starts, batches, the
 * full-system and static-scratch calls.  Host only.  Errors: FDD_E_ARG for n odd, n < 4,
 * n > 1024 (one loop vector per workgroup in LDS) or a coarsest grid beyond 16 x 16, K <= 0,
 * gamma < 0, t outside (-1, 1), or non-finite values.                                        */
int fdd_setup_model(int n, double K, double gamma, double t, int hip_device, fdd_problem* out);

/* The H(div) problem of Sec. 3's remark on H(div)-elliptic problems (eq. (graddiv)): find u in
 * V = H(div, Omega), Omega = (0,1)^2, with
 *     K int (u.v + div u div v) + gamma int_{dOmega} (u.nu)(v.nu) = <b, v>   for all v,
 * lowest-order Brezzi-Douglas-Marini elements (BDM1) on the diagonal-split mesh of n cells per
 * side, Gamma the whole boundary, trace space Q_h = discontinuous P1 on the 4n boundary segments.
 * Dofs: two per edge, the normal component u.n_e at the edge's first and at its second endpoint
 * (edge e holds dofs 2e, 2e + 1).  Edge order: interior horizontal (i,j)->(i+1,j), j = 1..n-1,
 * i = 0..n-1, n_e = (0,1), index (j-1)n + i; interior vertical (i,j)->(i,j+1), i = 1..n-1,
 * j = 0..n-1, n_e = (1,0), index n(n-1) + j(n-1) + i-1; diagonal (i,j)->(i+1,j+1), n_e =
 * (1,-1)/sqrt 2, index 2n(n-1) + jn + i; then the 4n boundary segments counter-clockwise from
 * (0,0) (bottom, right, top, left; first endpoint = the one met first), n_e = the outward normal,
 * index 3n^2 - 2n + k.  So N = 6n^2 + 4n, N_I = 6n^2 - 4n interior dofs and N_G = 8n trace dofs
 * (the DG P1 values of u.nu, segment by segment along the loop) last.
 * The preconditioner is S_Gamma = K L^{-1/2} + gamma I_Gamma with I_Gamma the DG P1 mass M_Q and
 * L the symmetric interior-penalty matrix of -u'' + u on the loop (penalty 4/h), both block
 * circulant; FDD_RA_PRECOND tables approximate f(lam)/lam = (K lam^{1/2} + gamma lam)^{-1} on the
 * spectrum of (L, M_Q) (f = (K lam^{-1/2} + gamma)^{-1}; the preconditioner applies
 * lam (table)(lam)).  The operator has no fractional term: the operator-table argument of
 * fdd_schur_apply, fdd_apply_operator and fdd_solve must be NULL, and FDD_RA_OPERATOR tables are
 * refused.  The interior block A^00 = K(I - grad div) on the zero-normal-trace subspace is
 * solved by PCG with a V-cycle (additive Schwarz over vertex patches, damping 1/2, opts.mg_nu
 * sweeps; nested BDM1 spaces, so the coarse matrices are the Galerkin ones); inner_rtol and
 * inner_maxit apply, precision and step_rtol do not (FP64 throughout).  Not offered for it: warm
 * starts, batches, the full-system and static-scratch calls.  Host only (assembly of every level
 * on the host; the workspace holds the matrices, uploaded by fdd_bind_workspace).
 * Errors: FDD_E_ARG for n not a power of two in [4, 1024] (one loop vector per workgroup in LDS),
 * K <= 0, gamma < 0 or non-finite values.                                                     */
int fdd_setup_hdiv(int n, double K, double gamma, int hip_device, fdd_problem* out);

/* Sizes: N free dofs, N_I interior, N_G interface; [lam_lo, lam_hi] encloses the discrete
 * spectrum of L_h w.r.t. M_h (2D: the exact extreme eigenvalues).  Host only.               */
int fdd_problem_info(fdd_problem prob, int64_t* N, int64_t* N_I, int64_t* N_G,
                     double* lam_lo, double* lam_hi);

/* Device bytes the solver needs for these options (host only). */
int fdd_workspace_bytes(fdd_problem prob, const fdd_opts* opts, size_t* bytes);

/* Binds caller-owned device memory (256-byte aligned, >= fdd_workspace_bytes) and initializes
 * it on `stream` (device call).  Errors: FDD_E_WORKSPACE if too small or misaligned.        */
int fdd_bind_workspace(fdd_problem prob, void* dev_ptr, size_t bytes, void* stream);

/* ---- rational approximation (eq. (RA)) ------------------------------------------------------
 * which = FDD_RA_PRECOND: f(lam) = (K lam^{1/2} + mu^{-1} lam^{-1/2})^{-1}, the symbol of
 *         S_Gamma^{-1} (eq. (schur_precond) with s = 1/2, t = -1/2).
 * which = FDD_RA_OPERATOR: g(lam) = lam^{-1/2}, so that H = M (d0 M^{-1} + sum d_k (L + q_k M)^{-1}) M.
 * Built on the host in FP64 by relative-error AAA on [lam_lo, lam_hi], keeping only real
 * shifts p_k >= 0, followed by a weighted least-squares refit of (c0, c_k).  `tol` is the
 * target max relative error on the spectrum, max_poles caps m (<= 64).  Host only.
 * Errors: FDD_E_RA if no admissible table meets 10 * tol.                                   */
int fdd_build_rational_pc(fdd_problem prob, int which, double tol, int max_poles, fdd_ratpc* out);

/* Wraps a caller-given table (host arrays of length m).  Rejects (FDD_E_RA) any shift p_k < 0
 * or non-finite entries, since L + p_k M must be SPD.  Host only.                            */
int fdd_ratpc_from_table(fdd_problem prob, int which, int m, double c0, const double* c,
                         const double* p, fdd_ratpc* out);

/* Reads a table back (host arrays with room for m entries; any pointer may be NULL).
 * max_rel_err: max |f - f_RA| / |f| over the sample set and, in 2D, the exact eigenvalues. */
int fdd_ratpc_query(fdd_ratpc t, int* m, double* c0, double* c, double* p, double* max_rel_err);

/* ---- operators ---------------------------------------------------------------------------- */

/* Interior Dirichlet solve A_II u = f (the leading block A^00 / K of eq. (block_op)), by
 * multigrid-preconditioned CG.  f, u: device, length N_I, free-dof order of the interior.
 * Synchronizes the stream.  its (may be NULL) receives the multigrid-PCG iteration count.   */
int fdd_interior_solve(fdd_problem prob, const double* f, double* u, const fdd_opts* opts,
                       void* stream, int* its);

/* y_G = S x_G with S = K (A_GG - A_GI A_II^{-1} A_IG) + gamma H_RA  (eq. (block_op); H by the
 * table H of kind FDD_RA_OPERATOR).  Synchronizes the stream (one interior solve).          */
int fdd_schur_apply(fdd_problem prob, fdd_ratpc H, const double* x_G, double* y_G,
                    const fdd_opts* opts, void* stream);

/* z_G = (c0 M^{-1} + sum_k c_k (A_G + p_k M_G)^{-1}) r_G with the table P of kind
 * FDD_RA_PRECOND (eq. (RA)); all m + 1 shifted systems are solved in one batched launch.
 * Asynchronous.                                                                              */
int fdd_precond_apply(fdd_problem prob, fdd_ratpc P, const double* r_G, double* z_G, void* stream);

/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same z_G as fdd_precond_apply (same kernels,
 * same summation order, bit-identical), with the systems' solutions staged in a library-owned
 * static device array of (64 + 1) x 2048 FP64 entries (1.02 MiB, held on each device the
 * library runs on until the process ends) instead of the bound workspace.  No workspace needs
 * to be bound (2D only); nothing is allocated.  Every call on one device shares that array, so
 * calls that overlap on one device (different streams, or threads) race: serialize them.
 * Errors: FDD_E_ARG for dim 3, or a table / interface size beyond the array (m + 1 > 65
 * systems or N_G > 2048); FDD_E_HIP if the array's device address cannot be found.
 * Asynchronous.                                                                              */
int fdd_precond_apply_static(fdd_problem prob, fdd_ratpc P, const double* r_G, double* z_G,
                             void* stream);

/* y = A x = K A_Omega x + gamma T^T H_RA T x on all N free dofs.  Asynchronous.             */
int fdd_apply_operator(fdd_problem prob, fdd_ratpc H, const double* x, double* y, void* stream);

/* ---- the solve -------------------------------------------------------------------------------
 * x = A^{-1} b: reduce to g = b_G - A_GI A_II^{-1} b_I, run PCG on S x_G = g from x_G = 0 with
 * preconditioner P (stop rule of Sec. 3), then back-substitute x_I = A_II^{-1}(b_I/K - A_IG x_G).
 * b, x: device, length N.  stats may be NULL.  Returns FDD_NOT_CONVERGED if outer_maxit was
 * reached (x holds the last iterate), FDD_E_BREAKDOWN / FDD_E_NONFINITE on breakdown.       */
int fdd_solve(fdd_problem prob, fdd_ratpc P, fdd_ratpc H, const double* b, double* x,
              const fdd_opts* opts, void* stream, fdd_stats* stats);

/* ---- full-system PCG with the lazy block preconditioner -------------------------------------
 * The preconditioner of eq. (dd_preconditioner) in the form of the paper's remark on evaluating
 * the operator (Sec. 3, Fig. 4-left), 2D only: the leading block (A^00)^{-1} = (K A_II)^{-1} is
 * replaced by one multigrid V-cycle V / K (the interior solver's symmetric V(nu, nu) cycle,
 * nu = opts->mg_nu; FP64 arithmetic for opts->precision = FDD_FP64, FP32 for FDD_MIXED) and
 * S_Gamma^{-1} by the table P (eq. (RA)):
 *     t_G = r_G - A_GI V r_I,   z_G = S_Gamma^{-1} t_G,   z_I = V (r_I - K A_IG z_G) / K.
 * fdd_dd_precond_apply: z = B r on all N free dofs (r, z: device, length N, caller layout).
 * Asynchronous.  Errors: FDD_E_ARG (dim 3, null vector, invalid options), FDD_E_STATE (a
 * table of another problem or kind), FDD_E_WORKSPACE (none bound).                          */
int fdd_dd_precond_apply(fdd_problem prob, fdd_ratpc P, const double* r, double* z,
                         const fdd_opts* opts, void* stream);
/* fdd_solve_full: x = A^{-1} b by PCG on the whole system, A = K A_Omega + gamma T^T H_RA T with
 * H by the table H (so every iteration costs two V-cycles, two batches of shifted interface
 * solves and two stencil passes, and no interior solve), preconditioned by B above; x_0 = 0,
 * stop when (r^T z)^{1/2} <= outer_rtol (r_0^T z_0)^{1/2} (Sec. 3).  inner_rtol, step_rtol and
 * use_graph are not used (eager launches, one read-back per iteration).  stats: outer_its = PCG
 * iterations, inner_solves = V-cycles, true_rel_res if check_true_residual.  Returns
 * FDD_NOT_CONVERGED after outer_maxit iterations (x holds the last iterate), FDD_E_BREAKDOWN /
 * FDD_E_NONFINITE on breakdown.  Synchronizes the stream once per iteration.                */
int fdd_solve_full(fdd_problem prob, fdd_ratpc P, fdd_ratpc H, const double* b, double* x,
                   const fdd_opts* opts, void* stream, fdd_stats* stats);

/* ---- the Darcy-Stokes outer solver (Sec. 4, eq. (darcy_stokes), eq. (darcy_stokes_precond)) --
 * The coupled problem: Stokes velocity u and pressure p_S on Omega_S = (0,1) x (1,2), Darcy
 * pressure p_D on Omega_D = (0,1)^2, interface Gamma = (0,1) x {1} with nu = (0,-1) (out of
 * Omega_S); no slip on the Stokes sides x = 0, 1, zero traction on the Stokes top y = 2, p_D = 0
 * on the rest of the Darcy boundary; on Gamma mass conservation u.nu + K grad p_D . nu = 0,
 * normal stress balance -nu.sigma nu = p_D and the Beavers-Joseph-Saffman condition
 * -P_nu(sigma nu) = alpha mu K^{-1/2} P_nu u, with sigma = mu grad u - p_S I.  Taylor-Hood P2-P1
 * for Stokes and P1 for p_D on the diagonal-split meshes of n cells per side (matching on Gamma).
 * Symmetric weak form (the Darcy equation multiplied by -1):
 *     [A_u  B^T  C    ] [u  ]   A_u: mu int grad u : grad v + alpha mu K^{-1/2} int_Gamma u_x v_x
 *     [B    0    0    ] [p_S]   B: -int q div v       C: int_Gamma q_D v.nu = -int_Gamma q_D v_y
 *     [C^T  0    -K A_D] [p_D]   A_D: the facet problem's stiffness (fdd_setup_mesh, dim 2)
 * Unknown order: u_x then u_y at the P2 nodes (A h/2, 1 + B h/2), A = 1..2n-1, B = 0..2n, index
 * c (2n-1)(2n+1) + B (2n-1) + (A-1); p_S at the vertices (i h, 1 + j h), index Nu + j (n+1) + i;
 * p_D in the facet problem's order (interior points row by row, Gamma last), index Nu + Np + k.
 * Nu = 2 (2n-1)(2n+1), Np = (n+1)^2, ND = n (n-1).
 *
 * fdd_setup_darcy_stokes: host set-up of every matrix (and of the facet problem of the Darcy
 * block, with the same n, K, mu); krylov = the FGMRES basis the workspace holds (iterations
 * without restart).  fdd_problem_info gives N = Nu + Np + ND, N_I = Nu + Np, N_G = ND and the
 * facet problem's spectral interval; fdd_build_rational_pc / fdd_ratpc_from_table on this problem
 * build the facet problem's tables (the preconditioner's S_Gamma and the operator's H of the
 * Darcy block); fdd_workspace_bytes / fdd_bind_workspace cover both parts; fdd_apply_operator
 * (table NULL) applies the coupled operator above.  Host only.  Errors: FDD_E_ARG for n not a
 * power of two in [8, 1024], K <= 0, mu <= 0, alpha < 0, non-finite values, or krylov outside
 * [1, 400].                                                                                   */
int fdd_setup_darcy_stokes(int n, double K, double mu, double alpha, int krylov, int hip_device,
                           fdd_problem* out);
int fdd_ds_sizes(fdd_problem prob, int64_t* Nu, int64_t* Np, int64_t* ND);

/* Options of the outer solver and of the preconditioner's blocks (fdd_ds_opts_default fills
 * the defaults given below). */
typedef struct {
  double rtol;            /* FGMRES: stop when ||b - A x_k||_2 <= rtol ||b||_2 (1e-10)         */
  int maxit;              /* FGMRES iterations, capped by the problem's krylov (400)          */
  double velocity_rtol;   /* A_u block: PCG with the P2 multigrid V-cycle to this relative
                             residual (1e-12); 0: one V-cycle instead (the setting of Sec. 4) */
  int velocity_maxit;     /* (100) */
  int mg_nu;              /* smoothing steps of the velocity V-cycle, 1 (default: the PCG to
                             velocity_rtol) or 2 (the better choice for one V-cycle)          */
  double pressure_rtol;   /* mu^{-1} M_p block: Jacobi-preconditioned Chebyshev iteration on the
                             spectrum [1/2, 2] of D^{-1} M_p with the step count that bounds the
                             relative residual by this (1e-12: 27 steps)                      */
  int pressure_maxit;     /* cap on those steps (200) */
  double darcy_rtol;      /* Darcy block: fdd_solve_full on the facet problem to this relative
                             preconditioned residual (1e-5, the Appendix; Sec. 4: 1e-4)      */
  int darcy_maxit;        /* (200) */
  int darcy_precision;    /* FDD_FP64 (default) or FDD_MIXED: the Darcy PCG's V-cycles        */
  int darcy_mg_nu;        /* (2) */
  int check_true_residual; /* nonzero (default): ||b - A x|| / ||b|| of the returned x        */
} fdd_ds_opts;

typedef struct {
  int status;
  int its;                  /* FGMRES iterations                                             */
  int velocity_its_total;   /* PCG iterations (or V-cycles) of the velocity block, summed     */
  int velocity_its_max;
  int pressure_its_total;   /* Chebyshev steps of the pressure block, summed                  */
  int darcy_its_total;      /* PCG iterations of the Darcy block, summed                      */
  int darcy_its_max;
  double rel_res;           /* FGMRES's least-squares residual / ||b||                        */
  double true_rel_res;      /* ||b - A x||_2 / ||b||_2 if requested, else -1                  */
  double t_solve_ms;        /* host wall time                                                 */
} fdd_ds_stats;

void fdd_ds_opts_default(fdd_ds_opts* opts);

/* fdd_ds_precond_apply: z = B r, the block-diagonal preconditioner of eq. (darcy_stokes_precond)
 *     B = diag(A_u, mu^{-1} M_p, K A_D + mu^{-1} T^T H T)^{-1},
 * its blocks applied by the inner solves of the options (the Darcy block by the full-system PCG
 * of fdd_solve_full with tables P and H).  r, z: device, length N.  Synchronizes the stream.
 * fdd_ds_solve: x = A^{-1} b by flexible GMRES (right preconditioned by B, x_0 = 0, no restart,
 * Arnoldi by classical Gram-Schmidt applied twice); stops when the least-squares residual
 * ||b - A x_k||_2 <= rtol ||b||_2.  Returns FDD_NOT_CONVERGED after maxit iterations (x holds
 * the last iterate), FDD_E_NONFINITE on non-finite values, and the errors of the inner solves.
 * Synchronizes the stream at least once per iteration.
 * Errors: FDD_E_ARG (not a Darcy-Stokes problem, null vector, invalid options), FDD_E_STATE
 * (tables of another problem or kind), FDD_E_WORKSPACE (none bound).                          */
int fdd_ds_precond_apply(fdd_problem prob, fdd_ratpc P, fdd_ratpc H, const double* r, double* z,
                         const fdd_ds_opts* opts, void* stream, fdd_ds_stats* stats);
int fdd_ds_solve(fdd_problem prob, fdd_ratpc P, fdd_ratpc H, const double* b, double* x,
                 const fdd_ds_opts* opts, void* stream, fdd_ds_stats* stats);

/* ---- batched solves -------------------------------------------------------------------------
 * Many independent problems of possibly different n, K, mu (and tables) solved together: the
 * same method as fdd_solve, applied to every instance, with each kernel launch covering all
 * instances (one grid over the concatenated multigrid tiles of every instance, one grid over all
 * shifted interface systems of eq. (RA) of every instance).  Each instance runs its own outer
 * PCG with its own stop rule; an instance that has converged is skipped by the kernels of later
 * iterations.  All instances share one launch schedule, and each outer iteration of the batch
 * is replayed from a captured hipGraph (opts->use_graph).  Only FDD_MIXED precision.
 * opts->warmstart may name a network (fdd_cnn) whose batch_max covers the whole batch and whose
 * n_max covers every instance: each outer iteration then runs one forward pass per group of
 * instances of equal n on their search directions and starts every lifted interior solve from
 * its instance's guess, scaled by its Galerkin factor (as in fdd_solve).
 *
 * fdd_batch_create: count >= 1 distinct problems, each with its own workspace bound, and their
 * tables (P[i] of kind FDD_RA_PRECOND and H[i] of kind FDD_RA_OPERATOR built for probs[i]).
 * The batch keeps pointers to the problems and tables: they must outlive it and keep their
 * workspaces.  Host only.  Errors: FDD_E_ARG (empty, duplicate problem, mixed devices),
 * FDD_E_WORKSPACE (a problem without workspace), FDD_E_STATE (a table of the wrong problem). */
int fdd_batch_create(int count, const fdd_problem* probs, const fdd_ratpc* P, const fdd_ratpc* H,
                     fdd_batch* out);
/* Device bytes of the batch's own workspace (descriptors, work lists, tables).  Host only. */
int fdd_batch_workspace_bytes(fdd_batch batch, size_t* bytes);
/* Binds caller-owned device memory (256-byte aligned) to the batch and initializes it on
 * `stream`; synchronizes the stream.  Errors: FDD_E_WORKSPACE.                              */
int fdd_batch_bind_workspace(fdd_batch batch, void* dev_ptr, size_t bytes, void* stream);
/* Tile edge of the intermediate multigrid levels (every level below the finest that runs tiled
 * kernels; the finest level always runs 32 x 32 tiles): 16 or 32 for every such level, or 0 (the
 * default) to choose per level by tile count (16 x 16 where the batch has fewer than four
 * 32 x 32 tiles per compute unit on that level).  A change drops the batch's captured graphs and
 * re-uploads its tile lists at the next solve; results are the same up to rounding order (the
 * levels' arithmetic does not depend on the tiling).  Host only.  Errors: FDD_E_ARG.       */
int fdd_batch_set_mid_tile(fdd_batch batch, int edge);
/* *levels = number of tiled levels; edges (NULL or room for 16 entries) = tile edge per level. */
int fdd_batch_tile_edges(fdd_batch batch, int* levels, int* edges);
/* x[i] = A_i^{-1} b[i] for every instance.  b, x: host arrays of `count` device pointers (each
 * of length N of its problem).  stats: NULL or an array of `count` entries (per-instance
 * status, iteration counts and residuals; t_solve_ms is the batch's wall time).  Returns
 * FDD_NOT_CONVERGED if any instance hit outer_maxit (that instance's x holds its last
 * iterate), or an error code on breakdown or invalid input (the message names the instance).
 * Returns after the whole batch has finished.                                                */
int fdd_solve_batched(fdd_batch batch, const double* const* b, double* const* x,
                      const fdd_opts* opts, void* stream, fdd_stats* stats);
void fdd_batch_destroy(fdd_batch batch);

/* ---- learned warm start ----------------------------------------------------------------------
 * A convolutional network predicts the discrete harmonic extension E t (the interior solution of
 * A_II u = lift(t), eq. (block_op)) of an interface trace t, as the initial guess of the interior
 * solves inside the outer PCG.  Six 3x3 'same' convolutions, widths 5 -> 32 (x5) -> 1, exact
 * GELU after the first five; BF16 weights and activations with FP32 accumulation on the matrix
 * cores.  Input channels of an image (n - 1 rows j, n - 1 columns i): t_i / s, y = j / n,
 * y t_i / s, log10 K, log10 mu, with s the root-mean-square of t.  Parameters: one FP32 device
 * vector, per layer W[3][3][c_in][c_out] then b[c_out] (fdd_cnn_param_count entries); they are
 * owned by the caller, as are gradients and Adam moments.  Images and outputs are row-major
 * (row j - 1, column i - 1), i.e. the interior free-dof order.
 *
 * fdd_cnn_create: sizes for up to batch_max images of up to n_max (n - 1 pixels a side); train
 * != 0 keeps the activations for fdd_cnn_backward.  Host only.  Errors: FDD_E_ARG.          */
int fdd_cnn_create(int batch_max, int n_max, int train, int hip_device, fdd_cnn* out);
int fdd_cnn_param_count(fdd_cnn cnn, int64_t* count);
int fdd_cnn_workspace_bytes(fdd_cnn cnn, size_t* bytes);
/* Binds caller-owned device memory (256-byte aligned).  Parameters must be set again after.  */
int fdd_cnn_bind_workspace(fdd_cnn cnn, void* dev_ptr, size_t bytes, void* stream);
/* Converts the FP32 parameters to the BF16 layouts the kernels read (asynchronous).          */
int fdd_cnn_set_params(fdd_cnn cnn, const float* theta, void* stream);
/* out (FP32, batch x (n-1)^2) = network(features of traces[b] (row stride ld >= n - 1),
 * log10K[b], log10mu[b]); rescale != 0 multiplies image b by s_b (the guess for t itself),
 * else the output is that for t / s_b.  All pointers device.  Asynchronous.                  */
int fdd_cnn_forward(fdd_cnn cnn, const double* traces, int ld, int batch, int n,
                    const double* log10K, const double* log10mu, float* out, int rescale,
                    void* stream);
/* Mean squared error of out against target (both batch x (n-1)^2, FP32, device) into *loss
 * (device double; NULL: internal), and its gradient for fdd_cnn_backward.  Asynchronous.     */
int fdd_cnn_loss(fdd_cnn cnn, const float* out, const float* target, int batch, int n,
                 double* loss, void* stream);
/* grad (FP32, parameter layout) = gradient of the last loss against the parameters, through the
 * last forward pass (same batch and n).  Deterministic.  Asynchronous.                       */
int fdd_cnn_backward(fdd_cnn cnn, int batch, int n, float* grad, void* stream);
/* One Adam step (Kingma and Ba 2015) on theta with moments m, v (FP32, device); step >= 1. */
int fdd_cnn_adam_step(fdd_cnn cnn, float* theta, const float* grad, float* m, float* v, float lr,
                      float b1, float b2, float eps, int step, void* stream);
void fdd_cnn_destroy(fdd_cnn cnn);

/* ---- measurement ---------------------------------------------------------------------------
 * Times every launch of one kernel kind with a pair of HIP events attached to that kernel's own
 * dispatch on the stream it is launched on (hipExtLaunchKernelGGL: stamped at kernel begin and
 * end); events are harvested at the solver's synchronization points.  While a timer is set,
 * fdd_solve launches eagerly.  Setting a timer resets the totals.
 * kind: FDD_KT_NONE (off), FDD_KT_DOWN0 (finest-level down kernel carrying the PCG update),
 * FDD_KT_UP0 (finest-level up kernel producing z, A z and the dots), FDD_KT_COARSE (the
 * single-workgroup coarse-level V-cycle).  Host call; creates events on first use.          */
enum { FDD_KT_NONE = 0, FDD_KT_DOWN0 = 1, FDD_KT_UP0 = 2, FDD_KT_COARSE = 3 };
/* split_us: launches lasting at least this long are also counted separately ("long" launches:
 * those that did their work, as opposed to launches that returned at once because their solve
 * had already converged).                                                                     */
int fdd_set_kernel_timer(fdd_problem prob, int kind, double split_us);
/* launches / total_ms: all timed launches and their summed durations; long_launches / long_ms:
 * the same for launches of at least split_us; untimed: launches missed because more than 4096
 * were pending between two synchronizations.  Any pointer may be NULL.                        */
int fdd_get_kernel_timer(fdd_problem prob, int64_t* launches, double* total_ms,
                         int64_t* long_launches, double* long_ms, int64_t* untimed);
/* The same timer for the batched kernels of a batch (FDD_KT_DOWN0 / FDD_KT_UP0: the finest-level
 * kernels over the tiles of all instances; FDD_KT_COARSE: the coarse-level kernel, one workgroup
 * per instance).  While set, fdd_solve_batched launches eagerly.                              */
int fdd_batch_set_kernel_timer(fdd_batch batch, int kind, double split_us);
int fdd_batch_get_kernel_timer(fdd_batch batch, int64_t* launches, double* total_ms,
                               int64_t* long_launches, double* long_ms, int64_t* untimed);

void fdd_destroy_problem(fdd_problem prob);
void fdd_destroy_ratpc(fdd_ratpc t);
const char* fdd_last_error(void);
const char* fdd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FDD_H */
