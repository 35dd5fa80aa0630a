// The coupled Darcy-Stokes problem (Sec. 4, eq. (darcy_stokes); Appendix) on the C ABI: flexible
// GMRES on the whole system, right-preconditioned by the block-diagonal operator of eq.
// (darcy_stokes_precond),
//
//   B = diag(A_u, mu^{-1} M_p, K A_D + mu^{-1} T^T H T)^{-1},
//
// whose blocks are applied by
//   * A_u (mu-Laplacian of the P2 velocity plus the Beavers-Joseph-Saffman term on Gamma): PCG
//     with a multigrid V-cycle (nested P2 spaces, additive Schwarz over vertex patches) to a
//     relative tolerance, or one V-cycle (the setting of Sec. 4);
//   * mu^{-1} M_p (P1 Stokes pressure mass): Jacobi-preconditioned Chebyshev iteration with the
//     step count that guarantees a relative tolerance (the spectrum of D^{-1} M_p is known);
//   * the Darcy block, the Riesz map of eq. (riesz) with gamma = 1/mu: PCG on the facet problem
//     with the lazy preconditioner of eq. (dd_preconditioner) (one V-cycle for the leading block,
//     the rational table for S_Gamma, H by its rational table in the operator) to a relative
//     tolerance (Sec. 4: 1e-4; Appendix: 1e-5).
// The inner solves stop at tolerances, so the preconditioner varies between applications; FGMRES
// keeps the preconditioned directions Z and stays minimal in the residual for that reason.
// Every step runs in kernels; the host enqueues them and reads the stop flags back.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "api_internal.h"
#include "ds_internal.h"
#include "ell_mg.h"

using namespace fdd;

namespace {

constexpr double kThetaU = 0.5;   // damping of the velocity smoother (overlapping vertex patches)

// The P1 pressure mass under Jacobi: on a triangle, D_T^{-1} M_T (D_T = diag(M_T) = |T|/6 I,
// M_T = |T|/12 (I + 1 1^T)) has eigenvalues 1/2 (twice) and 2; since x^T M x = sum_T x_T^T M_T x_T
// and D = sum_T D_T, the spectrum of D^{-1} M_p lies in [1/2, 2].  Chebyshev on that interval
// reduces the residual in the D^{-1} norm by 2 rho^k after k steps, rho = (sqrt(4) - 1) /
// (sqrt(4) + 1) = 1/3; the diagonal varies by at most a factor 6 (one to six triangles at a
// vertex), so the Euclidean residual falls by 2 sqrt(6) rho^k.
constexpr double kMassLo = 0.5, kMassHi = 2.0;

int cheb_steps(double rtol, int maxit) {
  const double rho = 1.0 / 3.0;
  const int k = (int)std::ceil(std::log(rtol / (2.0 * std::sqrt(6.0))) / std::log(rho));
  return std::max(1, std::min(k, maxit));
}

// x = M_p^{-1} b by `steps` Jacobi-Chebyshev steps (x_0 = 0); returns the buffer holding x
const double* mass_solve(const ProblemDS* D, hipStream_t s, int steps, const double* b) {
  const double theta = 0.5 * (kMassHi + kMassLo), delta = 0.5 * (kMassHi - kMassLo);
  const double sigma = theta / delta;
  double* cur = D->pz;
  double* nxt = D->pq;
  launch_hd_cheb_step(s, D->mass, b, nullptr, cur, D->pp, 0.0, 1.0 / theta, 1);
  double rho_prev = 1.0 / sigma;
  for (int k = 1; k < steps; ++k) {
    const double rho = 1.0 / (2.0 * sigma - rho_prev);
    launch_hd_cheb_step(s, D->mass, b, cur, nxt, D->pp, rho * rho_prev, 2.0 * rho / delta, 0);
    std::swap(cur, nxt);
    rho_prev = rho;
  }
  return cur;
}

EllHier hier_u(const ProblemDS* D) {
  EllHier H;
  H.lev = D->lev;
  H.nlev = D->nlev;
  H.cinv = D->dcinv;
  H.theta = kThetaU;
  H.n0 = D->Nu;
  H.r = D->ur;
  H.z = D->uz;
  H.p = D->up;
  H.q = D->uq;
  H.partials = D->partials;
  H.st = D->st_u;
  H.hst = D->hst_u;
  return H;
}

int read_ds(ProblemDS* D, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(D->hst, D->st, sizeof(DsState), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

// y = A x, the three row blocks
void apply_op(const ProblemDS* D, hipStream_t s, const double* x, double* y) {
  launch_hd_spmv(s, view(D->Au), x, y, 1.0, 0.0, nullptr);
  launch_hd_spmv(s, view(D->Bp), x, y + D->Nu, 1.0, 0.0, nullptr);
  launch_hd_spmv(s, view(D->Dd), x, y + D->Nu + D->Np, 1.0, 0.0, nullptr);
}

bool ds_opts_ok(const fdd_ds_opts& o) {
  return o.rtol > 0 && o.rtol < 1 && o.maxit >= 1 && o.velocity_rtol >= 0 &&
         o.velocity_rtol < 1 && o.velocity_maxit >= 1 && (o.mg_nu == 1 || o.mg_nu == 2) &&
         o.pressure_rtol > 0 && o.pressure_rtol < 1 && o.pressure_maxit >= 1 &&
         o.darcy_rtol > 0 && o.darcy_rtol < 1 && o.darcy_maxit >= 1 &&
         (o.darcy_precision == FDD_FP64 || o.darcy_precision == FDD_MIXED) &&
         (o.darcy_mg_nu == 1 || o.darcy_mg_nu == 2);
}

// z = B r (one application of every block), counts into st
int precond(fdd_problem_s* P, const fdd_ratpc_s* PT, const fdd_ratpc_s* HT, const fdd_ds_opts& o,
            hipStream_t s, const double* r, double* z, fdd_ds_stats* st) {
  ProblemDS* D = P->pds;
  const int Nu = D->Nu, Np = D->Np;
  int its = 0, rc;
  // velocity
  if (o.velocity_rtol > 0) {
    rc = ell_pcg(hier_u(D), s, o.mg_nu, o.velocity_rtol, o.velocity_maxit, r, z, &D->its_u, &its,
                 "Darcy-Stokes velocity block");
    if (rc) return rc;
  } else {
    ell_vcycle(hier_u(D), s, o.mg_nu, 0, r, z, nullptr);
    its = 1;
  }
  st->velocity_its_total += its;
  st->velocity_its_max = std::max(st->velocity_its_max, its);
  // Stokes pressure: (mu^{-1} M_p)^{-1} r_p = mu M_p^{-1} r_p
  const int steps = cheb_steps(o.pressure_rtol, o.pressure_maxit);
  launch_ds_scale(s, Np, D->mu, mass_solve(D, s, steps, r + Nu), z + Nu);
  st->pressure_its_total += steps;
  // Darcy: PCG on the Riesz map with the lazy preconditioner
  fdd_opts fo;
  fdd_opts_default(&fo);
  fo.outer_rtol = o.darcy_rtol;
  fo.outer_maxit = o.darcy_maxit;
  fo.precision = o.darcy_precision;
  fo.mg_nu = o.darcy_mg_nu;
  fo.check_true_residual = 0;
  fdd_stats ds;
  rc = fdd_solve_full(D->darcy, const_cast<fdd_ratpc>(PT), const_cast<fdd_ratpc>(HT), r + Nu + Np,
                      z + Nu + Np, &fo, s, &ds);
  if (rc) return rc;
  st->darcy_its_total += ds.outer_its;
  st->darcy_its_max = std::max(st->darcy_its_max, ds.outer_its);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int check_ds(fdd_problem_s* P, const fdd_ratpc_s* PT, const fdd_ratpc_s* HT, const void* in,
             const void* out, const fdd_ds_opts& o) {
  int rc = check_problem(P);
  if (rc) return rc;
  if (P->kind != kProblemDarcyStokes) return fail(FDD_E_ARG, "not a Darcy-Stokes problem");
  if (!in || !out) return fail(FDD_E_ARG, "null vector");
  if (!ds_opts_ok(o)) return fail(FDD_E_ARG, "invalid Darcy-Stokes options");
  if ((rc = check_table(P->pds->darcy, PT, FDD_RA_PRECOND))) return rc;
  return check_table(P->pds->darcy, HT, FDD_RA_OPERATOR);
}

}  // namespace

namespace fdd {

size_t ds_workspace_bytes(fdd_problem_s* P) {
  size_t nd = 0;
  if (fdd_workspace_bytes(P->pds->darcy, nullptr, &nd)) return 0;
  return (nd + 255) / 256 * 256 + ds_plan(P->pds, nullptr);
}

int ds_bind(fdd_problem_s* P, void* dev, size_t bytes, hipStream_t s) {
  ProblemDS* D = P->pds;
  size_t nd = 0;
  int rc = fdd_workspace_bytes(D->darcy, nullptr, &nd);
  if (rc) return rc;
  nd = (nd + 255) / 256 * 256;
  const size_t need = nd + ds_plan(D, nullptr);
  if (bytes < need) return fail(FDD_E_WORKSPACE, "workspace %zu bytes < %zu needed", bytes, need);
  if ((rc = fdd_bind_workspace(D->darcy, dev, nd, s))) return rc;
  HIPCHK(hipSetDevice(P->device));
  char* base = (char*)dev + nd;
  P->ws = (char*)dev;
  P->ws_bytes = bytes;
  ds_plan(D, base);
  if (!D->hst) HIPCHK(hipHostMalloc((void**)&D->hst, sizeof(DsState), hipHostMallocDefault));
  if (!D->hst_u) HIPCHK(hipHostMalloc((void**)&D->hst_u, sizeof(HdState), hipHostMallocDefault));
  HIPCHK(hipMemsetAsync(base, 0, need - nd, s));
  auto up = [&](void* dst, const void* src, size_t nb) -> int {
    if (nb) HIPCHK(hipMemcpyAsync(dst, src, nb, hipMemcpyHostToDevice, s));
    return FDD_OK;
  };
  auto upm = [&](const HdMat& M) -> int {
    int r = M.toff.empty() ? up(M.dcol, M.col.data(), M.col.size() * sizeof(int))
                           : up(M.dtoff, M.toff.data(), M.toff.size() * sizeof(int));
    if (!r) r = up(M.drtype, M.rtype.data(), M.rtype.size() * sizeof(int));
    return r ? r : up(M.dtval, M.tval.data(), M.tval.size() * sizeof(double));
  };
  auto upl = [&](const HdLevel& L, bool transfers) -> int {
    int r = upm(L.A);
    if (!r && transfers) r = upm(L.P);
    if (!r && transfers) r = upm(L.R);
    if (!r) r = up(L.dpatch, L.patch.data(), L.patch.size() * sizeof(int));
    if (!r) r = up(L.dptype, L.ptype.data(), L.ptype.size() * sizeof(int));
    if (!r) r = up(L.dslot, L.slot.data(), L.slot.size() * sizeof(int));
    return r ? r : up(L.dpinv, L.pinv.data(), L.pinv.size() * sizeof(double));
  };
  for (int l = 0; l < D->nlev && !rc; ++l) rc = upl(D->lev[l], l + 1 < D->nlev);
  if (!rc) rc = upl(D->mass, false);
  if (!rc) rc = up(D->dcinv, D->cinv.data(), D->cinv.size() * sizeof(double));
  if (!rc) rc = upm(D->Au);
  if (!rc) rc = upm(D->Bp);
  if (!rc) rc = upm(D->Dd);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

void ds_destroy(fdd_problem_s* P) {
  if (!P->pds) return;
  ProblemDS* D = P->pds;
  fdd_destroy_problem(D->darcy);
  if (D->hst) (void)hipHostFree(D->hst);
  if (D->hst_u) (void)hipHostFree(D->hst_u);
  delete D;
  P->pds = nullptr;
}

int ds_apply_operator(fdd_problem_s* P, const double* x, double* y, hipStream_t s) {
  apply_op(P->pds, s, x, y);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

}  // namespace fdd

extern "C" {

void fdd_ds_opts_default(fdd_ds_opts* o) {
  std::memset(o, 0, sizeof(*o));
  o->rtol = 1e-10;
  o->maxit = kDsMaxKrylov;
  o->velocity_rtol = 1e-12;
  o->velocity_maxit = 100;
  o->mg_nu = 1;
  o->pressure_rtol = 1e-12;
  o->pressure_maxit = 200;
  o->darcy_rtol = 1e-5;
  o->darcy_maxit = 200;
  o->darcy_precision = FDD_FP64;
  o->darcy_mg_nu = 2;
  o->check_true_residual = 1;
}

int fdd_setup_darcy_stokes(int n, double K, double mu, double alpha, int krylov, int hip_device,
                           fdd_problem* out) {
  if (!out) return fail(FDD_E_ARG, "null argument");
  *out = nullptr;
  if (n < 2 * kDsCoarseN || n > kDsMaxN || (n & (n - 1)))
    return fail(FDD_E_ARG, "Darcy-Stokes problem: n must be a power of two, %d <= n <= %d (got %d)",
                2 * kDsCoarseN, kDsMaxN, n);
  if (!(K > 0) || !std::isfinite(K) || !(mu > 0) || !std::isfinite(mu) || !(alpha >= 0) ||
      !std::isfinite(alpha))
    return fail(FDD_E_ARG, "Darcy-Stokes problem: K > 0, mu > 0 and alpha >= 0 must be finite");
  if (krylov < 1 || krylov > kDsMaxKrylov)
    return fail(FDD_E_ARG, "Darcy-Stokes problem: krylov must be in [1, %d]", kDsMaxKrylov);
  fdd_desc dd{2, n, K, mu};
  fdd_problem darcy = nullptr;
  int rc = fdd_setup_mesh(&dd, hip_device, &darcy);
  if (rc) return rc;
  fdd_problem_s* P = new (std::nothrow) fdd_problem_s();
  ProblemDS* D = P ? new (std::nothrow) ProblemDS() : nullptr;
  if (!D) {
    delete P;
    fdd_destroy_problem(darcy);
    return fail(FDD_E_NOMEM, "out of host memory");
  }
  P->pds = D;
  D->darcy = darcy;
  if (const char* err = ds_build(D, n, K, mu, alpha, krylov)) {
    fdd_destroy_problem(P);
    return fail(FDD_E_ARG, "Darcy-Stokes problem set-up: %s", err);
  }
  P->dim = 2;
  P->kind = kProblemDarcyStokes;
  P->n = n;
  P->device = hip_device;
  P->K = K;
  P->mu = mu;
  P->gamma = 1.0 / mu;
  P->h = 1.0 / n;
  P->tpow = darcy->tpow;
  P->N = D->N;
  P->NI = D->Nu + D->Np;
  P->NG = D->ND;
  // rational tables are those of the Darcy block (the facet problem's spectrum)
  P->eig = darcy->eig;
  P->lam_lo = darcy->lam_lo;
  P->lam_hi = darcy->lam_hi;
  *out = P;
  return FDD_OK;
}

int fdd_ds_sizes(fdd_problem P, int64_t* Nu, int64_t* Np, int64_t* ND) {
  if (!P || P->kind != kProblemDarcyStokes) return fail(FDD_E_ARG, "not a Darcy-Stokes problem");
  if (Nu) *Nu = P->pds->Nu;
  if (Np) *Np = P->pds->Np;
  if (ND) *ND = P->pds->ND;
  return FDD_OK;
}

int fdd_ds_precond_apply(fdd_problem P, fdd_ratpc PT, fdd_ratpc HT, const double* r, double* z,
                         const fdd_ds_opts* opts, void* stream, fdd_ds_stats* stats) {
  fdd_ds_opts o;
  if (opts) o = *opts;
  else fdd_ds_opts_default(&o);
  int rc = check_ds(P, PT, HT, r, z, o);
  if (rc) return rc;
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  fdd_ds_stats st;
  std::memset(&st, 0, sizeof(st));
  st.true_rel_res = -1.0;
  rc = precond(P, PT, HT, o, s, r, z, &st);
  if (!rc) {
    HIPCHK(hipStreamSynchronize(s));
  }
  st.status = rc;
  if (stats) *stats = st;
  return rc;
}

int fdd_ds_solve(fdd_problem P, fdd_ratpc PT, fdd_ratpc HT, const double* b, double* x,
                 const fdd_ds_opts* opts, void* stream, fdd_ds_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  fdd_ds_opts o;
  if (opts) o = *opts;
  else fdd_ds_opts_default(&o);
  int rc = check_ds(P, PT, HT, b, x, o);
  if (rc) return rc;
  HIPCHK(hipSetDevice(P->device));
  hipStream_t s = (hipStream_t)stream;
  ProblemDS* D = P->pds;
  const int N = D->N, ldh = D->krylov + 1;
  const int maxit = std::min(o.maxit, D->krylov);
  fdd_ds_stats st;
  std::memset(&st, 0, sizeof(st));
  st.true_rel_res = -1.0;
  auto finish = [&](int code) {
    st.status = code;
    st.t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return code;
  };
  launch_ds_start(s, N, b, D->V, D->g, D->partials, D->st);
  HIPCHK(hipGetLastError());
  if ((rc = read_ds(D, s))) return finish(rc);
  int its = 0;
  while (!D->hst->done && its < maxit) {
    const int k = its;
    double* w = D->V + (size_t)(k + 1) * N;
    if ((rc = precond(P, PT, HT, o, s, D->V + (size_t)k * N, D->Z + (size_t)k * N, &st)))
      return finish(rc);
    apply_op(D, s, D->Z + (size_t)k * N, w);
    launch_ds_orthogonalize(s, N, k, D->V, w, D->Hm + (size_t)k * ldh, D->hp, D->partials, D->st);
    launch_ds_normalize_givens(s, N, k, ldh, w, D->Hm, D->cs, D->sn, D->g, D->partials, D->st,
                               o.rtol);
    HIPCHK(hipGetLastError());
    if ((rc = read_ds(D, s))) return finish(rc);
    its = D->hst->its;
  }
  const DsState h = *D->hst;
  st.its = its;
  if (h.breakdown & 4)
    return finish(fail(FDD_E_NONFINITE, "Darcy-Stokes FGMRES: non-finite value at iteration %d", its));
  launch_ds_solution(s, N, its, ldh, D->Hm, D->g, D->y, D->Z, x);
  st.rel_res = h.beta > 0 ? h.res / h.beta : 0.0;
  if (o.check_true_residual)
    launch_ds_true_residual(s, view(D->Au), view(D->Bp), view(D->Dd), b, x, D->partials, D->st);
  HIPCHK(hipGetLastError());
  if ((rc = read_ds(D, s))) return finish(rc);
  if (o.check_true_residual && D->hst->t_res[1] > 0)
    st.true_rel_res = std::sqrt(D->hst->t_res[0] / D->hst->t_res[1]);
  return finish(h.done ? FDD_OK : FDD_NOT_CONVERGED);
}

}  // extern "C"
