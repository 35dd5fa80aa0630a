// The H(div) variant of the interface-perturbed problem (Sec. 3, remark on H(div)-elliptic
// problems, eq. (graddiv)) on the C ABI: find u in BDM1 on the unit square with
//
//   K int (u.v + div u div v) + gamma int_{dOmega} (u.nu)(v.nu) = <b, v>,
//
// by the domain-decomposition method of eq. (dd_preconditioner) in its Schur-complement form:
//   * the interior block A^00 = K(I - grad div) on V_0 (zero normal trace) is inverted by PCG
//     preconditioned with a V-cycle whose smoother is additive Schwarz over vertex patches (the
//     patches hold the curls of P2 functions, the kernel of div, so the cycle is uniform in h);
//   * Gamma is the whole boundary, the trace space the discontinuous P1 functions on its 4n
//     segments, and the Schur complement is preconditioned by S_Gamma = K L^{-1/2} + gamma I_Gamma
//     (the remark), realized by a rational table (eq. (RA)) of f(lam) / lam,
//     f = 1 / (K lam^{-1/2} + gamma): S_Gamma^{-1} ~ d0 M^{-1} L M^{-1} + (sum d) M^{-1}
//     - sum d_k q_k (L + q_k M)^{-1}, with L the interior-penalty -u'' + u on the loop;
//   * PCG on the trace (x_0 = 0, stop rule of Sec. 3), then the interior part by one more
//     interior solve.
// Every step runs in kernels (kernels_hdiv.hip); the host enqueues and reads stop flags back.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "api_internal.h"
#include "ell_mg.h"
#include "hdiv_internal.h"

using namespace fdd;

namespace {

constexpr double kTheta = 0.5;   // damping of the additive Schwarz smoother

EllHier hier(const ProblemHdiv* Q) {
  EllHier H;
  H.lev = Q->lev;
  H.nlev = Q->nlev;
  H.cinv = Q->dcinv;
  H.theta = Q->theta;
  H.n0 = Q->N0;
  H.r = Q->r;
  H.z = Q->z;
  H.p = Q->p;
  H.q = Q->q;
  H.partials = Q->partials;
  H.st = Q->st;
  H.hst = Q->hst;
  return H;
}

int read_hd(ProblemHdiv* Q, hipStream_t s) { return ell_read_state(hier(Q), s); }

// A^00 u = f (f in Q->f, u into Q->u) to ||f - A^00 u|| <= inner_rtol ||f||.  As many iterations
// as the last interior solve took are enqueued ahead of the read-back.
int inner(ProblemHdiv* Q, hipStream_t s, const fdd_opts& o, int* its) {
  return ell_pcg(hier(Q), s, o.mg_nu, o.inner_rtol, o.inner_maxit, Q->f, Q->u, &Q->its_hint, its,
                 "H(div) interior solve");
}

HdTable table_of(const fdd_ratpc_s* T) {
  HdTable t{};
  t.m = T->r.m;
  t.d0 = T->r.c0;
  double s = 0.0;
  for (int k = 0; k < t.m; ++k) {
    t.d[k] = T->r.c[k];
    t.q[k] = T->r.p[k];
    s += t.d[k];
  }
  t.dsum = s;
  return t;
}

// y = S p = A_GG p + A_G0 u with u = (A^00)^{-1} (-A_0G p)
int schur_product(ProblemHdiv* Q, hipStream_t s, const fdd_opts& o, const double* p, double* y,
                  int* its) {
  launch_hd_spmv(s, view(Q->A0G), p, Q->f, -1.0, 0.0, nullptr);
  int rc = inner(Q, s, o, its);
  if (rc) return rc;
  launch_hd_spmv(s, view(Q->AGG), p, y, 1.0, 0.0, nullptr);
  launch_hd_spmv(s, view(Q->AG0), Q->u, y, 1.0, 1.0, nullptr);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int clear_state(ProblemHdiv* Q, hipStream_t s) {
  HIPCHK(hipMemsetAsync(Q->st, 0, sizeof(HdState), s));
  return FDD_OK;
}

}  // namespace

namespace fdd {

size_t hdiv_workspace_bytes(fdd_problem_s* P) { return hdiv_plan(P->ph, nullptr); }

int hdiv_bind(fdd_problem_s* P, void* dev, size_t bytes, hipStream_t s) {
  ProblemHdiv* Q = P->ph;
  const size_t need = hdiv_plan(Q, nullptr);
  if (bytes < need) return fail(FDD_E_WORKSPACE, "workspace %zu bytes < %zu needed", bytes, need);
  HIPCHK(hipSetDevice(P->device));
  P->ws = (char*)dev;
  P->ws_bytes = bytes;
  hdiv_plan(Q, (char*)dev);
  if (!Q->hst) HIPCHK(hipHostMalloc((void**)&Q->hst, sizeof(HdState), hipHostMallocDefault));
  HIPCHK(hipMemsetAsync(dev, 0, need, s));
  auto up = [&](void* dst, const void* src, size_t nb) -> int {
    if (nb) HIPCHK(hipMemcpyAsync(dst, src, nb, hipMemcpyHostToDevice, s));
    return FDD_OK;
  };
  auto upm = [&](const HdMat& M) -> int {
    int rc = M.toff.empty() ? up(M.dcol, M.col.data(), M.col.size() * sizeof(int))
                            : up(M.dtoff, M.toff.data(), M.toff.size() * sizeof(int));
    if (!rc) rc = up(M.drtype, M.rtype.data(), M.rtype.size() * sizeof(int));
    return rc ? rc : up(M.dtval, M.tval.data(), M.tval.size() * sizeof(double));
  };
  int rc = FDD_OK;
  for (int l = 0; l < Q->nlev && !rc; ++l) {
    const HdLevel& L = Q->lev[l];
    rc = upm(L.A);
    if (!rc && l + 1 < Q->nlev) rc = upm(L.P);
    if (!rc && l + 1 < Q->nlev) rc = upm(L.R);
    if (!rc) rc = up(L.dpatch, L.patch.data(), L.patch.size() * sizeof(int));
    if (!rc) rc = up(L.dptype, L.ptype.data(), L.ptype.size() * sizeof(int));
    if (!rc) rc = up(L.dslot, L.slot.data(), L.slot.size() * sizeof(int));
    if (!rc) rc = up(L.dpinv, L.pinv.data(), L.pinv.size() * sizeof(double));
  }
  if (!rc) rc = up(Q->dcinv, Q->cinv.data(), Q->cinv.size() * sizeof(double));
  if (!rc) rc = upm(Q->A0G);
  if (!rc) rc = upm(Q->AG0);
  if (!rc) rc = upm(Q->AGG);
  if (!rc) rc = upm(Q->Afull);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

void hdiv_destroy(fdd_problem_s* P) {
  if (!P->ph) return;
  if (P->ph->hst) (void)hipHostFree(P->ph->hst);
  delete P->ph;
  P->ph = nullptr;
}

int hdiv_interior_solve(fdd_problem_s* P, const double* f, double* u, const fdd_opts& o,
                        hipStream_t s, int* its) {
  ProblemHdiv* Q = P->ph;
  int rc = clear_state(Q, s);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(Q->f, f, sizeof(double) * Q->N0, hipMemcpyDeviceToDevice, s));
  int k = 0;
  rc = inner(Q, s, o, &k);
  if (its) *its = k;
  if (rc < 0) return rc;
  HIPCHK(hipMemcpyAsync(u, Q->u, sizeof(double) * Q->N0, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return rc;
}

int hdiv_precond_apply(fdd_problem_s* P, const fdd_ratpc_s* T, const double* r, double* z,
                       hipStream_t s) {
  ProblemHdiv* Q = P->ph;
  launch_hd_loop_precond(s, Q->n, Q->blk, table_of(T), r, z, Q->scratch);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int hdiv_schur_apply(fdd_problem_s* P, const double* x, double* y, const fdd_opts& o,
                     hipStream_t s) {
  ProblemHdiv* Q = P->ph;
  int rc = clear_state(Q, s);
  if (rc) return rc;
  int its = 0;
  rc = schur_product(Q, s, o, x, y, &its);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(s));
  return FDD_OK;
}

int hdiv_apply_operator(fdd_problem_s* P, const double* x, double* y, hipStream_t s) {
  launch_hd_spmv(s, view(P->ph->Afull), x, y, 1.0, 0.0, nullptr);
  HIPCHK(hipGetLastError());
  return FDD_OK;
}

int hdiv_solve(fdd_problem_s* P, const fdd_ratpc_s* PT, const double* bv, double* x,
               const fdd_opts& o, hipStream_t s, fdd_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  ProblemHdiv* Q = P->ph;
  fdd_stats st;
  std::memset(&st, 0, sizeof(st));
  st.true_rel_res = -1.0;
  const int N0 = Q->N0, NG = Q->NG;
  const HdTable tP = table_of(PT);
  const double rtol2 = o.outer_rtol * o.outer_rtol;
  auto finish = [&](int code) {
    st.status = code;
    st.t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = st;
    return code;
  };
  auto solve_inner = [&](int* k) {
    int rc = inner(Q, s, o, k);
    st.inner_solves += 1;
    st.inner_its_total += *k;
    st.inner_its_max = std::max(st.inner_its_max, *k);
    return rc;
  };
  int rc = clear_state(Q, s);
  if (rc) return finish(rc);
  // g = b_G - A_G0 (A^00)^{-1} b_0; x_G = 0
  HIPCHK(hipMemcpyAsync(Q->f, bv, sizeof(double) * N0, hipMemcpyDeviceToDevice, s));
  int k = 0;
  if ((rc = solve_inner(&k))) return finish(rc);
  HIPCHK(hipMemcpyAsync(Q->rG, bv + N0, sizeof(double) * NG, hipMemcpyDeviceToDevice, s));
  launch_hd_spmv(s, view(Q->AG0), Q->u, Q->rG, -1.0, 1.0, nullptr);
  HIPCHK(hipMemsetAsync(Q->xG, 0, sizeof(double) * NG, s));
  launch_hd_loop_precond(s, Q->n, Q->blk, tP, Q->rG, Q->zG, Q->scratch);
  launch_hd_outer_direction(s, NG, Q->rG, Q->zG, Q->pG, Q->st, 1, rtol2);
  HIPCHK(hipGetLastError());
  int its = 0;
  for (;;) {
    if ((rc = read_hd(Q, s))) return finish(rc);
    if (Q->hst->o_done || its >= o.outer_maxit) break;
    if ((rc = schur_product(Q, s, o, Q->pG, Q->yG, &k))) return finish(rc);
    st.inner_solves += 1;
    st.inner_its_total += k;
    st.inner_its_max = std::max(st.inner_its_max, k);
    launch_hd_outer_alpha(s, NG, Q->pG, Q->yG, Q->st);
    launch_hd_outer_update(s, NG, Q->pG, Q->yG, Q->xG, Q->rG, Q->st);
    launch_hd_loop_precond(s, Q->n, Q->blk, tP, Q->rG, Q->zG, Q->scratch);
    launch_hd_outer_direction(s, NG, Q->rG, Q->zG, Q->pG, Q->st, 0, rtol2);
    HIPCHK(hipGetLastError());
    ++its;
  }
  const HdState h = *Q->hst;
  st.outer_its = its;
  if (h.breakdown & 6)
    return finish(fail(h.breakdown & 4 ? FDD_E_NONFINITE : FDD_E_BREAKDOWN,
                       "H(div) outer PCG breakdown at iteration %d (flags %d)", its, h.breakdown));
  st.rel_precond_res = h.o_rz0 > 0 ? std::sqrt(std::max(h.o_rz, 0.0) / h.o_rz0) : 0.0;
  // x_0 = (A^00)^{-1} (b_0 - A_0G x_G)
  HIPCHK(hipMemcpyAsync(Q->f, bv, sizeof(double) * N0, hipMemcpyDeviceToDevice, s));
  launch_hd_spmv(s, view(Q->A0G), Q->xG, Q->f, -1.0, 1.0, nullptr);
  if ((rc = solve_inner(&k))) return finish(rc);
  HIPCHK(hipMemcpyAsync(x, Q->u, sizeof(double) * N0, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(x + N0, Q->xG, sizeof(double) * NG, hipMemcpyDeviceToDevice, s));
  if (o.check_true_residual) launch_hd_true_residual(s, view(Q->Afull), bv, x, Q->partials, Q->st);
  HIPCHK(hipGetLastError());
  if ((rc = read_hd(Q, s))) return finish(rc);
  if (o.check_true_residual && Q->hst->t_res[1] > 0)
    st.true_rel_res = std::sqrt(Q->hst->t_res[0] / Q->hst->t_res[1]);
  return finish(h.o_done ? FDD_OK : FDD_NOT_CONVERGED);
}

}  // namespace fdd

extern "C" {

int fdd_setup_hdiv(int n, double K, double gamma, int hip_device, fdd_problem* out) {
  if (!out) return fail(FDD_E_ARG, "null argument");
  *out = nullptr;
  if (n < 4 || n > kHdMaxN || (n & (n - 1)))
    return fail(FDD_E_ARG, "H(div) problem: n must be a power of two, 4 <= n <= %d (got %d)",
                kHdMaxN, n);
  if (!(K > 0) || !std::isfinite(K) || !(gamma >= 0) || !std::isfinite(gamma))
    return fail(FDD_E_ARG, "H(div) problem: K > 0 and gamma >= 0 must be finite");
  fdd_problem_s* P = new (std::nothrow) fdd_problem_s();
  if (!P) return fail(FDD_E_NOMEM, "out of host memory");
  P->ph = new (std::nothrow) ProblemHdiv();
  if (!P->ph) {
    delete P;
    return fail(FDD_E_NOMEM, "out of host memory");
  }
  P->ph->theta = kTheta;
  if (const char* err = hdiv_build(P->ph, n, K, gamma)) {
    delete P->ph;
    delete P;
    return fail(FDD_E_ARG, "H(div) problem set-up: %s", err);
  }
  P->dim = 2;
  P->kind = kProblemHdiv;
  P->n = n;
  P->device = hip_device;
  P->K = K;
  P->gamma = gamma;
  P->mu = gamma > 0 ? 1.0 / gamma : INFINITY;
  P->h = 1.0 / n;
  // the preconditioner's table approximates f(lam) / lam = 1 / (K lam^{1/2} + gamma lam^1)
  P->tpow = 1.0;
  P->N = P->ph->N;
  P->NI = P->ph->N0;
  P->NG = P->ph->NG;
  P->eig = hdiv_loop_eigs(P->ph);
  P->lam_lo = P->eig.front();
  P->lam_hi = P->eig.back();
  *out = P;
  return FDD_OK;
}

}  // extern "C"
